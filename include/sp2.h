/*
 * sp2.h -- C ABI of libsp2.so: SP2 density-matrix purification on one AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (paper: Fattebert et al., arXiv 2401.13772):
 *   Given a symmetric n x n Hamiltonian H and an occupation n_occ, return the
 *   zero-temperature density matrix D, the projector onto the n_occ lowest
 *   eigenvectors of H (Section "Single-particle density matrix", Fermi-Dirac
 *   construction with the occupations 0 or 1 of an insulator).
 *   SP2 reaches it without eigenvectors (Section "SP2 solver"):
 *     X_0 = (emax I - H)/(emax - emin), with emin/emax Gershgorin bounds
 *       (Section "Distributed matrices" names the Gershgorin-circle method);
 *     X_{m+1} = X_m^2 if tr X_m > n_occ, else 2 X_m - X_m^2 (the listing's
 *       "tr - nel <= 0" sends the tie to 2X - X^2);
 *   until X is idempotent.
 *
 * Conventions of this library (where the paper is silent):
 *   - H is read through its symmetric part (H + H^T)/2.
 *   - e_m = ||X_m^2 - X_m||_F (FP64).  The loop stops after the update of
 *     step m when e_m <= tol (SP2_OK), or when m >= 2, e_m >= e_{m-2} and
 *     e_m < 0.1 (SP2_E_STAGNATED: the rounding floor was reached above tol),
 *     or after max_iter steps (SP2_E_NOT_CONVERGED).  `iterations` counts the
 *     squarings.  D receives the last iterate X_{m+1}.
 *   - n_occ == 0 gives D = 0, n_occ == n gives D = I, with no iteration.
 *
 * Memory: every matrix argument is a DEVICE pointer, row-major, leading
 * dimension `ld` elements (ld >= n).  Because H is symmetric, row-major and
 * column-major storage are the same matrix.  The caller owns H, D and the
 * workspace; the library never frees them and allocates no device memory in
 * these calls.  The only host allocation is a small pinned status buffer made
 * once per calling thread.  H is read only; D must not overlap H or the
 * workspace.
 *
 * Streams: every call is ordered on `hip_stream` (a hipStream_t; NULL = the
 * null stream) and returns after `info` has been copied back (one host
 * synchronisation at the end, plus a non-blocking poll of a "done" flag every
 * few steps).  Calls that share a workspace must not overlap.
 *
 * Errors: negative status = nothing computed and D untouched (for
 * SP2_E_DEGENERATE D is untouched unless n_occ is 0 or n); positive status =
 * D holds the last iterate and `info` says why the loop ended.  No C++
 * exception crosses this boundary.
 */
#ifndef SP2_H
#define SP2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* storage type of H and D */
typedef enum { SP2_F64 = 0, SP2_F32 = 1 } sp2_dtype;

/* arithmetic of the squarings (steering, traces and norms are always FP64) */
typedef enum {
    SP2_C_F64 = 0,    /* FP64 MFMA squarings */
    SP2_C_F32 = 1,    /* reserved */
    SP2_C_F16X2 = 2,  /* mixed: FP64 prefix, then X = h + l (two FP16 planes),
                         S = hh + hl + lh on FP16 MFMA with FP32 accumulation,
                         then FP64 refinement */
    SP2_C_BF16X3 = 3, /* mixed, as above with three BF16 planes (6 products) */
    SP2_C_BF16X2 = 4, /* mixed, as above with two BF16 planes (3 products) */
    SP2_C_FP8 = 5     /* reserved */
} sp2_compute;

typedef enum {
    SP2_OK = 0,
    SP2_E_NOT_CONVERGED = 1,
    SP2_E_STAGNATED = 2,
    SP2_E_FALLBACK = 3,
    SP2_E_INVALID = -1,     /* bad argument, or a non-finite entry in H */
    SP2_E_DEGENERATE = -2,  /* emax == emin with 0 < n_occ < n */
    SP2_E_WORKSPACE = -3,   /* workspace missing, too small or misaligned */
    SP2_E_HIP = -4,         /* a HIP runtime call failed */
    SP2_E_UNSUPPORTED = -5  /* a reserved compute mode that is not built */
} sp2_status;

#define SP2_MAX_ITER 128
#define SP2_WORKSPACE_ALIGN 256

/* Written to host memory when sp2_density returns. */
typedef struct {
    int32_t status;            /* an sp2_status value */
    int32_t iterations;        /* squarings performed */
    int32_t fp64_prefix_iters; /* squarings done in FP64 */
    int32_t refine_steps;      /* FP64 refinement squarings after a low-precision phase */
    double trace;              /* tr D (FP64) */
    double trace_error;        /* |tr D - n_occ| */
    double idempotency;        /* e_m = ||X_m^2 - X_m||_F of the last step (FP64) */
    double emin, emax;         /* Gershgorin bounds of (H + H^T)/2 */
    uint64_t branch_mask[2];   /* bit m set when step m used 2X - X^2 */
} sp2_info;

/* Library version (integer, major*100 + minor). */
int sp2_version(void);

/* Static string for a status code. */
const char* sp2_status_str(int status);

/*
 * Bytes of device workspace sp2_density needs for an n x n problem with the
 * given storage type and compute mode (0 for invalid arguments).  The
 * workspace holds two padded FP64 iterates (plus two sets of 16-bit planes for
 * the split modes), the per-tile partial sums, the stream-K fix-up tiles and
 * the device-side loop state.
 */
size_t sp2_workspace_size(int n, sp2_dtype dtype, sp2_compute compute);

/*
 * SP2 density matrix of H (paper: Section "SP2 solver", equations for D_0 and
 * D_{m+1} and the listing's branch rule; bounds from Section "Distributed
 * matrices").
 *   H, D        device pointers, n x n, row-major, leading dimension ld, of
 *               type `dtype` (FP64 or FP32); D may be uninitialised.
 *   n_occ       number of occupied states, 0 <= n_occ <= n.
 *   tol         stop when ||X_m^2 - X_m||_F <= tol (tol > 0).
 *   max_iter    at most this many squarings, 0 <= max_iter <= SP2_MAX_ITER.
 *   compute     arithmetic of the squarings.  SP2_C_F64: every step in FP64.
 *               The split modes (F16X2, BF16X3, BF16X2) run a mixed-precision
 *               schedule (not in the paper; its dense SP2 is FP64 throughout):
 *                 1. fp64_prefix_iters trace-steered FP64 steps, while the
 *                    gap around the Fermi level is still small in the mapped
 *                    spectrum and rounding errors would be amplified;
 *                 2. trace-steered steps with split-operand 16-bit products
 *                    and FP32 accumulation (traces and norms in FP64) until
 *                    the idempotency stops decreasing;
 *                 3. FP64 refinement steps alternating X^2 and 2X - X^2
 *                    (not steered by the trace) until e <= tol, at most 8.
 *               info->fp64_prefix_iters and info->refine_steps report 1 and 3.
 *   fp64_prefix_iters  steps of phase 1 for the split modes: -1 = automatic
 *               (12), otherwise 1..SP2_MAX_ITER; ignored for SP2_C_F64.
 *   workspace   device buffer of at least sp2_workspace_size(n, dtype,
 *               compute) bytes, aligned to SP2_WORKSPACE_ALIGN.
 *   hip_stream  hipStream_t or NULL.
 *   info        host pointer, filled on return (may be NULL).
 * Returns the status also stored in info->status.
 */
int sp2_density(const void* H, void* D, int n, int ld, int n_occ, double tol, int max_iter,
                sp2_dtype dtype, sp2_compute compute, int fp64_prefix_iters, void* workspace,
                size_t workspace_bytes, void* hip_stream, sp2_info* info);

/*
 * Copy the per-step history of the last sp2_density call that used
 * `workspace`: tr_hist[m] = tr X_m (before step m), e_hist[m] = e_m.
 * Copies min(count, iterations) entries into the host arrays (either may be
 * NULL) and returns that number, or a negative status.
 */
int sp2_history(const void* workspace, int count, double* tr_hist, double* e_hist,
                void* hip_stream);

/*
 * Kernel timing for measurement (not part of the method).  With
 * sp2_profile_enable(1), later sp2_density calls on this thread and device
 * record a HIP event pair around every squaring-kernel launch on the call's
 * stream; sp2_profile_read then returns the summed event time of the real
 * (not skipped) squarings of the last call and their number.  Host pointers;
 * either may be NULL.  Returns SP2_OK or SP2_E_HIP.
 */
int sp2_profile_enable(int on);
int sp2_profile_read(double* step_ms_total, int* steps);
/* The same, split into FP64 step kernels and split-operand step kernels. */
int sp2_profile_read_split(double* f64_ms, int* f64_steps, double* split_ms, int* split_steps);

#ifdef __cplusplus
}
#endif

#endif /* SP2_H */
