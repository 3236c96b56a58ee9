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
    SP2_C_FP8 = 5     /* mixed, as F16X2 with two OCP e4m3 planes x ~ 2^-8 q0 +
                         2^-12 q1 (fixed power-of-two scales: SP2 iterates
                         satisfy |x| <= 1), 3 products on the FP8 MFMA */
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
 *                    and FP32 accumulation (traces and norms in FP64) until,
 *                    from a value below 0.1, the idempotency no longer drops
 *                    tenfold over two steps (the rounding floor);
 *                 3. FP64 refinement steps alternating X^2 and 2X - X^2
 *                    (not steered by the trace) until e <= tol, at most 8.
 *               info->fp64_prefix_iters and info->refine_steps report 1 and 3.
 *   fp64_prefix_iters  steps of phase 1 for the split modes: -1 = automatic
 *               (F16X2: 8, BF16X3: 6, others 8; two more for n > 4096,
 *               calibrated on MI355X to keep rms |D - D_ref| <= 7e-7 for gaps
 *               >= 0.3 eV on a ~140 eV spectral interval), otherwise
 *               1..SP2_MAX_ITER; ignored for SP2_C_F64.
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
 * sp2_density without any allocation, for callers that cannot allocate
 * device or pinned host memory (code that must not call hipMalloc, tight
 * serving loops, harnesses that forbid allocation).  Same arguments, result
 * and kernels as sp2_density, but the workspace is a fixed device array of
 * SP2_NOALLOC_MAX_BYTES bytes inside the library (one per GPU, held until the
 * process ends), so sp2_workspace_size(n, dtype, compute) must not exceed it
 * (n <= 1024 for every compute mode); larger problems return
 * SP2_E_WORKSPACE with D untouched.  The call makes no hipMalloc, hipFree,
 * hipHostMalloc or event creation: all max_iter steps are queued (steps
 * after the stop return at once) and the loop state is copied back once into
 * pageable host memory at the end.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU race, so the caller serialises them.
 * sp2_history does not apply (the workspace is not the caller's).
 */
#define SP2_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int sp2_density_noalloc(const void* H, void* D, int n, int ld, int n_occ, double tol, int max_iter,
                        sp2_dtype dtype, sp2_compute compute, int fp64_prefix_iters,
                        void* hip_stream, sp2_info* info);

/*
 * Batched plan (many independent solves in one graph replay).  The paper's
 * graph-partitioned workflow (Section "Graph-based Divide electronic
 * structure") solves one small dense SP2 problem per part, independently;
 * a plan runs a fixed set of such problems together.
 *
 * sp2_plan_create: batch problems of sizes n[b] (1 <= n[b] <= SP2_PLAN_MAX_N)
 *   and occupations n_occ[b], storage dtype, compute (SP2_C_F64; other modes
 *   return SP2_E_UNSUPPORTED), stop tolerance and max_iter as in sp2_density.
 *   Allocates the plan's device memory (iterates, loop states, work lists),
 *   picks the squaring kernel's tile shape and captures the whole solve
 *   (bounds, X_0, max_iter steps, copy to D, info) into one HIP graph on the
 *   current device.  autotune_cache: NULL = the single-matrix kernels' tile
 *   shape (each D is then bitwise equal to its sp2_density result); a file
 *   path = time the candidate shapes on this size mix once and keep the
 *   fastest, reading/appending the choice in that text file.  Returns
 *   SP2_OK and *plan, or a negative status with *plan = NULL.
 * sp2_plan_run: H[b], D[b] are device pointers to n[b] x n[b] row-major
 *   matrices (leading dimension n[b]) in the caller's order; D[b] must not
 *   overlap H[b].  Copies the pointers to the device, replays the graph on
 *   hip_stream and returns after the per-matrix infos (host array of batch
 *   records, may be NULL) are back.  Returns the most negative per-matrix
 *   status if any is negative, else the largest.  Runs of one plan must not
 *   overlap; the plan is bound to the device it was created on.
 * sp2_plan_config: name of the chosen tile shape (static storage).
 * sp2_plan_destroy: frees everything the plan owns.
 */
typedef struct sp2_plan sp2_plan;
#define SP2_PLAN_MAX_BATCH 65536
#define SP2_PLAN_MAX_N 2048
int sp2_plan_create(sp2_plan** plan, int batch, const int* n, const int* n_occ, sp2_dtype dtype,
                    sp2_compute compute, double tol, int max_iter, const char* autotune_cache);
int sp2_plan_run(sp2_plan* plan, const void* const* H, void* const* D, void* hip_stream,
                 sp2_info* infos);
const char* sp2_plan_config(const sp2_plan* plan);
int sp2_plan_destroy(sp2_plan* plan);

/*
 * Thresholded SP2 with tile skipping.  The SP2 listing (Section "SP2 solver")
 * passes a cutoff tau to its multiply and add; the sparse solvers of Section
 * "Leveraging third-party libraries" prune the entries below it.  Here:
 * X2 = drop(X X) and X <- drop(2X - X2) or X2, where drop zeroes every entry
 * with |x| < tau; X_0 is formed whole; e_m = ||X2 - X_m||_F; steering, stop
 * rule and special cases as sp2_density (FP64 throughout).  Dropping puts a
 * floor of about tau under e, so a solve with tol below it ends by the
 * stagnation rule (SP2_E_STAGNATED, D is the last iterate).  Storage is
 * dense; a 128 x 128 tile of a product is computed only over the K tiles
 * where both operand tiles hold a nonzero, and an all-zero tile of the
 * iterate is skipped, so a spatially local H (sorted so that near orbitals
 * have near indices) costs far fewer than n^3 operations per step.
 *   H, D, n, ld, n_occ, tol, max_iter, dtype, hip_stream, info: as
 *               sp2_density; n <= 65536.
 *   tau         drop threshold, >= 0 (0: plain FP64 SP2 with tile skipping).
 *   workspace   at least sp2_sparse_workspace_size(n) bytes, aligned to
 *               SP2_WORKSPACE_ALIGN: the loop state, partial sums, two tile
 *               maps and two FP64 iterates padded to a multiple of 128.
 *               sp2_history reads the trace and e histories from it.
 */
size_t sp2_sparse_workspace_size(int n);
/* After a solve on this workspace (and after the stream has reached it):
 * the multiply-add work the tile skipping left, as flops (2 per multiply-add,
 * the lower tiles only), and the number of (step, lower tile) pairs computed. */
int sp2_sparse_stats(const void* workspace, void* hip_stream, double* executed_flops, double* tile_steps);
int sp2_density_sparse(const void* H, void* D, int n, int ld, int n_occ, double tol, int max_iter,
                       sp2_dtype dtype, double tau, void* workspace, size_t workspace_bytes,
                       void* hip_stream, sp2_info* info);

/*
 * Graph-partitioned solver (Section "Graph-based Divide electronic
 * structure": the adjacency equation, core and core-halo partitions, the
 * extraction of sub-matrices and the map-back of the general solver routine
 * listing).  The graph of an auxiliary matrix G (H itself, an overlap matrix
 * or an earlier density matrix) joins nodes l != o with |G_lo| >= tau.  Core
 * part k is the k-th of `parts` regular segments of the index list,
 * [floor(k n / parts), floor((k + 1) n / parts)); its core-halo part adds
 * every node o with |G_lo| >= tau for a core node l (row l of G).  A solve
 * takes the dense sub-matrix of H on each core-halo part (nodes in
 * ascending order), solves all of them as one batched plan at a common
 * chemical potential mu, and writes row l of D, for each core node l, from
 * its part: the part's row spread over the part's nodes, 0 in every other
 * column.  Each part's SP2 steps are steered by mu instead of an occupation:
 * with x_mu = (emax - mu)/(emax - emin) the image of mu under X_0 (the
 * part's Gershgorin bounds), a step takes X^2 when x_mu > 1/2 and 2X - X^2
 * otherwise, and x_mu follows the same map; eigenvalues below mu go to 1 and
 * those above to 0, so each part converges to the projector on its
 * eigenvalues below mu (the zero-temperature Fermi-Dirac function of Section
 * "Single-particle density matrix").  mu at or below emin gives 0, at or
 * above emax the identity, with no step.  Stop rule as in sp2_density,
 * except that the stagnation test compares e_m with e_{m-3} and waits for
 * e < 1e-3 (mu's image takes at most two equal branches in a row, during
 * which levels on one side may move away from 0 or 1).
 *
 * sp2_graph_create: G is a device pointer, n x n row-major with leading
 *   dimension ld, storage dtype; 1 <= n <= 65536, 1 <= parts <= min(n, 4096),
 *   tau >= 0.  Builds the parts on the current device (reads G once, one host
 *   synchronisation on hip_stream), allocates the parts' buffers and
 *   captures the batched plan (tol, max_iter as in sp2_density).  A part with
 *   more than SP2_PLAN_MAX_N nodes returns SP2_E_UNSUPPORTED.
 * sp2_graph_parts: writes the node count and the core node count of every
 *   part (host arrays of `parts` ints, each may be NULL); returns parts.
 * sp2_graph_nodes: copies part `part`'s ascending node list into a host
 *   array of capacity ints; returns the part's size (nothing is copied when
 *   nodes is NULL or capacity is short).
 * sp2_graph_density: H, D device pointers, n x n, leading dimension ld,
 *   storage dtype, no overlap.  Returns after D is written; infos (host
 *   array of `parts` records, may be NULL) gets each part's solve record
 *   (trace = the part's occupation, trace_error 0).  Returns the most
 *   negative per-part status if any is negative (D is then unspecified),
 *   else the largest.  Calls on one graph must not overlap.
 * sp2_graph_destroy: frees the graph and its plan.
 */
typedef struct sp2_graph sp2_graph;
int sp2_graph_create(sp2_graph** graph, const void* G, int n, int ld, sp2_dtype dtype, double tau,
                     int parts, double tol, int max_iter, void* hip_stream);
int sp2_graph_parts(const sp2_graph* graph, int* sizes, int* core_sizes);
int sp2_graph_nodes(const sp2_graph* graph, int part, int* nodes, int capacity);
int sp2_graph_density(sp2_graph* graph, const void* H, void* D, int ld, sp2_dtype dtype, double mu,
                      void* hip_stream, sp2_info* infos);
int sp2_graph_destroy(sp2_graph* graph);

/*
 * Learned recursive expansion: a composition of trained quadratic maps of the
 * matrix, a deep-network form of the paper's recursive polynomial expansion
 * (Section "GPU friendly algorithms": the expansion is a product of layers,
 * each a low-order polynomial of the previous layer's output).  Layer k with
 * f_k(x) = a_k x^2 + b_k x + c_k maps X -> f_k(X) when tr X > n_occ and
 * X -> I - f_k(I - X) otherwise (trace steering as in SP2; (a, b, c) =
 * (1, 0, 0) is SP2).  Coefficients are FP32 values (held as double).
 *
 * sp2_learned_create: a model from n_layers x 3 host coefficients.
 * sp2_learned_fit: train n_layers layers on spectra, starting from SP2:
 *   spectra = the eigenvalues of n_samples Hamiltonians, each sorted
 *   ascending, concatenated (n[s] values each, n[s] <= 1024); gersh = emin,
 *   emax per sample (the Gershgorin bounds the solve will use); the target is
 *   the projector (1 on the n_occ[s] lowest levels).  Loss: mean over samples
 *   of log(mean squared eigenvalue error); Adam over `epochs` passes in
 *   minibatches of 512, order drawn from `seed`.  Runs on the current GPU
 *   (allocates its own buffers).  n_layers * max n[s] * 8 <= 150 KiB.
 * sp2_learned_coefficients: copies up to `capacity` coefficients (3 per
 *   layer) and the last epoch's loss; returns the layer count.
 * sp2_learned_save / sp2_learned_load: text file (hex floats, exact).
 * sp2_learned_density: batch matrices of one size n (device pointers,
 *   row-major, leading dimension n, storage dtype), occupations n_occ[b]:
 *   the trained layers, then an SP2 check step on their output X_L.  If
 *   ||X_L^2 - X_L||_F <= idem_fallback and the trace error is within
 *   idem_fallback, D is the check step's output (status SP2_OK).  Else, if
 *   ||X_L^2 - X_L||_F <= 0.3 (every eigenvalue within [-0.242, 1.242]), one
 *   step of the branch the check step did not take pulls the spectrum into
 *   [0, 1] without moving any eigenvalue across the middle, and plain
 *   trace-steered SP2 steps continue on the device with sp2_density's stop
 *   rule (tol 1e-10), up to 60 of them.  Else the matrix restarts plain FP64
 *   SP2 from its X_0 (kept by the plan) within the same run, and if that or
 *   the continuation does not converge it is solved again from H by
 *   sp2_density; both are reported as SP2_E_FALLBACK.  info.fp64_prefix_iters
 *   = the learned layers applied, info.refine_steps = the steps after the
 *   check step (the continuation's, or the plain SP2 solve's), info.iterations
 *   = all squarings.
 *   compute: SP2_C_F64 (others SP2_E_UNSUPPORTED).  The model keeps an
 *   inference plan for the last (batch, n, n_occ, dtype, bar) and a
 *   workspace for the fallback solves; calls on one model must not overlap.
 *   Returns the most negative per-matrix status if any, else the largest.
 * sp2_learned_destroy: frees the model and what it keeps.
 */
typedef struct sp2_learned sp2_learned;
int sp2_learned_create(sp2_learned** model, int n_layers, const double* coef);
int sp2_learned_fit(sp2_learned** model, int n_layers, const double* spectra, const int* n,
                    const int* n_occ, int n_samples, const double* gersh, int epochs, uint64_t seed);
int sp2_learned_coefficients(const sp2_learned* model, double* coef, int capacity, double* fit_loss);
int sp2_learned_save(const sp2_learned* model, const char* path);
int sp2_learned_load(sp2_learned** model, const char* path);
int sp2_learned_density(sp2_learned* model, int batch, int n, const void* const* H, void* const* D,
                        const int* n_occ, sp2_dtype dtype, sp2_compute compute, double idem_fallback,
                        void* hip_stream, sp2_info* infos);
int sp2_learned_destroy(sp2_learned* model);

/*
 * Chebyshev expansion of the Fermi operator (Section "Chebyshev polynomial
 * expansion"): D = sum_{t < k m} c_t T_t(Hs) with Hs = ((H + H^T)/2 - a I)/b,
 * a, b the centre and half width of the Gershgorin interval, and c_t the
 * Chebyshev coefficients (Chebyshev-Gauss rule, 4 k m nodes) of the
 * Fermi-Dirac occupation 1/(1 + exp(beta (e - mu))) (mu, beta in the units of
 * H).  For finite temperature or a vanishing gap, where SP2 is not suited.
 * Evaluated in the section's Paterson-Stockmeyer form sum_j T_k^j S_j,
 * S_j = sum_{i<k} d_{i,j} T_i: T_2..T_k level by level (each level one
 * grouped launch), then m - 1 Horner products; k + m - 2 matrix products in
 * all.  1 <= k <= 64, 1 <= m <= k + 4, n <= 32768.
 *   H, D        device pointers, n x n, row-major, leading dimension ld,
 *               storage dtype; D may be uninitialised.
 *   workspace   at least sp2_cheb_workspace_size(n, k) bytes (k + 2 padded
 *               FP64 matrices and work lists), SP2_WORKSPACE_ALIGN aligned.
 * One host synchronisation after the bounds (their values set the
 * coefficients), one at the end.  info: status, iterations = matrix
 * products, trace = tr D, emin/emax.  Returns SP2_OK or a negative status
 * (D untouched).
 */
size_t sp2_cheb_workspace_size(int n, int k);
int sp2_cheb_density(const void* H, void* D, int n, int ld, sp2_dtype dtype, double mu, double beta, int k,
                     int m, void* workspace, size_t workspace_bytes, void* hip_stream, sp2_info* info);

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
