// sp2_internal.h -- device-side loop state, workspace layout and helpers shared by
// the gfx950 kernels and the host driver of libsp2.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sp2.h"

namespace sp2 {

constexpr int kThreads = 256;        // every kernel uses 4 wave64s per workgroup
constexpr int kBndTile = 64;         // tile edge of the bounds / init / finalize kernels
constexpr int kMaxPersistent = 1024; // upper bound on the stream-K grid

// Loop state, resident in the workspace.  Written by one workgroup per kernel
// (a step's steering kernel, or the last-arriving block of a kernel that
// reduces by arrival); read by every kernel at start (kernel boundaries order
// it).
struct State {
    double emin, emax;
    double tr;          // trace of the current iterate X_m
    double fro2;        // ||X_m||_F^2
    double idem;        // e of the last step
    double tol;
    double nocc;
    int32_t n, max_iter;
    int32_t grow;       // 1 when the next step takes 2X - X^2
    int32_t done;
    int32_t status;
    int32_t iterations; // squarings done; X_m lives in buffer (m & 1)
    int32_t special;    // 1: n_occ == 0 -> D = 0; 2: n_occ == n -> D = I
    int32_t bad;        // a non-finite entry was seen in H
    uint32_t ticket;    // arrival counter of the kernels that reduce by arrival
    int32_t fp64_steps; // trace-steered FP64 steps (phase 0)
    // mixed precision: phase 0 = FP64 prefix, 1 = split-operand steps,
    // 2 = FP64 refinement (alternating x^2 / 2x - x^2)
    int32_t phase;
    int32_t m0;         // FP64 steps before the split phase (0: FP64 only)
    int32_t lp_start;   // first split-phase step
    int32_t lp_steps;
    int32_t refine_steps;
    int32_t max_refine;
    int32_t stale;      // 1: the newest iterate lives only in the split planes
    int32_t pad0;
    double lp_switch;   // leave the split phase once e <= lp_switch
    // learned expansion: phase 3 = trained layers, phase 4 = the SP2 check
    // step after them
    int32_t n_layers;
    int32_t pad1;
    double idem_fallback;  // the check step's idempotency bar
    // steering by a chemical potential instead of the occupation: the branch
    // follows mu's image x_mu under the maps applied so far (graph parts)
    int32_t mu_mode;
    int32_t pad2;
    double mu;
    double xmu;
    // learned expansion: restart from X_0 inside the plan after a rejected
    // check (restart_step: the step that reads the kept copy of X_0; -1 none)
    int32_t restart_step;
    int32_t restarted;
    double tr0;         // trace of X_0
    // thresholded SP2: K slices multiplied and output tiles computed, summed
    // over the steps of the solve
    unsigned long long sp_slices;
    unsigned long long sp_tiles;
    uint64_t branch_mask[2];
    uint64_t lp_mask[2];  // bit m set when step m was a split-operand step
    double tr_hist[SP2_MAX_ITER];
    double e_hist[SP2_MAX_ITER];
};

// Workspace layout (byte offsets from the 256-byte aligned base).
struct Layout {
    int n, ldp, bt;          // padded edge, FP64 SYRK tile edge
    int tiles;               // lower tiles of the FP64 SYRK grid
    int max_groups;          // stream-K grid bound: min(tiles, kMaxPersistent)
    int lp_groups;           // grid bound of the split-operand kernel (0: FP64 only)
    int np;                  // split-operand planes per iterate (0: FP64 only)
    int pb;                  // bytes per plane element
    size_t plane_stride;     // elements between planes of one iterate (ldp^2)
    size_t off_state, off_part, off_rowpart, off_cnt, off_scratch, off_x0, off_x1;
    size_t off_p0, off_p1, total;
};

constexpr int kLpTile = 128;  // tile edge of the split-operand kernels
constexpr int kFixRows = 8;   // S rows per workgroup of a step's finishing kernel (k_step_finish)

inline int planes_of(sp2_compute c) {
    return c == SP2_C_F16X2 ? 2 : c == SP2_C_BF16X3 ? 3 : c == SP2_C_BF16X2 ? 2 : c == SP2_C_FP8 ? 2 : 0;
}

// bytes per plane element (FP8 planes are one byte)
inline int plane_elem_bytes(sp2_compute c) { return c == SP2_C_FP8 ? 1 : 2; }

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// SYRK tile edge for an n x n problem.
inline int syrk_tile(int n) { return n <= 2048 ? 64 : 128; }

inline Layout make_layout(int n, sp2_compute compute) {
    Layout L{};
    L.n = n;
    L.bt = syrk_tile(n);
    L.np = planes_of(compute);
    L.pb = plane_elem_bytes(compute);
    L.ldp = (int)align_up((size_t)n, (size_t)(L.np ? kLpTile : L.bt));
    L.plane_stride = (size_t)L.ldp * L.ldp;
    int T = L.ldp / L.bt;
    L.tiles = T * (T + 1) / 2;
    int nb = L.ldp / kBndTile;
    const int nbt = L.ldp / kBndTile;   // 64-row tiles of the bounds / X_0 kernels
    // the 128-tile FP64 kernel runs up to kMaxPersistent workgroups whatever
    // the tile count (its stream-K remainder spreads a few tiles over many)
    L.max_groups = (L.bt == 128 || L.tiles > kMaxPersistent) ? kMaxPersistent : L.tiles;
    // per-tile sums: the whole tiles, plus one entry per kFixRows-row block of
    // each split tile of a 128-tile step (fewer split tiles than workgroups)
    const int Tl128 = L.ldp / kLpTile;
    const int tiles128 = Tl128 * (Tl128 + 1) / 2;
    size_t part_entries = (size_t)(L.tiles > tiles128 ? L.tiles : tiles128) +
                          (size_t)(kLpTile / kFixRows - 1) * kMaxPersistent;
    part_entries *= 4;
    size_t init_entries = (size_t)nb * nb * 4;
    if (init_entries > part_entries) part_entries = init_entries;
    size_t off = 0;
    L.off_state = off;   off = align_up(off + sizeof(State), 256);
    L.off_part = off;    off = align_up(off + part_entries * sizeof(double), 256);
    L.off_rowpart = off; off = align_up(off + ((size_t)nbt * L.ldp + 2 * (size_t)L.ldp) * sizeof(double), 256);
    size_t scratch_f64 = 2 * (size_t)(L.max_groups + 1) * L.bt * L.bt * sizeof(double);
    int Tl = L.ldp / kLpTile;
    // split-operand grid: one workgroup per 128-tile for n <= 2048, the full
    // persistent grid above (the FP64 scratch is already that large there)
    int lp_groups = Tl * (Tl + 1) / 2 < kMaxPersistent ? Tl * (Tl + 1) / 2 : kMaxPersistent;
    if (L.bt == 128) lp_groups = kMaxPersistent;
    L.lp_groups = L.np ? lp_groups : 0;
    size_t scratch_lp = L.np ? 2 * (size_t)(lp_groups + 1) * kLpTile * kLpTile * sizeof(double) : 0;
    if (L.np && lp_groups > L.max_groups) L.max_groups = lp_groups;
    L.off_cnt = off;     off = align_up(off + (size_t)(L.max_groups + 2) * sizeof(unsigned), 256);
    L.off_scratch = off; off = align_up(off + (scratch_f64 > scratch_lp ? scratch_f64 : scratch_lp), 256);
    L.off_x0 = off;      off = align_up(off + (size_t)L.ldp * L.ldp * sizeof(double), 256);
    L.off_x1 = off;      off = align_up(off + (size_t)L.ldp * L.ldp * sizeof(double), 256);
    L.off_p0 = off;      off = align_up(off + (size_t)L.np * L.plane_stride * L.pb, 256);
    L.off_p1 = off;      off = align_up(off + (size_t)L.np * L.plane_stride * L.pb, 256);
    L.total = off;
    return L;
}

// ---------------------------------------------------------------- device helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_min(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Sum of v over the 256 threads in a fixed order (wave sums, then waves 0..3).
// `scratch` holds at least 4 doubles of LDS.  Result valid in every thread.
__device__ inline double block_sum(double v, double* scratch) {
    v = wave_sum(v);
    int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double r = ((scratch[0] + scratch[1]) + scratch[2]) + scratch[3];
    __syncthreads();
    return r;
}

// Called by every thread after this block's partial results are stored.
// Returns true in every thread of the single block that arrives last; that
// block then sees all other blocks' partials.
__device__ inline bool arrive_last(State* st, unsigned nblocks, int* flag_lds) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(&st->ticket, 1u);
        *flag_lds = (t == nblocks - 1);
    }
    __syncthreads();
    bool last = *flag_lds != 0;
    if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return last;
}

// ---------------------------------------------------------------- host side

// The solve behind sp2_density (and its no-allocation variant); see sp2_api.hip.
int density_impl(const void* H, void* D, int n, int ld, int n_occ, double tol, int max_iter,
                 sp2_dtype dtype, sp2_compute compute, int fp64_prefix_iters, void* workspace,
                 size_t workspace_bytes, void* hip_stream, sp2_info* info, bool no_alloc);

// Pinned status buffers and events of one in-flight call.  Calls take a set
// from a per-device free list and give it back when they return, so the sets
// made equal the largest number of concurrent calls on a device, whatever
// the number of threads that ever called; they are reused for the life of
// the process (the pool is never destroyed, so no HIP call runs during
// static destruction).
struct HostSlots {
    int* flags = nullptr;     // 2 pinned ints
    State* state = nullptr;   // pinned copy of the device state
    hipEvent_t ev[2] = {nullptr, nullptr};
};

// Holds one set for the duration of a call.
struct SlotLease {
    HostSlots* s = nullptr;
    int dev = -1;
    hipStream_t pending = nullptr;   // a copy into the set may still be queued here
    bool has_pending = false;
    ~SlotLease();
};

// Takes a set of the current device's pool (made on first use).
hipError_t slots_for_current(SlotLease& lease);

// The batched plan behind sp2_plan_create and the learned expansion (sp2_batch.hip).
int plan_create_impl(sp2_plan** plan, int batch, const int* n, const int* n_occ, sp2_dtype dtype,
                     sp2_compute compute, double tol, int max_iter, const char* autotune_cache,
                     const double* coef, int n_layers, double idem_fallback, int mu_mode);
int plan_run_impl(sp2_plan* p, const void* const* H, void* const* D, const double* mu, void* hip_stream,
                  sp2_info* infos);

// ---------------------------------------------------------------- host launchers

hipError_t launch_reset(State* st, int n, int n_occ, double tol, int max_iter, int m0,
                        unsigned* cnt, int ncnt, hipStream_t s);
hipError_t launch_bounds(const void* H, sp2_dtype dt, int n, int ld, const Layout& L, State* st,
                         double* rowpart, double* part, hipStream_t s);
hipError_t launch_init(const void* H, sp2_dtype dt, int n, int ld, const Layout& L, State* st,
                       double* x0, double* part, hipStream_t s);
hipError_t launch_syrk_f64(const Layout& L, const double* X, double* Y, State* st, double* part,
                           double* scratch, unsigned* cnt, int step, hipStream_t s);
hipError_t launch_syrk_lp(const Layout& L, sp2_compute mode, const void* Pin, void* Pout,
                          double* X, State* st, double* part, double* scratch, int step, hipStream_t s);
// Workgroups of the step kernels (0 for the self-steering 64-tile FP64 step).
hipError_t lp_step_groups(const Layout& L, sp2_compute mode, int* G);
hipError_t f64_step_groups(const Layout& L, int* G);
// End of step `step`, after the step kernels: the split tiles of whichever
// 128-tile step ran (FP64 X -> Y, or planes Pin -> Pout), then the steering.
hipError_t launch_step_end(const Layout& L, sp2_compute mode, const void* Pin, void* Pout, const double* X,
                           double* Y, State* st, double* part, const double* scratch, int step,
                           hipStream_t s);
hipError_t launch_f64_to_planes(const Layout& L, sp2_compute mode, const double* X, void* Pout,
                                const State* st, int step, hipStream_t s);
hipError_t launch_finalize(void* D, sp2_dtype dt, int n, int ld, const Layout& L, sp2_compute mode,
                           const State* st, const double* x0, const double* x1, const void* p0,
                           const void* p1, hipStream_t s);

}  // namespace sp2
