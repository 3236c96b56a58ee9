// sp2_sparse.hip -- SP2 with the drop threshold tau of the SP2 listing (its
// multiply and add take a cutoff; the sparse solvers of Section "Leveraging
// third-party libraries" prune the entries below it), run on dense storage
// with 128 x 128 tile skipping: entries with |x| < tau are dropped after the
// product and after the 2X - X^2 update, and a tile of the product is only
// computed over the K tiles where both operand tiles hold a nonzero.  For a
// spatially local H the iterates stay banded around the diagonal (in a
// Morton-ordered basis), so most of the O(n^3) products are skipped.
//
// Per iterate buffer a T x T byte map says which 128-tiles hold a nonzero
// (symmetric, as the iterates are).  A step launches one workgroup per lower
// tile (I, J):
//   * the K tiles with flag(I, K) and flag(J, K) are gathered into runs of
//     consecutive tiles, and the LDS-DMA FP64 MFMA main loop of the dense step
//     runs over each run;
//   * the thresholded update is applied in the LDS-staged epilogue of the
//     dense step (S' = drop(S), X' = drop(2X - S') or S'), which also reports
//     whether X' has a nonzero (the new flag);
//   * a tile with no product and a zero X tile is X' = 0: it is only written
//     (as zeros) when the output buffer's tile held a nonzero;
//   * per-tile sums go to fixed slots; k_sparse_steer, launched after the
//     step, adds them in tile order and steers (sp2_steer_thread0), so the
//     step needs no arrival fence (an L2 write-back on every XCD, paid by
//     each of its workgroups).
#include <cmath>

#include "syrk_f64_core.h"

namespace sp2 {

using SpCfg = SyrkCfg<128, 2, 2>;     // the 128-tile FP64 step's shape
constexpr int kSpMaxT = 512;          // n <= 65536
constexpr int kSpSlices = 128 / kBK;  // K slices per tile
constexpr int kSpGroupM = 8;          // row panels per raster group

// Flags of X_0 (any nonzero in the tile) and of the other buffer (all set:
// its content is unknown until the first step writes every tile).
__global__ __launch_bounds__(256) void k_sparse_flags0(const double* __restrict__ X0, int ldp, int T,
                                                       unsigned char* __restrict__ f0,
                                                       unsigned char* __restrict__ f1) {
    __shared__ int any;
    int ti, tj;
    tri_tile(blockIdx.x, ti, tj);
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int mine = 0;
    for (int e = threadIdx.x; e < 128 * 32; e += 256) {
        const int r = e >> 5, c4 = (e & 31) * 4;
        const d4 v = *(const d4*)(X0 + (size_t)(ti * 128 + r) * ldp + tj * 128 + c4);
        mine |= (v[0] != 0.0) | (v[1] != 0.0) | (v[2] != 0.0) | (v[3] != 0.0);
    }
    if (mine) any = 1;
    __syncthreads();
    if (threadIdx.x == 0) {
        f0[ti * T + tj] = (unsigned char)any;
        f0[tj * T + ti] = (unsigned char)any;
        f1[ti * T + tj] = 1;
        f1[tj * T + ti] = 1;
    }
}

template <class C>
__global__ __launch_bounds__(C::NT, 2) void k_sparse_step(const double* __restrict__ X, double* __restrict__ Y,
                                                       int ldp, int T, State* st, double* __restrict__ part,
                                                       const unsigned char* __restrict__ fin,
                                                       unsigned char* __restrict__ fout, double tau,
                                                       int step) {
    extern __shared__ __attribute__((aligned(16))) char lsm[];
    __shared__ double red[C::NW];
    __shared__ int s_nz;
    __shared__ unsigned char act[kSpMaxT];
    if (st->done || st->iterations != step) return;
    const int grow = st->grow;
    const int tid = threadIdx.x;
    const unsigned t = xcd_remap(blockIdx.x, gridDim.x);
    int ti, tj;
    grouped_tile(t, T, kSpGroupM, ti, tj);
    // the K tiles where both operand tiles hold a nonzero
    for (int K = tid; K < T; K += C::NT) act[K] = fin[ti * T + K] & fin[tj * T + K];
    if (tid == 0) s_nz = 0;
    __syncthreads();
    d4 acc[C::MI][C::NI];
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    bool any = false;
    int slices = 0;
    int K = 0;
    while (K < T) {
        if (!act[K]) {
            ++K;
            continue;
        }
        int K1 = K + 1;
        while (K1 < T && act[K1]) ++K1;
        // one main-loop instance (a diagonal tile loads its panel twice): the
        // second instance of the dense step costs more registers than it saves
        syrk_mainloop_dma<C, false>(X, ldp, ti, tj, K * kSpSlices, K1 * kSpSlices, lsm, acc);
        any = true;
        slices += (K1 - K) * kSpSlices;
        K = K1;
    }
    const bool xnz = fin[ti * T + tj] != 0;
    double e2 = 0.0, trp = 0.0, fro = 0.0;
    if (!any && !xnz) {
        // S = 0 and X = 0 on this tile: X' = 0
        if (fout[ti * T + tj]) {
            for (int e = tid; e < 128 * 32; e += C::NT) {
                const int r = e >> 5, c4 = (e & 31) * 4;
                *(d4*)(Y + (size_t)(ti * 128 + r) * ldp + tj * 128 + c4) = d4{0.0, 0.0, 0.0, 0.0};
                if (ti != tj) *(d4*)(Y + (size_t)(tj * 128 + r) * ldp + ti * 128 + c4) = d4{0.0, 0.0, 0.0, 0.0};
            }
        }
    } else {
        int nz = 0;
        sp2_epilogue_lds<C, true>(X, Y, ldp, ti, tj, grow, acc, (double*)lsm, e2, trp, fro, tau, &nz);
        if (nz) s_nz = 1;
    }
    e2 = group_sum<C::NW>(e2, red);
    trp = group_sum<C::NW>(trp, red);
    fro = group_sum<C::NW>(fro, red);
    if (tid == 0) {
        const unsigned char f = (unsigned char)(s_nz != 0);
        fout[ti * T + tj] = f;
        fout[tj * T + ti] = f;
        part[4 * t + 0] = e2;
        part[4 * t + 1] = trp;
        part[4 * t + 2] = fro;
        if (slices) atomicAdd(&st->sp_slices, (unsigned long long)slices);
        if (any || xnz) atomicAdd(&st->sp_tiles, 1ull);
    }
}

// The steering of step `step`: the step's tile sums in tile order.  One
// workgroup.
template <class C>
__global__ __launch_bounds__(C::NT) void k_sparse_steer(State* st, const double* __restrict__ part, int T,
                                                        int step) {
    __shared__ double red[C::NW];
    if (st->done || st->iterations != step) return;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const int tid = threadIdx.x;
    double E = 0.0, TR = 0.0, F = 0.0;
    for (unsigned k = tid; k < ntiles; k += C::NT) {
        E += part[4 * k + 0];
        TR += part[4 * k + 1];
        F += part[4 * k + 2];
    }
    E = group_sum<C::NW>(E, red);
    TR = group_sum<C::NW>(TR, red);
    F = group_sum<C::NW>(F, red);
    if (tid == 0) sp2_steer_thread0(st, E, TR, F, st->grow);
}

// Workspace: state | pair/tile partials | row partials | flags x 2 | X0 | X1.
struct SparseLayout {
    int ldp, T, tiles;
    size_t off_state, off_part, off_rowpart, off_flags, off_x0, off_x1, total;
};

inline SparseLayout sparse_layout(int n) {
    SparseLayout L{};
    L.ldp = (int)align_up((size_t)n, (size_t)128);
    L.T = L.ldp / 128;
    L.tiles = L.T * (L.T + 1) / 2;
    const int nb = L.ldp / kBndTile;
    size_t part_entries = (size_t)L.tiles * 4;
    if ((size_t)nb * nb * 4 > part_entries) part_entries = (size_t)nb * nb * 4;
    size_t off = 0;
    L.off_state = off;   off = align_up(off + sizeof(State), 256);
    L.off_part = off;    off = align_up(off + part_entries * sizeof(double), 256);
    L.off_rowpart = off; off = align_up(off + ((size_t)nb * L.ldp + 2 * (size_t)L.ldp) * sizeof(double), 256);
    L.off_flags = off;   off = align_up(off + 2 * (size_t)L.T * L.T, 256);
    L.off_x0 = off;      off = align_up(off + (size_t)L.ldp * L.ldp * sizeof(double), 256);
    L.off_x1 = off;      off = align_up(off + (size_t)L.ldp * L.ldp * sizeof(double), 256);
    L.total = off;
    return L;
}

}  // namespace sp2

extern "C" {

size_t sp2_sparse_workspace_size(int n) {
    if (n <= 0 || n > 65536) return 0;
    return sp2::sparse_layout(n).total;
}

int sp2_density_sparse(const void* H, void* D, int n, int ld, int n_occ, double tol, int max_iter,
                       sp2_dtype dtype, double tau, void* workspace, size_t workspace_bytes, void* hip_stream,
                       sp2_info* info) {
    using namespace sp2;
    auto fail = [&](int code) {
        if (info) {
            *info = sp2_info{};
            info->status = code;
        }
        return code;
    };
    if (info) *info = sp2_info{};
    if (!H || !D || n <= 0 || n > 65536 || ld < n || n_occ < 0 || n_occ > n) return fail(SP2_E_INVALID);
    if (!(tol > 0.0) || !(tol < 1e300) || max_iter < 0 || max_iter > SP2_MAX_ITER) return fail(SP2_E_INVALID);
    if (dtype != SP2_F64 && dtype != SP2_F32) return fail(SP2_E_INVALID);
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(SP2_E_INVALID);
    const SparseLayout SL = sparse_layout(n);
    if (!workspace || workspace_bytes < SL.total ||
        (reinterpret_cast<uintptr_t>(workspace) % SP2_WORKSPACE_ALIGN) != 0)
        return fail(SP2_E_WORKSPACE);
    const size_t esz = dtype == SP2_F64 ? sizeof(double) : sizeof(float);
    const size_t mbytes = ((size_t)(n - 1) * ld + n) * esz;
    const char* hp = (const char*)H;
    const char* dp = (const char*)D;
    const char* wp = (const char*)workspace;
    if ((hp < dp + mbytes && dp < hp + mbytes) || (dp < wp + SL.total && wp < dp + mbytes))
        return fail(SP2_E_INVALID);

    hipStream_t s = (hipStream_t)hip_stream;
    char* ws = (char*)workspace;
    State* st = (State*)(ws + SL.off_state);
    double* part = (double*)(ws + SL.off_part);
    double* rowpart = (double*)(ws + SL.off_rowpart);
    unsigned char* flags[2] = {(unsigned char*)(ws + SL.off_flags),
                               (unsigned char*)(ws + SL.off_flags) + (size_t)SL.T * SL.T};
    double* xb[2] = {(double*)(ws + SL.off_x0), (double*)(ws + SL.off_x1)};
    Layout L{};   // what the bounds, X_0 and copy-out launchers read
    L.n = n;
    L.ldp = SL.ldp;
    L.bt = 128;
    L.plane_stride = (size_t)SL.ldp * SL.ldp;

    SlotLease lease;
#define SP2_SP_HIP(call)                                   \
    do {                                                   \
        if ((call) != hipSuccess) return fail(SP2_E_HIP); \
    } while (0)
    SP2_SP_HIP(slots_for_current(lease));
    HostSlots* hs = lease.s;
    using C = SpCfg;
    constexpr size_t lds = DmaLayout<C>::LDS > LdsEpi<C>::LDS ? DmaLayout<C>::LDS : LdsEpi<C>::LDS;
    static bool attr_set = false;
    if (!attr_set) {
        SP2_SP_HIP(hipFuncSetAttribute((const void*)k_sparse_step<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
        attr_set = true;
    }
    SP2_SP_HIP(launch_reset(st, n, n_occ, tol, max_iter, 0, nullptr, 0, s));
    SP2_SP_HIP(launch_bounds(H, dtype, n, ld, L, st, rowpart, part, s));
    SP2_SP_HIP(launch_init(H, dtype, n, ld, L, st, xb[0], part, s));
    hipLaunchKernelGGL(k_sparse_flags0, dim3(SL.tiles), dim3(256), 0, s, xb[0], SL.ldp, SL.T, flags[0], flags[1]);
    SP2_SP_HIP(hipGetLastError());

    const int chunk = SL.ldp >= 2048 ? 4 : 8;
    int issued = 0, pending = -1, slot = 0;
    bool stop = false;
    while (issued < max_iter && !stop) {
        const int c = (max_iter - issued) < chunk ? (max_iter - issued) : chunk;
        for (int i = 0; i < c; ++i, ++issued) {
            const int odd = issued & 1;
            hipLaunchKernelGGL(k_sparse_step<C>, dim3(SL.tiles), dim3(C::NT), lds, s, xb[odd], xb[odd ^ 1], SL.ldp,
                               SL.T, st, part, flags[odd], flags[odd ^ 1], tau, issued);
            hipLaunchKernelGGL(k_sparse_steer<C>, dim3(1), dim3(C::NT), 0, s, st, part, SL.T, issued);
            SP2_SP_HIP(hipGetLastError());
        }
        lease.pending = s;
        lease.has_pending = true;
        SP2_SP_HIP(hipMemcpyAsync(&hs->flags[slot], &st->done, sizeof(int), hipMemcpyDeviceToHost, s));
        SP2_SP_HIP(hipEventRecord(hs->ev[slot], s));
        if (pending >= 0) {
            SP2_SP_HIP(hipEventSynchronize(hs->ev[pending]));
            if (hs->flags[pending]) stop = true;
        }
        pending = slot;
        slot ^= 1;
    }
    SP2_SP_HIP(launch_finalize(D, dtype, n, ld, L, SP2_C_F64, st, xb[0], xb[1], nullptr, nullptr, s));
    SP2_SP_HIP(hipMemcpyAsync(hs->state, st, sizeof(State), hipMemcpyDeviceToHost, s));
    SP2_SP_HIP(hipStreamSynchronize(s));
    lease.has_pending = false;
#undef SP2_SP_HIP
    const State& h = *hs->state;
    if (info) {
        info->status = h.status;
        info->iterations = h.iterations;
        info->fp64_prefix_iters = h.fp64_steps;
        info->refine_steps = h.refine_steps;
        info->trace = h.tr;
        info->trace_error = std::fabs(h.tr - (double)n_occ);
        info->idempotency = h.idem;
        info->emin = h.emin;
        info->emax = h.emax;
        info->branch_mask[0] = h.branch_mask[0];
        info->branch_mask[1] = h.branch_mask[1];
    }
    return h.status;
}

int sp2_sparse_stats(const void* workspace, void* hip_stream, double* executed_flops, double* tile_steps) {
    using namespace sp2;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % SP2_WORKSPACE_ALIGN) != 0) return SP2_E_INVALID;
    SlotLease lease;
    if (slots_for_current(lease) != hipSuccess) return SP2_E_HIP;
    hipStream_t s = (hipStream_t)hip_stream;
    lease.pending = s;
    lease.has_pending = true;
    if (hipMemcpyAsync(lease.s->state, workspace, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SP2_E_HIP;
    lease.has_pending = false;
    const State& h = *lease.s->state;
    // one K slice of a 128 x 128 tile: 128 * 128 * 16 multiply-adds
    if (executed_flops) *executed_flops = 2.0 * 128.0 * 128.0 * kBK * (double)h.sp_slices;
    if (tile_steps) *tile_steps = (double)h.sp_tiles;
    return SP2_OK;
}

}  // extern "C"
