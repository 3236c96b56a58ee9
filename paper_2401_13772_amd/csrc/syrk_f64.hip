// syrk_f64.hip -- one SP2 step in FP64 on the gfx950 matrix cores:
//   S = X X^T (= X^2, X symmetric), the product the paper's SP2 loop spends
//   its time in (Section "SP2 solver": the cost is dominated by the matrix
//   multiplications of the recursion), fused with the step itself:
//     e^2  += (S - X)^2        idempotency of X_m, for the stop test
//     X'    = S or 2X - S      the branch chosen by tr X_m vs n_occ
//     tr   += X'_ii, ||X'||^2  for the next branch decision
//   and the steering of the next step, taken on the device by k_step_steer
//   (step_end.hip), launched after the step.
//
// Design for CDNA4:
//   * only the lower block-triangle of BT x BT tiles is computed (X X^T is
//     symmetric); each off-diagonal tile is written twice (direct and
//     mirrored), so the next step reads whole row panels of a fully stored
//     symmetric matrix;
//   * v_mfma_f64_16x16x4_f64; WM x WN wave64s per workgroup, each wave owning
//     a (BT/WM) x (BT/WN) sub-tile of 16 x 16 accumulators;
//   * row panels are staged in LDS in double-buffered BK = 16 slices (rows
//     padded to 17 doubles so the 16 rows one fragment read touches fall into
//     distinct banks), one barrier per slice, the next slice's global loads
//     in flight under the current slice's MFMAs;
//   * diagonal tiles read one panel only;
//   * stream-K scheduling: a persistent grid of G workgroups (as many as are
//     co-resident, at most the tile count) splits the (tile, K-slice) work
//     into G equal contiguous ranges.  A tile cut by a range boundary is
//     finished by whichever of its two workgroups arrives second, which adds
//     the two partial sums in the fixed order seg0 + seg1 (no waiting, and
//     the result does not depend on arrival order).  This removes the idle
//     tail of a one-tile-per-workgroup grid (528 tiles on 256 CUs is 2.06
//     waves of work in 3 waves of time);
//   * workgroups are renumbered so each XCD (blocks are dealt round-robin to
//     the 8 XCDs) works on a contiguous run of tiles, which share row panels
//     in that XCD's L2;
//   * per-tile sums go to a partial buffer that k_step_steer adds in tile
//     order after the kernel: deterministic, no floating-point atomics, and
//     no arrival fence (an L2 write-back on every XCD) in the step kernel.
#include "sk_finish.h"

namespace sp2 {

// Stream-K SYRK + SP2 step.  grid = G persistent workgroups (G <= ntiles).
// scratch: 2 (G + 1) C-tile partials; cnt: G + 1 arrival counters, zero on
// entry and left zero on exit.  `step` is the index of the step this launch
// performs; it does nothing unless the loop state says that step is due and
// in an FP64 phase (the trace-steered prefix or the refinement).
template <class C>
__global__ __launch_bounds__(C::NT) void k_syrk_f64(const double* __restrict__ X,
                                                    double* __restrict__ Y, int ldp, int T,
                                                    State* st, double* __restrict__ part,
                                                    double* __restrict__ scratch,
                                                    unsigned* __restrict__ cnt, int step) {
    extern __shared__ double smem[];
    __shared__ double red[C::NW];
    __shared__ int flag;

    if (st->done || st->iterations != step || st->phase == 1) return;
    const int grow = st->grow;
    const unsigned G = gridDim.x;
    const unsigned g = xcd_remap(blockIdx.x, G);
    const int KT = ldp / kBK;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const uint64_t U = (uint64_t)ntiles * KT;
    const uint64_t u0 = U * g / G, u1 = U * (g + 1) / G;
    double* sA = smem;
    double* sB = smem + 2 * C::BT * kLDK;
    const int tid = threadIdx.x;

    uint64_t u = u0;
    while (u < u1) {
        const unsigned t = (unsigned)(u / KT);
        const int k0 = (int)(u % KT);
        const uint64_t kend = (uint64_t)k0 + (u1 - u);
        const int k1 = kend < (uint64_t)KT ? (int)kend : KT;
        int ti, tj;
        tri_tile(t, ti, tj);
        d4 acc[C::MI][C::NI];
#pragma unroll
        for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
        if (ti == tj) syrk_mainloop<C, true>(X, ldp, ti, tj, k0, k1, sA, sB, acc);
        else syrk_mainloop<C, false>(X, ldp, ti, tj, k0, k1, sA, sB, acc);
        u += (uint64_t)(k1 - k0);

        if (!(k0 == 0 && k1 == KT)) {
            // a split tile: seg 0 = [0, kb) ends at this group's range end
            // (boundary g + 1); seg 1 = [kb, KT) starts at its range start
            // (boundary g).
            const int seg = (k0 == 0) ? 0 : 1;
            const unsigned bidx = (seg == 0) ? g + 1 : g;
            const size_t tile_elems = (size_t)C::BT * C::BT;
            d4* mine = (d4*)(scratch + (2 * (size_t)bidx + seg) * tile_elems);
            const d4* other = (const d4*)(scratch + (2 * (size_t)bidx + (1 - seg)) * tile_elems);
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni) mine[(mi * C::NI + ni) * C::NT + tid] = acc[mi][ni];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __syncthreads();
            if (tid == 0) flag = (int)atomicAdd(&cnt[bidx], 1u);
            __syncthreads();
            if (flag == 0) continue;             // the other segment will finish the tile
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni) {
                    const d4 o = other[(mi * C::NI + ni) * C::NT + tid];
                    acc[mi][ni] = (seg == 0) ? (acc[mi][ni] + o) : (o + acc[mi][ni]);
                }
            if (tid == 0) cnt[bidx] = 0u;
        }

        double e2 = 0.0, trp = 0.0, fro = 0.0;
        sp2_epilogue<C>(X, Y, ldp, ti, tj, grow, acc, e2, trp, fro);
        e2 = group_sum<C::NW>(e2, red);
        trp = group_sum<C::NW>(trp, red);
        fro = group_sum<C::NW>(fro, red);
        if (tid == 0) {
            part[4 * t + 0] = e2;
            part[4 * t + 1] = trp;
            part[4 * t + 2] = fro;
        }
    }
}

// ---------------------------------------------------------------- 128-tile kernel
// Data-parallel waves plus a stream-K remainder.  With G co-resident
// workgroups and N lower tiles, the first floor(N/G) * G tiles (grouped
// raster order) go out in whole waves: every workgroup starts its tile at
// K = 0 at the same time, so the workgroups of one XCD (a contiguous run of
// the order) stream the same row and column panels through its L2 together.
// The R = N mod G tiles left over are split evenly over all G workgroups as
// contiguous ranges of K slices (a range is shorter than a tile, so it touches
// at most two tiles).  Each segment of a split tile is stored as an FP64
// partial in slot 2g (the workgroup's first tile) or 2g + 1 (its second).
// The kernels launched after it (k_step_finish, k_step_steer) add a split
// tile's partials in workgroup order (the sum does not depend on which segment
// finished last), run the split tiles' epilogue and take the steering
// decision: this kernel needs no fence or counter between its workgroups.
// Even XCDs run the remainder before their waves, odd XCDs after, so the
// tile epilogues of the two halves (HBM-bound bursts) do not coincide.
constexpr int kGroupM = 8;

template <class C>
__global__ __launch_bounds__(C::NT) void k_syrk_f64_hyb(const double* __restrict__ X, double* __restrict__ Y,
                                                        int ldp, int T, State* st, double* __restrict__ part,
                                                        double* __restrict__ scratch, int step) {
    extern __shared__ __attribute__((aligned(16))) char lsm[];
    __shared__ double red[C::NW];

    if (st->done || st->iterations != step || st->phase == 1) return;
    const int grow = st->grow;
    const unsigned G = gridDim.x;
    const unsigned g = xcd_remap(blockIdx.x, G);
    const int KT = ldp / kBK;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const unsigned waves = ntiles / G;
    const unsigned Dt = waves * G;
    const unsigned R = ntiles - Dt;
    const int tid = threadIdx.x;

    auto finish = [&](unsigned t, int ti, int tj, d4 (&acc)[C::MI][C::NI]) {
        double e2 = 0.0, trp = 0.0, fro = 0.0;
        sp2_epilogue_lds<C>(X, Y, ldp, ti, tj, grow, acc, (double*)lsm, e2, trp, fro);
        e2 = group_sum<C::NW>(e2, red);
        trp = group_sum<C::NW>(trp, red);
        fro = group_sum<C::NW>(fro, red);
        if (tid == 0) {
            part[4 * t + 0] = e2;
            part[4 * t + 1] = trp;
            part[4 * t + 2] = fro;
        }
    };

    // stream-K remainder (the split of SkSplit): each segment of a split tile
    // leaves its FP64 partial tile, row-major, in slot 2g (the range's first
    // tile) or 2g + 1; k_step_finish adds them after this kernel.  R < G <= 1024
    // and KT <= 4096 keep every product below 2^32 (32-bit range arithmetic).
    auto remainder = [&]() {
        if (R > 0) {
            const SkSplit sk(R, (unsigned)KT, G);
            // remainder owners by hardware block index: blocks are dealt round-robin
            // to the XCDs, so the owners spread over all of them
            const unsigned gr = blockIdx.x;
            unsigned u, u1;
            sk.range(gr, u, u1);
            int seg_no = 0;
            const int lane = tid & 63, w = tid >> 6;
            const int wm = w / C::WN, wn = w % C::WN;
            while (u < u1) {
                const unsigned r = u / (unsigned)KT;
                const int k0 = (int)(u - r * (unsigned)KT);
                const unsigned kend = (unsigned)k0 + (u1 - u);
                const int k1 = kend < (unsigned)KT ? (int)kend : KT;
                int ti, tj;
                grouped_tile(Dt + r, T, kGroupM, ti, tj);
                d4 acc[C::MI][C::NI];
#pragma unroll
                for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                    for (int ni = 0; ni < C::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
                if (ti == tj) syrk_mainloop_dma<C, true>(X, ldp, ti, tj, k0, k1, lsm, acc);
                else syrk_mainloop_dma<C, false>(X, ldp, ti, tj, k0, k1, lsm, acc);
                u += (unsigned)(k1 - k0);
                double* mine = scratch + (2 * (size_t)gr + seg_no++) * (size_t)C::BT * C::BT;
                // accumulator (mi, ni, r) of a lane: row 16 mi + lane / 16 + 4 r of
                // the wave's sub-tile, column 16 ni + lane % 16
#pragma unroll
                for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                    for (int ni = 0; ni < C::NI; ++ni)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int row = wm * C::WTM + mi * 16 + (lane >> 4) + 4 * q;
                            const int col = wn * C::WTN + ni * 16 + (lane & 15);
                            mine[row * C::BT + col] = acc[mi][ni][q];
                        }
            }
        }
    };
    auto waves_part = [&]() {
        // data-parallel waves
        for (unsigned w = 0; w < waves; ++w) {
            const unsigned t = w * G + g;
            int ti, tj;
            grouped_tile(t, T, kGroupM, ti, tj);
            d4 acc[C::MI][C::NI];
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
            if (ti == tj) syrk_mainloop_dma<C, true>(X, ldp, ti, tj, 0, KT, lsm, acc);
            else syrk_mainloop_dma<C, false>(X, ldp, ti, tj, 0, KT, lsm, acc);
            finish(t, ti, tj, acc);
        }
    };
    // Blocks are dealt round-robin to the 8 XCDs, so a block's index parity is
    // its XCD's: even XCDs run their remainder share before their waves, odd
    // XCDs after.  The two halves' tile epilogues (HBM-bound bursts of X reads
    // and X' writes) then come at different times instead of all at once.
    const bool remainder_first = (blockIdx.x & 1) == 0;
    for (int half = 0; half < 2; ++half) {
        if ((half == 0) == remainder_first) remainder();
        else waves_part();
    }
}

using CfgHyb = SyrkCfg<128, 2, 2>;   // 256 threads, 64 x 64 per wave, LDS-DMA operands

// Workgroups of the 128-tile step: as many as are co-resident, at most
// L.max_groups (the workspace holds 2 G partial tiles).
static hipError_t hyb_groups(const Layout& L, int* G) {
    using C = CfgHyb;
    constexpr size_t lds = DmaLayout<C>::LDS > LdsEpi<C>::LDS ? DmaLayout<C>::LDS : LdsEpi<C>::LDS;
    static int per_cu = -1;
    static int cus = 0;
    if (per_cu < 0) {
        hipError_t e = hipFuncSetAttribute((const void*)k_syrk_f64_hyb<C>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        int dev = 0, nb = 0;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_syrk_f64_hyb<C>, C::NT, lds);
        if (e != hipSuccess) return e;
        per_cu = nb < 1 ? 1 : nb;
    }
    int g = per_cu * cus;
    if (g > L.max_groups) g = L.max_groups;
    *G = g < 1 ? 1 : g;
    return hipSuccess;
}

static hipError_t launch_hyb(const Layout& L, const double* X, double* Y, State* st, double* part,
                             double* scratch, int step, hipStream_t s) {
    using C = CfgHyb;
    constexpr size_t lds = DmaLayout<C>::LDS > LdsEpi<C>::LDS ? DmaLayout<C>::LDS : LdsEpi<C>::LDS;
    int G = 0;
    hipError_t e = hyb_groups(L, &G);
    if (e != hipSuccess) return e;
    const int T = L.ldp / C::BT;
    hipLaunchKernelGGL(k_syrk_f64_hyb<C>, dim3(G), dim3(C::NT), lds, s, X, Y, L.ldp, T, st, part, scratch, step);
    return hipGetLastError();
}

template <class C>
static hipError_t launch_cfg(const Layout& L, const double* X, double* Y, State* st, double* part,
                             double* scratch, unsigned* cnt, int step, hipStream_t s) {
    static int per_cu = -1;
    static int cus = 0;
    if (per_cu < 0) {
        hipError_t e = hipFuncSetAttribute((const void*)k_syrk_f64<C>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
        if (e != hipSuccess) return e;
        int dev = 0, nb = 0;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_syrk_f64<C>, C::NT, C::LDS);
        if (e != hipSuccess) return e;
        per_cu = nb < 1 ? 1 : nb;
    }
    const int T = L.ldp / C::BT;
    const int ntiles = T * (T + 1) / 2;
    int G = per_cu * cus;
    if (G > kMaxPersistent) G = kMaxPersistent;
    if (G > ntiles) G = ntiles;
    if (G < 1) G = 1;
    hipLaunchKernelGGL(k_syrk_f64<C>, dim3(G), dim3(C::NT), C::LDS, s, X, Y, L.ldp, T, st, part,
                       scratch, cnt, step);
    return hipGetLastError();
}

hipError_t launch_syrk_f64(const Layout& L, const double* X, double* Y, State* st, double* part,
                           double* scratch, unsigned* cnt, int step, hipStream_t s) {
    if (L.bt == CfgSmall::BT) return launch_cfg<CfgSmall>(L, X, Y, st, part, scratch, cnt, step, s);
    return launch_hyb(L, X, Y, st, part, scratch, step, s);
}

hipError_t f64_step_groups(const Layout& L, int* G) {
    if (L.bt == CfgSmall::BT) {   // the 64-tile kernel: no remainder for the step end to finish
        *G = 0;
        return hipSuccess;
    }
    return hyb_groups(L, G);
}

}  // namespace sp2
