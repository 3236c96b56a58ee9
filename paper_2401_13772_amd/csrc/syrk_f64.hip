// syrk_f64.hip -- one SP2 step in FP64 on the gfx950 matrix cores:
//   S = X X^T (= X^2, X symmetric), the product the paper's SP2 loop spends
//   its time in (Section "SP2 solver": the cost is dominated by the matrix
//   multiplications of the recursion), fused with the step itself:
//     e^2  += (S - X)^2        idempotency of X_m, for the stop test
//     X'    = S or 2X - S      the branch chosen by tr X_m vs n_occ
//     tr   += X'_ii, ||X'||^2  for the next branch decision
//   and the steering of the next step, taken on the device by the last block.
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
//   * per-tile sums go to a partial buffer that the last-arriving workgroup
//     adds in tile order: deterministic, no floating-point atomics.
#include "sp2_device.h"

namespace sp2 {

constexpr int kBK = 16;
constexpr int kLDK = kBK + 1;

template <int BT_, int WM_, int WN_>
struct SyrkCfg {
    static constexpr int BT = BT_, WM = WM_, WN = WN_;
    static constexpr int NT = 64 * WM * WN;          // threads per workgroup
    static constexpr int NW = WM * WN;               // waves per workgroup
    static constexpr int WTM = BT / WM, WTN = BT / WN;
    static constexpr int MI = WTM / 16, NI = WTN / 16;
    static constexpr int LOADS = BT * kBK / 2 / NT;  // double2 chunks per thread per panel
    static constexpr size_t LDS = (size_t)2 * 2 * BT * kLDK * sizeof(double);
    static_assert(LOADS >= 1 && (BT * kBK / 2) % NT == 0, "panel slice must split evenly");
};

using CfgSmall = SyrkCfg<64, 2, 2>;    // 256 threads, 32 x 32 per wave
using CfgLarge = SyrkCfg<128, 2, 4>;   // 512 threads, 64 x 32 per wave

// Accumulate the C tile over K slices [kt0, kt1) of the row panels of tiles
// ti and tj.  DIAG: ti == tj, both operands come from one panel.
template <class C, bool DIAG>
__device__ __forceinline__ void syrk_mainloop(const double* __restrict__ X, int ldp, int ti, int tj,
                                              int kt0, int kt1, double* sA, double* sB,
                                              d4 (&acc)[C::MI][C::NI]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const double* Ap = X + (size_t)ti * C::BT * ldp;
    const double* Bp = X + (size_t)tj * C::BT * ldp;
    int goff[C::LOADS], soff[C::LOADS];
#pragma unroll
    for (int i = 0; i < C::LOADS; ++i) {
        const int c = tid + C::NT * i;
        const int row = c >> 3, kk = (c & 7) * 2;
        goff[i] = row * ldp + kk;
        soff[i] = row * kLDK + kk;
    }
    d2 ra[C::LOADS], rb[C::LOADS];
#pragma unroll
    for (int i = 0; i < C::LOADS; ++i) {
        ra[i] = *(const d2*)(Ap + goff[i] + kt0 * kBK);
        if (!DIAG) rb[i] = *(const d2*)(Bp + goff[i] + kt0 * kBK);
    }
#pragma unroll
    for (int i = 0; i < C::LOADS; ++i) {
        sA[soff[i]] = ra[i].x;
        sA[soff[i] + 1] = ra[i].y;
        if (!DIAG) {
            sB[soff[i]] = rb[i].x;
            sB[soff[i] + 1] = rb[i].y;
        }
    }
    __syncthreads();
    const int arow = (wm * C::WTM + (lane & 15)) * kLDK + (lane >> 4);
    const int brow = (wn * C::WTN + (lane & 15)) * kLDK + (lane >> 4);
    for (int kt = kt0; kt < kt1; ++kt) {
        const int stg = (kt - kt0) & 1;
        const bool more = kt + 1 < kt1;
        if (more) {
#pragma unroll
            for (int i = 0; i < C::LOADS; ++i) {
                ra[i] = *(const d2*)(Ap + goff[i] + (kt + 1) * kBK);
                if (!DIAG) rb[i] = *(const d2*)(Bp + goff[i] + (kt + 1) * kBK);
            }
        }
        const double* a = sA + stg * C::BT * kLDK;
        const double* b = DIAG ? a : (sB + stg * C::BT * kLDK);
#pragma unroll
        for (int s = 0; s < kBK / 4; ++s) {
            double af[C::MI], bf[C::NI];
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi) af[mi] = a[arow + mi * 16 * kLDK + 4 * s];
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) bf[ni] = b[brow + ni * 16 * kLDK + 4 * s];
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
        }
        if (more) {
            double* na = sA + (stg ^ 1) * C::BT * kLDK;
            double* nb = sB + (stg ^ 1) * C::BT * kLDK;
#pragma unroll
            for (int i = 0; i < C::LOADS; ++i) {
                na[soff[i]] = ra[i].x;
                na[soff[i] + 1] = ra[i].y;
                if (!DIAG) {
                    nb[soff[i]] = rb[i].x;
                    nb[soff[i] + 1] = rb[i].y;
                }
            }
        }
        __syncthreads();
    }
}

// The SP2 update of one finished C tile, and this thread's share of the
// tile's e^2, trace and ||X'||^2.
// Accumulator layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l
// holds column l%16 of the 16x16 block at rows l/16 + 4r, r = 0..3.  For a
// fixed r the 64 lanes cover 4 rows x 16 consecutive columns, so the direct
// reads and writes are 128-byte row segments.
template <class C>
__device__ __forceinline__ void sp2_epilogue(const double* __restrict__ X, double* __restrict__ Y,
                                             int ldp, int ti, int tj, int grow,
                                             const d4 (&acc)[C::MI][C::NI], double& e2,
                                             double& trp, double& fro) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const bool diag = (ti == tj);
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi) {
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) {
            const int gi0 = ti * C::BT + wm * C::WTM + mi * 16 + (lane >> 4);
            const int gj = tj * C::BT + wn * C::WTN + ni * 16 + (lane & 15);
            double xv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) xv[r] = X[(size_t)(gi0 + 4 * r) * ldp + gj];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = gi0 + 4 * r;
                const double s = acc[mi][ni][r];
                const double x = xv[r];
                const double d = s - x;
                const double xn = grow ? (2.0 * x - s) : s;
                const double wgt = (gi > gj) ? 2.0 : ((gi == gj) ? 1.0 : 0.0);
                e2 += wgt * (d * d);
                fro += wgt * (xn * xn);
                if (gi == gj) trp += xn;
                // lower copy; the upper copy mirrors it (diagonal tiles: lower half wins)
                if (!diag || gi >= gj) Y[(size_t)gi * ldp + gj] = xn;
                if (!diag || gi > gj) Y[(size_t)gj * ldp + gi] = xn;
            }
        }
    }
}

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
            __threadfence();
            __syncthreads();
            if (tid == 0) flag = (int)atomicAdd(&cnt[bidx], 1u);
            __syncthreads();
            if (flag == 0) continue;             // the other segment will finish the tile
            __threadfence();
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
    if (!group_arrive_last(&st->ticket, G, &flag)) return;
    double E = 0.0, TR = 0.0, F = 0.0;
    for (unsigned k = tid; k < ntiles; k += C::NT) {
        E += part[4 * k + 0];
        TR += part[4 * k + 1];
        F += part[4 * k + 2];
    }
    E = group_sum<C::NW>(E, red);
    TR = group_sum<C::NW>(TR, red);
    F = group_sum<C::NW>(F, red);
    if (tid == 0) sp2_steer_thread0(st, E, TR, F, grow);
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
    return launch_cfg<CfgLarge>(L, X, Y, st, part, scratch, cnt, step, s);
}

}  // namespace sp2
