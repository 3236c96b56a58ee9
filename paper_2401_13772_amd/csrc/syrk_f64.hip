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
//   * only the lower block-triangle of tiles is computed (X X^T is symmetric);
//     each off-diagonal tile is written twice (direct and mirrored), so the
//     next step reads whole row panels of a fully stored symmetric matrix;
//   * v_mfma_f64_16x16x4_f64 with 4 wave64s per workgroup in a 2 x 2 layout,
//     each wave owning a (BT/2) x (BT/2) sub-tile of 16 x 16 accumulators;
//   * row panels are staged in LDS in double-buffered BK = 16 slices (rows
//     padded to 17 doubles so the 16 rows a fragment read touches fall into
//     distinct banks), one barrier per slice, the next slice's global loads
//     in flight under the current slice's MFMAs;
//   * diagonal tiles read one panel only;
//   * workgroups are renumbered so each XCD (blocks are dealt round-robin to
//     the 8 XCDs) receives a contiguous run of tiles, which share row panels
//     in that XCD's L2;
//   * the per-tile sums are written to a partial buffer and summed in tile
//     order by the last-arriving block: deterministic, no FP64 atomics.
#include "sp2_internal.h"

namespace sp2 {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 16;
constexpr int kLDK = kBK + 1;

template <int BT>
constexpr size_t syrk_lds_bytes() { return (size_t)2 * 2 * BT * kLDK * sizeof(double); }

// Map the hardware block index to a logical tile index so that each XCD gets
// a contiguous range (blocks b, b+8, b+16, ... run on the same XCD).
__device__ inline unsigned xcd_remap(unsigned b, unsigned nblocks) {
    const unsigned q = nblocks / 8, r = nblocks % 8;
    const unsigned x = b % 8, k = b / 8;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Logical index -> lower-triangle tile (ti >= tj), row-major over the triangle.
__device__ inline void tri_tile(unsigned L, int& ti, int& tj) {
    int i = (int)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
    while ((unsigned)((i + 1) * (i + 2) / 2) <= L) ++i;
    while ((unsigned)(i * (i + 1) / 2) > L) --i;
    ti = i;
    tj = (int)(L - (unsigned)(i * (i + 1) / 2));
}

template <int BT>
__global__ __launch_bounds__(kThreads, 1) void k_syrk_f64(const double* __restrict__ X,
                                                          double* __restrict__ Y, int ldp,
                                                          State* st, double* __restrict__ part) {
    constexpr int WT = BT / 2;            // wave sub-tile edge
    constexpr int MI = WT / 16;           // 16x16 accumulator blocks per wave edge
    constexpr int LOADS = BT * kBK / 2 / kThreads;  // double2 chunks per thread per panel
    extern __shared__ double smem[];
    __shared__ double red[4];
    __shared__ int last_flag;

    if (st->done) return;
    const int grow = st->grow;
    const unsigned nblocks = gridDim.x;
    const unsigned L = xcd_remap(blockIdx.x, nblocks);
    int ti, tj;
    tri_tile(L, ti, tj);
    const bool diag = (ti == tj);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const double* Ap = X + (size_t)ti * BT * ldp;
    const double* Bp = X + (size_t)tj * BT * ldp;
    double* sA = smem;
    double* sB = smem + 2 * BT * kLDK;

    d2 ra[LOADS], rb[LOADS];
    auto gload = [&](int kt) {
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            const int c = tid + kThreads * i;
            const int row = c >> 3, kk = (c & 7) * 2;
            ra[i] = *(const d2*)(Ap + (size_t)row * ldp + kt * kBK + kk);
            if (!diag) rb[i] = *(const d2*)(Bp + (size_t)row * ldp + kt * kBK + kk);
        }
    };
    auto sstore = [&](int stg) {
        double* a = sA + stg * BT * kLDK;
        double* b = sB + stg * BT * kLDK;
#pragma unroll
        for (int i = 0; i < LOADS; ++i) {
            const int c = tid + kThreads * i;
            const int row = c >> 3, kk = (c & 7) * 2;
            a[row * kLDK + kk] = ra[i].x;
            a[row * kLDK + kk + 1] = ra[i].y;
            if (!diag) {
                b[row * kLDK + kk] = rb[i].x;
                b[row * kLDK + kk + 1] = rb[i].y;
            }
        }
    };

    d4 acc[MI][MI];
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < MI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};

    const int KT = ldp / kBK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < KT; ++kt) {
        const int stg = kt & 1;
        if (kt + 1 < KT) gload(kt + 1);
        const double* a = sA + stg * BT * kLDK;
        const double* b = diag ? a : (sB + stg * BT * kLDK);
#pragma unroll
        for (int s = 0; s < kBK / 4; ++s) {
            const int kk = 4 * s + (lane >> 4);
            double af[MI], bf[MI];
#pragma unroll
            for (int mi = 0; mi < MI; ++mi) af[mi] = a[(wm * WT + mi * 16 + (lane & 15)) * kLDK + kk];
#pragma unroll
            for (int ni = 0; ni < MI; ++ni) bf[ni] = b[(wn * WT + ni * 16 + (lane & 15)) * kLDK + kk];
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < MI; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
        }
        if (kt + 1 < KT) sstore(stg ^ 1);
        __syncthreads();
    }

    // ---------------- fused SP2 epilogue
    // Accumulator layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l
    // holds column l%16 of the 16x16 block at rows l/16 + 4r, r = 0..3.
    // For a fixed r the 64 lanes cover 4 rows x 16 consecutive columns, so the
    // direct reads/writes are 128-byte row segments.
    double e2 = 0.0, trp = 0.0, fro = 0.0;
#pragma unroll
    for (int mi = 0; mi < MI; ++mi) {
#pragma unroll
        for (int ni = 0; ni < MI; ++ni) {
            const int gi0 = ti * BT + wm * WT + mi * 16 + (lane >> 4);
            const int gj = tj * BT + wn * WT + ni * 16 + (lane & 15);
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
    e2 = block_sum(e2, red);
    trp = block_sum(trp, red);
    fro = block_sum(fro, red);
    if (tid == 0) {
        part[4 * L + 0] = e2;
        part[4 * L + 1] = trp;
        part[4 * L + 2] = fro;
    }
    if (!arrive_last(st, nblocks, &last_flag)) return;

    // ---------------- last block: fixed-order sums and steering
    double E = 0.0, TR = 0.0, F = 0.0;
    for (unsigned k = tid; k < nblocks; k += kThreads) {
        E += part[4 * k + 0];
        TR += part[4 * k + 1];
        F += part[4 * k + 2];
    }
    E = block_sum(E, red);
    TR = block_sum(TR, red);
    F = block_sum(F, red);
    if (tid == 0) {
        const int m = st->iterations;
        const double e = sqrt(E);
        st->tr_hist[m] = st->tr;
        st->e_hist[m] = e;
        if (grow) st->branch_mask[m >> 6] |= 1ull << (m & 63);
        st->iterations = m + 1;
        st->fp64_steps = st->fp64_steps + 1;
        st->tr = TR;
        st->fro2 = F;
        st->idem = e;
        st->grow = (TR - st->nocc <= 0.0) ? 1 : 0;
        if (e <= st->tol) {
            st->done = 1;
            st->status = SP2_OK;
        } else if (m >= 2 && e >= st->e_hist[m - 2] && e < 0.1) {
            st->done = 1;
            st->status = SP2_E_STAGNATED;
        } else if (m + 1 >= st->max_iter) {
            st->done = 1;
            st->status = SP2_E_NOT_CONVERGED;
        }
        st->ticket = 0;
    }
}

template <int BT>
static hipError_t launch_bt(const Layout& L, const double* X, double* Y, State* st, double* part,
                            hipStream_t s) {
    static bool attr_set = false;
    const size_t lds = syrk_lds_bytes<BT>();
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_syrk_f64<BT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(k_syrk_f64<BT>, dim3(L.tiles), dim3(kThreads), lds, s, X, Y, L.ldp, st, part);
    return hipGetLastError();
}

hipError_t launch_syrk_f64(const Layout& L, const double* X, double* Y, State* st, double* part,
                           hipStream_t s) {
    if (L.bt == 64) return launch_bt<64>(L, X, Y, st, part, s);
    return launch_bt<128>(L, X, Y, st, part, s);
}

}  // namespace sp2
