// syrk_f64_core.h -- the FP64 tile of the SP2 step on the gfx950 matrix cores
// (Section "SP2 solver": S = X X, X' = S or 2X - S): the LDS-staged MFMA main
// loop over K slices and the fused epilogue.  Shared by the single-matrix
// stream-K kernel (syrk_f64.hip) and the batched plan (sp2_batch.hip).
#pragma once

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
// Two-operand form: the row panels of tile ti come from XA, those of tj from
// XB (C = XA XB^T, equal to XA XB for symmetric XB); DIAG (same matrix and
// ti == tj) reads one panel.
template <class C, bool DIAG>
__device__ __forceinline__ void syrk_mainloop2(const double* __restrict__ XA, const double* __restrict__ XB,
                                               int ldp, int ti, int tj, int kt0, int kt1, double* sA, double* sB,
                                               d4 (&acc)[C::MI][C::NI]) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const double* Ap = XA + (size_t)ti * C::BT * ldp;
    const double* Bp = XB + (size_t)tj * C::BT * ldp;
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

template <class C, bool DIAG>
__device__ __forceinline__ void syrk_mainloop(const double* __restrict__ X, int ldp, int ti, int tj,
                                              int kt0, int kt1, double* sA, double* sB,
                                              d4 (&acc)[C::MI][C::NI]) {
    syrk_mainloop2<C, DIAG>(X, X, ldp, ti, tj, kt0, kt1, sA, sB, acc);
}

// The SP2 update of one finished C tile, and this thread's share of the
// tile's e^2, trace and ||X'||^2.
// Accumulator layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l
// holds column l%16 of the 16x16 block at rows l/16 + 4r, r = 0..3.  For a
// fixed r the 64 lanes cover 4 rows x 16 consecutive columns, so the direct
// reads and writes are 128-byte row segments.
// GENERAL: X' = al S + be X + ga I (a layer of the learned expansion);
// otherwise the SP2 update S or 2X - S.
template <class C, bool GENERAL = false>
__device__ __forceinline__ void sp2_epilogue(const double* __restrict__ X, double* __restrict__ Y,
                                             int ldp, int ti, int tj, int grow,
                                             const d4 (&acc)[C::MI][C::NI], double& e2,
                                             double& trp, double& fro, double al = 1.0,
                                             double be = 0.0, double ga = 0.0) {
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
                double xn;
                if constexpr (GENERAL) xn = (al * s + be * x) + ((gi == gj) ? ga : 0.0);
                else xn = grow ? (2.0 * x - s) : s;
                const double wgt = (gi > gj) ? 2.0 : ((gi == gj) ? 1.0 : 0.0);
                e2 += wgt * (d * d);
                fro += wgt * (xn * xn);
                if (gi == gj) trp += xn;
                // lower copy; the upper copy mirrors it (diagonal tiles: lower half wins)
                if (!diag || gi >= gj) Y[(size_t)gi * ldp + gj] = xn;
                if (!diag || gi > gj) Y[(size_t)gj * ldp + gi] = xn;
            }
            // one block at a time: hoisting every block's X loads ahead of the
            // arithmetic would hold 4 x MI x NI doubles live per lane
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ---------------------------------------------------------------- LDS-DMA main loop
// Operand K slices go from global memory straight to LDS with the 16-byte
// LDS-DMA load (no staging registers).  One wave instruction fills 1 KiB =
// 8 rows x 128 B (16 doubles); a row's eight 16-byte chunks are stored
// XOR-swizzled by (row >> 1) & 7, so the 16 rows one fragment read touches
// fall into distinct bank groups.

__device__ __forceinline__ int swz8(int row) { return (row >> 1) & 7; }

template <class C>
struct DmaLayout {
    static constexpr int PANEL = C::BT * kBK * (int)sizeof(double);  // one K slice of one panel
    static constexpr int STAGE = 2 * PANEL;
    static constexpr size_t LDS = 2 * (size_t)STAGE;
    static constexpr int BLOCKS = PANEL / 1024;
    static constexpr int BPW = BLOCKS / C::NW;
    static_assert(kBK == 16 && BLOCKS % C::NW == 0, "one K slice is 128 B per row, split evenly over waves");
};

template <class C, bool DIAG>
__device__ __forceinline__ void f64_issue(const double* __restrict__ X, int ldp, int rowA, int rowB, int k0,
                                          char* stage) {
    using Lay = DmaLayout<C>;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int q = 0; q < (DIAG ? 1 : 2); ++q) {
        const int prow0 = q ? rowB : rowA;
#pragma unroll
        for (int j = 0; j < Lay::BPW; ++j) {
            const int blk = w * Lay::BPW + j;
            const int row = blk * 8 + (lane >> 3);
            const int c = (lane & 7) ^ swz8(row);
            const double* src = X + (size_t)(prow0 + row) * ldp + k0 + 2 * c;
            char* dst = stage + q * Lay::PANEL + blk * 1024;
            __builtin_amdgcn_global_load_lds((const void*)src, (__attribute__((address_space(3))) void*)dst, 16,
                                             0, 0);
        }
    }
}

template <class C, bool DIAG>
__device__ __forceinline__ void syrk_mainloop_dma(const double* __restrict__ X, int ldp, int ti, int tj, int kt0,
                                                  int kt1, char* smem, d4 (&acc)[C::MI][C::NI]) {
    using Lay = DmaLayout<C>;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const int rowA = ti * C::BT, rowB = tj * C::BT;
    f64_issue<C, DIAG>(X, ldp, rowA, rowB, kt0 * kBK, smem);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    // lane reads A[r][k], k = 4 s + (lane >> 4): chunk 2 s + (lane >> 5), half (lane >> 4) & 1
    int abase[C::MI], asw[C::MI], bbase[C::NI], bsw[C::NI];
    const int half = ((lane >> 4) & 1) * 8, csub = lane >> 5;
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi) {
        const int r = wm * C::WTM + mi * 16 + (lane & 15);
        abase[mi] = r * 128 + half;
        asw[mi] = swz8(r);
    }
#pragma unroll
    for (int ni = 0; ni < C::NI; ++ni) {
        const int r = wn * C::WTN + ni * 16 + (lane & 15);
        bbase[ni] = r * 128 + half;
        bsw[ni] = swz8(r);
    }
    for (int kt = kt0; kt < kt1; ++kt) {
        const int stg = (kt - kt0) & 1;
        if (kt + 1 < kt1) f64_issue<C, DIAG>(X, ldp, rowA, rowB, (kt + 1) * kBK, smem + (stg ^ 1) * Lay::STAGE);
        const char* A = smem + stg * Lay::STAGE;
        const char* B = DIAG ? A : A + Lay::PANEL;
#pragma unroll
        for (int s = 0; s < kBK / 4; ++s) {
            const int c = 2 * s + csub;
            double af[C::MI], bf[C::NI];
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi) af[mi] = *(const double*)(A + abase[mi] + ((c ^ asw[mi]) << 4));
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) bf[ni] = *(const double*)(B + bbase[ni] + ((c ^ bsw[ni]) << 4));
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni)
                    acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[mi], bf[ni], acc[mi][ni], 0, 0, 0);
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
}

// SP2 update of a finished tile through LDS, 64 rows at a time (the waves of
// one row half store their accumulators, then the whole workgroup works on
// runs of 4 consecutive doubles): X is read and Y written as coalesced 32-byte
// row runs, including the mirrored copy of an off-diagonal tile, which is read
// out of LDS transposed.  Diagonal tiles take the lower triangle's S for both
// halves.  Same update and sums as sp2_epilogue.  smem holds 64 x (BT + 1)
// doubles.
template <class C>
struct LdsEpi {
    static constexpr int HR = 64;              // rows per pass
    static constexpr int CLD = C::BT + 1;
    static constexpr size_t LDS = (size_t)HR * CLD * sizeof(double);
    static_assert(C::WTM == HR && C::WM * HR == C::BT, "one pass per row of waves");
};

// Entry kept by the drop threshold (|v| >= tau).
__device__ __forceinline__ double keep_large(double v, double tau) { return fabs(v) < tau ? 0.0 : v; }

// PRUNE: the thresholded update of the SP2 listing's cutoff: S' = drop(S),
// X' = drop(2X - S') or S', e^2 from S' - X; nz is set when X' has a nonzero.
template <class C, bool PRUNE = false>
__device__ __forceinline__ void sp2_epilogue_lds(const double* __restrict__ X, double* __restrict__ Y, int ldp,
                                                 int ti, int tj, int grow, const d4 (&acc)[C::MI][C::NI],
                                                 double* Cs, double& e2, double& trp, double& fro,
                                                 double tau = 0.0, int* nz = nullptr) {
    using E = LdsEpi<C>;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const bool diag = (ti == tj);
    constexpr int RUN = 4;
    constexpr int RPR = C::BT / RUN;           // runs per tile row
    for (int h = 0; h < C::WM; ++h) {
        __syncthreads();
        if (wm == h) {
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni) {
                    const int r0 = mi * 16 + (lane >> 4);
                    const int c = wn * C::WTN + ni * 16 + (lane & 15);
#pragma unroll
                    for (int r = 0; r < 4; ++r) Cs[(r0 + 4 * r) * E::CLD + c] = acc[mi][ni][r];
                }
        }
        __syncthreads();
        const int rt = ti * C::BT + h * E::HR;   // global row of local row 0
        const int ct = tj * C::BT;
        // direct part: local rows 0..63, tile columns 0..BT-1
        for (int q = tid; q < E::HR * RPR; q += C::NT) {
            const int r = q / RPR, c0 = (q % RPR) * RUN;
            const int lr = h * E::HR + r;        // row inside the tile
            const size_t gidx = (size_t)(rt + r) * ldp + ct + c0;
            const d4 xv = *(const d4*)(X + gidx);
            d4 out = xv;
#pragma unroll
            for (int k = 0; k < RUN; ++k) {
                const int c = c0 + k;
                double sv = Cs[r * E::CLD + c];
                if constexpr (PRUNE) sv = keep_large(sv, tau);
                const double x = xv[k];
                const double d = sv - x;
                double xn = grow ? (2.0 * x - sv) : sv;
                if constexpr (PRUNE) {
                    if (grow) xn = keep_large(xn, tau);
                    if (xn != 0.0 && (!diag || c <= lr)) *nz = 1;
                }
                const double wgt = diag ? (c < lr ? 2.0 : (c == lr ? 1.0 : 0.0)) : 2.0;
                e2 += wgt * (d * d);
                fro += wgt * (xn * xn);
                if (diag && c == lr) trp += xn;
                if (!diag || c <= lr) out[k] = xn;
            }
            if (!diag) {
                *(d4*)(Y + gidx) = out;
            } else {
#pragma unroll
                for (int k = 0; k < RUN; ++k)
                    if (c0 + k <= lr) Y[gidx + k] = out[k];
            }
        }
        // mirrored part: Y rows of the tile's columns, runs along the local rows
        constexpr int RPC = E::HR / RUN;       // runs per mirrored row
        for (int q = tid; q < C::BT * RPC; q += C::NT) {
            const int c = q / RPC, r0 = (q % RPC) * RUN;
            const size_t gidx = (size_t)(ct + c) * ldp + rt + r0;
            const d4 xv = *(const d4*)(X + gidx);   // X is bitwise symmetric
            d4 out;
            bool any = false;
#pragma unroll
            for (int k = 0; k < RUN; ++k) {
                double sv = Cs[(r0 + k) * E::CLD + c];
                if constexpr (PRUNE) sv = keep_large(sv, tau);
                const double x = xv[k];
                double xn = grow ? (2.0 * x - sv) : sv;
                if constexpr (PRUNE) {
                    if (grow) xn = keep_large(xn, tau);
                }
                out[k] = xn;
                any |= !diag || (c < h * E::HR + r0 + k);
            }
            if (!diag) {
                *(d4*)(Y + gidx) = out;
            } else if (any) {
#pragma unroll
                for (int k = 0; k < RUN; ++k)
                    if (c < h * E::HR + r0 + k) Y[gidx + k] = out[k];
            }
        }
    }
}

// Grouped raster over the lower block triangle of T x T tiles: row panels in
// groups of GM; inside a group, column by column (the square part, then the
// triangle at the group's diagonal).  Consecutive tiles share the group's row
// panels and one column panel, so the 64 tiles one XCD works on at a time
// read about 16 distinct panels.
__device__ inline void grouped_tile(unsigned L, int T, int GM, int& ti, int& tj) {
    int r0 = 0;
    for (;;) {
        const int rows = (T - r0) < GM ? (T - r0) : GM;
        const unsigned sq = (unsigned)(r0 * rows);                    // tj < r0: full columns
        const unsigned tri = (unsigned)(rows * (rows + 1) / 2);       // the diagonal block
        if (L < sq + tri) {
            if (L < sq) {
                tj = (int)(L / (unsigned)rows);
                ti = r0 + (int)(L % (unsigned)rows);
            } else {
                unsigned q = L - sq;
                int d = 0;
                while (q >= (unsigned)(rows - d)) {
                    q -= (unsigned)(rows - d);
                    ++d;
                }
                tj = r0 + d;
                ti = r0 + d + (int)q;
            }
            return;
        }
        L -= sq + tri;
        r0 += rows;
    }
}

}  // namespace sp2
