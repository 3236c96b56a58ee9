// bounds_init.hip -- the memory-bound ends of the SP2 path on gfx950:
//   * Gershgorin spectral bounds of Hs = (H + H^T)/2 (paper: Section
//     "Distributed matrices" names the Gershgorin-circle bounds; they are the
//     emin/emax of the SP2 listing in Section "SP2 solver"),
//   * the initial iterate X_0 = (emax I - Hs)/(emax - emin) (Section "SP2
//     solver", first equation) with its trace, written into the padded FP64
//     working buffer,
//   * the final copy of the converged iterate into the caller's D.
//
// The bounds and X_0 kernels each read H once: a block takes a pair of 64x64
// tiles (I, J) and (J, I), both read row-wise (consecutive lanes on
// consecutive columns) into LDS, where the transposed element that
// (H + H^T)/2 needs is at hand; X_0's mirrored tile is written row-wise from
// the transposed LDS tile.  Reductions are deterministic: fixed per-thread
// order, fixed wave/block order, and per-block partials added in block order
// by a final kernel.
#include "bounds_core.h"

namespace sp2 {

__global__ void k_reset(State* st, int n, int n_occ, double tol, int max_iter, int m0,
                        unsigned* cnt, int ncnt) {
    for (int i = threadIdx.x; i < ncnt; i += blockDim.x) cnt[i] = 0u;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    state_reset(st, n, n_occ, tol, max_iter, m0);
}

template <typename T>
__device__ inline double ld_h(const T* H, size_t idx) { return (double)H[idx]; }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_bounds_pair(const T* __restrict__ H, int n, int ld,
                                                          double* __restrict__ rowpart, int ldp,
                                                          State* st) {
    typedef typename PairLds<T>::type L;
    __shared__ L sA[kBndTile][kBndTile + 1];
    __shared__ L sB[kBndTile][kBndTile + 1];
    int I, J;
    tri_tile(blockIdx.x, I, J);
    int bad = 0;
    load_pair(H, n, ld, I, J, sA, sB, bad);
    __syncthreads();
    pair_row_partials(n, I, J, sA, sB, rowpart, ldp);
    if (bad) atomicOr(&st->bad, 1);
}

// Per-row disc ends (R_i = the column-tile partials added in tile order),
// block min/max, and the last block's global min/max.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bounds_final(const T* __restrict__ H, int n, int ld,
                                                           const double* __restrict__ rowpart,
                                                           int ldp, int nb,
                                                           double* __restrict__ bpart, State* st) {
    __shared__ double red[2][4];
    __shared__ int last_flag;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (i < n) {
        // R_i = the column-tile partials added in tile order; eight loads in
        // flight at a time (the sum's order is unchanged)
        double R = 0.0;
        int K = 0;
        for (; K + 8 <= nb; K += 8) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = rowpart[(size_t)(K + q) * ldp + i];
#pragma unroll
            for (int q = 0; q < 8; ++q) R += v[q];
        }
        for (; K < nb; ++K) R += rowpart[(size_t)K * ldp + i];
        const double c = (double)H[(size_t)i * ld + i];
        lo = c - R;
        hi = c + R;
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = lo;
        red[1][w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bpart[2 * blockIdx.x + 0] = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
        bpart[2 * blockIdx.x + 1] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    }
    if (!arrive_last(st, gridDim.x, &last_flag)) return;
    lo = INFINITY;
    hi = -INFINITY;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kThreads) {
        lo = fmin(lo, bpart[2 * b + 0]);
        hi = fmax(hi, bpart[2 * b + 1]);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = lo;
        red[1][w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->emin = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
        st->emax = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        st->ticket = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_init_pair(const T* __restrict__ H, int n, int ld, int ldp,
                                                        double* __restrict__ X0, double* __restrict__ part,
                                                        const State* st) {
    typedef typename PairLds<T>::type L;
    // two L tiles, later one FP64 tile for the transposed write (FP32 storage:
    // the two FP32 tiles and the FP64 tile share the same 33 KB)
    constexpr int kTileElems = kBndTile * (kBndTile + 1);
    constexpr int kRaw = sizeof(L) == sizeof(double) ? 2 * kTileElems : kTileElems;
    __shared__ double raw[kRaw];
    L (*sA)[kBndTile + 1] = (L (*)[kBndTile + 1])raw;
    L (*sB)[kBndTile + 1] = (L (*)[kBndTile + 1])((L*)raw + kTileElems);
    double (*sT)[kBndTile + 1] = (double (*)[kBndTile + 1])raw;
    __shared__ double red[4];
    int I, J;
    tri_tile(blockIdx.x, I, J);
    const double emax = st->emax, width = st->emax - st->emin;
    int bad = 0;
    load_pair(H, n, ld, I, J, sA, sB, bad);
    __syncthreads();
    pair_x0(n, ldp, I, J, emax, width, sA, sB, sT, X0, red, part, blockIdx.x);
}

// tr X_0 and ||X_0||^2 from the pair partials in pair order (one block), and
// the start of the loop.
__global__ __launch_bounds__(kThreads) void k_init_final(const double* __restrict__ part, int npairs,
                                                         State* st) {
    __shared__ double red[4];
    double t = 0.0, f = 0.0;
    for (int k = threadIdx.x; k < npairs; k += kThreads) {
        t += part[2 * k + 0];
        f += part[2 * k + 1];
    }
    t = block_sum(t, red);
    f = block_sum(f, red);
    if (threadIdx.x == 0) state_after_init(st, t, f);
}

// D <- last iterate (converted to the storage type), or 0 / I for the special
// occupations.  Leaves D untouched when the status is negative.  When the
// newest iterate lives only in split planes (a solve that ended in the split
// phase), it is decoded from them.
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_finalize(T* __restrict__ D, int n, int ld, int ldp,
                                                       const double* __restrict__ x0,
                                                       const double* __restrict__ x1,
                                                       const void* __restrict__ p0,
                                                       const void* __restrict__ p1,
                                                       size_t pstride, const State* st) {
    constexpr int PM = MODE == SP2_C_F64 ? SP2_C_F16X2 : MODE;   // plane format (unused for FP64)
    typedef typename Planes<PM>::Elem E;
    if (st->status < 0) return;
    const int special = st->special;
    const int odd = st->iterations & 1;
    const double* src = odd ? x1 : x0;
    const E* psrc = (const E*)(odd ? p1 : p0);
    const bool from_planes = (MODE != SP2_C_F64) && st->stale;
    const int i = blockIdx.x;
    // U elements per thread and trip, all loaded before the first store (one
    // memory latency per trip), then the row's tail one element at a time;
    // one copy of the loop per source, so no branch sits between the loads
    auto put = [&](auto&& value) {
        constexpr int U = 8;
        int j = threadIdx.x;
        for (; j + (U - 1) * kThreads < n; j += U * kThreads) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = value(j + u * kThreads);
#pragma unroll
            for (int u = 0; u < U; ++u) D[(size_t)i * ld + j + u * kThreads] = (T)v[u];
        }
        for (; j < n; j += kThreads) D[(size_t)i * ld + j] = (T)value(j);
    };
    if (special == 1) put([](int) { return 0.0; });
    else if (special == 2) put([&](int j) { return (i == j) ? 1.0 : 0.0; });
    else if (from_planes) put([&](int j) { return load_planes<PM>(psrc, pstride, ldp, (size_t)i, (size_t)j); });
    else put([&](int j) { return src[(size_t)i * ldp + j]; });
}

// ---------------------------------------------------------------- launchers

hipError_t launch_reset(State* st, int n, int n_occ, double tol, int max_iter, int m0,
                        unsigned* cnt, int ncnt, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, s, st, n, n_occ, tol, max_iter, m0, cnt, ncnt);
    return hipGetLastError();
}

hipError_t launch_bounds(const void* H, sp2_dtype dt, int n, int ld, const Layout& L, State* st,
                         double* rowpart, double* part, hipStream_t s) {
    (void)part;
    const int nb = L.ldp / kBndTile;
    const int npairs = nb * (nb + 1) / 2;
    const int nfb = (n + kThreads - 1) / kThreads;
    double* bpart = rowpart + (size_t)nb * L.ldp;
    if (dt == SP2_F64) {
        hipLaunchKernelGGL(k_bounds_pair<double>, dim3(npairs), dim3(kThreads), 0, s, (const double*)H, n, ld,
                           rowpart, L.ldp, st);
        hipLaunchKernelGGL(k_bounds_final<double>, dim3(nfb), dim3(kThreads), 0, s, (const double*)H, n, ld,
                           (const double*)rowpart, L.ldp, nb, bpart, st);
    } else {
        hipLaunchKernelGGL(k_bounds_pair<float>, dim3(npairs), dim3(kThreads), 0, s, (const float*)H, n, ld,
                           rowpart, L.ldp, st);
        hipLaunchKernelGGL(k_bounds_final<float>, dim3(nfb), dim3(kThreads), 0, s, (const float*)H, n, ld,
                           (const double*)rowpart, L.ldp, nb, bpart, st);
    }
    return hipGetLastError();
}

hipError_t launch_init(const void* H, sp2_dtype dt, int n, int ld, const Layout& L, State* st,
                       double* x0, double* part, hipStream_t s) {
    const int nb = L.ldp / kBndTile;
    const int npairs = nb * (nb + 1) / 2;
    if (dt == SP2_F64)
        hipLaunchKernelGGL(k_init_pair<double>, dim3(npairs), dim3(kThreads), 0, s, (const double*)H, n, ld,
                           L.ldp, x0, part, st);
    else
        hipLaunchKernelGGL(k_init_pair<float>, dim3(npairs), dim3(kThreads), 0, s, (const float*)H, n, ld,
                           L.ldp, x0, part, st);
    hipLaunchKernelGGL(k_init_final, dim3(1), dim3(kThreads), 0, s, (const double*)part, npairs, st);
    return hipGetLastError();
}

template <typename T>
static void finalize_t(T* D, int n, int ld, const Layout& L, sp2_compute mode, const State* st,
                       const double* x0, const double* x1, const void* p0, const void* p1,
                       hipStream_t s) {
    switch (mode) {
        case SP2_C_F16X2:
            hipLaunchKernelGGL((k_finalize<T, SP2_C_F16X2>), dim3(n), dim3(kThreads), 0, s, D, n, ld,
                               L.ldp, x0, x1, p0, p1, L.plane_stride, st);
            break;
        case SP2_C_BF16X3:
            hipLaunchKernelGGL((k_finalize<T, SP2_C_BF16X3>), dim3(n), dim3(kThreads), 0, s, D, n, ld,
                               L.ldp, x0, x1, p0, p1, L.plane_stride, st);
            break;
        case SP2_C_BF16X2:
            hipLaunchKernelGGL((k_finalize<T, SP2_C_BF16X2>), dim3(n), dim3(kThreads), 0, s, D, n, ld,
                               L.ldp, x0, x1, p0, p1, L.plane_stride, st);
            break;
        case SP2_C_FP8:
            hipLaunchKernelGGL((k_finalize<T, SP2_C_FP8>), dim3(n), dim3(kThreads), 0, s, D, n, ld,
                               L.ldp, x0, x1, p0, p1, L.plane_stride, st);
            break;
        default:
            hipLaunchKernelGGL((k_finalize<T, SP2_C_F64>), dim3(n), dim3(kThreads), 0, s, D, n, ld,
                               L.ldp, x0, x1, p0, p1, L.plane_stride, st);
    }
}

hipError_t launch_finalize(void* D, sp2_dtype dt, int n, int ld, const Layout& L, sp2_compute mode,
                           const State* st, const double* x0, const double* x1, const void* p0,
                           const void* p1, hipStream_t s) {
    if (dt == SP2_F64) finalize_t<double>((double*)D, n, ld, L, mode, st, x0, x1, p0, p1, s);
    else finalize_t<float>((float*)D, n, ld, L, mode, st, x0, x1, p0, p1, s);
    return hipGetLastError();
}

}  // namespace sp2
