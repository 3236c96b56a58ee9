// bounds_init.hip -- the memory-bound ends of the SP2 path on gfx950:
//   * Gershgorin spectral bounds of Hs = (H + H^T)/2 (paper: Section
//     "Distributed matrices" names the Gershgorin-circle bounds; they are the
//     emin/emax of the SP2 listing in Section "SP2 solver"),
//   * the initial iterate X_0 = (emax I - Hs)/(emax - emin) (Section "SP2
//     solver", first equation) with its trace, written into the padded FP64
//     working buffer,
//   * the final copy of the converged iterate into the caller's D.
//
// Every kernel streams H or X once through 64x64 tiles: rows are read with
// consecutive lanes on consecutive columns, and the transposed partner tile
// needed for (H + H^T)/2 goes through LDS so that both reads stay coalesced.
// Reductions are deterministic: fixed per-thread order, fixed wave/block
// order, and a last-arriving block that sums the per-block partials in index
// order.
#include "sp2_device.h"

namespace sp2 {

__global__ void k_reset(State* st, int n, int n_occ, double tol, int max_iter, int m0,
                        unsigned* cnt, int ncnt) {
    for (int i = threadIdx.x; i < ncnt; i += blockDim.x) cnt[i] = 0u;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    state_reset(st, n, n_occ, tol, max_iter, m0);
}

template <typename T>
__device__ inline double ld_h(const T* H, size_t idx) { return (double)H[idx]; }

// Row partial radii: block (rb, split) covers rows [64 rb, 64 rb + 64) and the
// column tiles [8 split, 8 split + 8).  rowpart[split * ldp + i] receives
// sum_{j in those columns, j != i} |Hs_ij|.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bounds_partial(const T* __restrict__ H, int n, int ld,
                                                             double* __restrict__ rowpart, int ldp,
                                                             State* st) {
    __shared__ double sA[kBndTile][kBndTile + 1];
    __shared__ double sB[kBndTile][kBndTile + 1];
    const int rb = blockIdx.x, split = blockIdx.y;
    const int tid = threadIdx.x;
    const int r = tid >> 2, sub = tid & 3;
    const int gi = rb * kBndTile + r;
    const int ncb = (n + kBndTile - 1) / kBndTile;
    const int per = kBndColsPerBlock / kBndTile;
    const int cb0 = split * per;
    const int cb1 = min(ncb, cb0 + per);
    double acc = 0.0;
    int bad = 0;
    for (int cb = cb0; cb < cb1; ++cb) {
        for (int e = tid; e < kBndTile * kBndTile; e += kThreads) {
            const int rr = e >> 6, cc = e & 63;
            const int ra = rb * kBndTile + rr, ca = cb * kBndTile + cc;
            const int rbb = cb * kBndTile + rr, cbb = rb * kBndTile + cc;
            sA[rr][cc] = (ra < n && ca < n) ? ld_h(H, (size_t)ra * ld + ca) : 0.0;
            sB[rr][cc] = (rbb < n && cbb < n) ? ld_h(H, (size_t)rbb * ld + cbb) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
            const int c = sub * 16 + j;
            const int gj = cb * kBndTile + c;
            const double a = sA[r][c];
            const double b = sB[c][r];
            bad |= !isfinite(a);
            const double hs = (a + b) / 2.0;
            if (gj != gi && gj < n && gi < n) acc += fabs(hs);
        }
        __syncthreads();
    }
    // the four threads of a row are adjacent lanes: combine in a fixed pattern
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (sub == 0 && gi < n) rowpart[(size_t)split * ldp + gi] = acc;
    if (bad) atomicOr(&st->bad, 1);
}

// Per-row disc ends, block min/max, and the last block's global min/max.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bounds_final(const T* __restrict__ H, int n, int ld,
                                                           const double* __restrict__ rowpart,
                                                           int ldp, int nsplit,
                                                           double* __restrict__ bpart, State* st) {
    __shared__ double red[2][4];
    __shared__ int last_flag;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    if (i < n) {
        double R = 0.0;
        for (int s = 0; s < nsplit; ++s) R += rowpart[(size_t)s * ldp + i];
        const double c = ld_h(H, (size_t)i * ld + i);
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

// X_0 tile (bi, bj) of the padded ldp x ldp FP64 buffer; zero outside n x n.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_init(const T* __restrict__ H, int n, int ld, int ldp,
                                                   double* __restrict__ X0, double* __restrict__ part,
                                                   State* st) {
    __shared__ double sB[kBndTile][kBndTile + 1];
    __shared__ double red[4];
    __shared__ int last_flag;
    const int bi = blockIdx.y, bj = blockIdx.x;
    const int nb = gridDim.x;
    const int tid = threadIdx.x;
    const double emin = st->emin, emax = st->emax;
    const double width = emax - emin;
    for (int e = tid; e < kBndTile * kBndTile; e += kThreads) {
        const int rr = e >> 6, cc = e & 63;
        const int gr = bj * kBndTile + rr, gc = bi * kBndTile + cc;
        sB[rr][cc] = (gr < n && gc < n) ? ld_h(H, (size_t)gr * ld + gc) : 0.0;
    }
    __syncthreads();
    double trp = 0.0, fro = 0.0;
    for (int e = tid; e < kBndTile * kBndTile; e += kThreads) {
        const int rr = e >> 6, cc = e & 63;
        const int gi = bi * kBndTile + rr, gj = bj * kBndTile + cc;
        double x = 0.0;
        if (gi < n && gj < n) {
            const double a = ld_h(H, (size_t)gi * ld + gj);
            const double hs = (a + sB[cc][rr]) / 2.0;
            const double num = (gi == gj) ? (emax - hs) : (0.0 - hs);
            x = num / width;
        }
        X0[(size_t)gi * ldp + gj] = x;
        fro += x * x;
        if (gi == gj) trp += x;
    }
    trp = block_sum(trp, red);
    fro = block_sum(fro, red);
    if (tid == 0) {
        part[2 * (bi * nb + bj) + 0] = trp;
        part[2 * (bi * nb + bj) + 1] = fro;
    }
    if (!arrive_last(st, gridDim.x * gridDim.y, &last_flag)) return;
    const int tiles = nb * nb;
    double t = 0.0, f = 0.0;
    for (int k = tid; k < tiles; k += kThreads) {
        t += part[2 * k + 0];
        f += part[2 * k + 1];
    }
    t = block_sum(t, red);
    f = block_sum(f, red);
    if (tid == 0) state_after_init(st, t, f);
}

// D <- last iterate (converted to the storage type), or 0 / I for the special
// occupations.  Leaves D untouched when the status is negative.  When the
// newest iterate lives only in split planes (a solve that ended in the split
// phase), it is decoded from them.
template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_finalize(T* __restrict__ D, int n, int ld, int ldp,
                                                       const double* __restrict__ x0,
                                                       const double* __restrict__ x1,
                                                       const uint16_t* __restrict__ p0,
                                                       const uint16_t* __restrict__ p1,
                                                       size_t pstride, const State* st) {
    if (st->status < 0) return;
    const int special = st->special;
    const int odd = st->iterations & 1;
    const double* src = odd ? x1 : x0;
    const uint16_t* psrc = odd ? p1 : p0;
    const bool from_planes = (MODE != SP2_C_F64) && st->stale;
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += kThreads) {
        double v;
        const size_t idx = (size_t)i * ldp + j;
        if (special == 1) v = 0.0;
        else if (special == 2) v = (i == j) ? 1.0 : 0.0;
        else if (from_planes) v = load_planes<MODE == SP2_C_F64 ? SP2_C_F16X2 : MODE>(psrc, pstride, idx);
        else v = src[idx];
        D[(size_t)i * ld + j] = (T)v;
    }
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
    const int nrb = (n + kBndTile - 1) / kBndTile;
    const int nsplit = (n + kBndColsPerBlock - 1) / kBndColsPerBlock;
    const int nfb = (n + kThreads - 1) / kThreads;
    double* bpart = rowpart + (size_t)nsplit * L.ldp;
    if (dt == SP2_F64) {
        hipLaunchKernelGGL(k_bounds_partial<double>, dim3(nrb, nsplit), dim3(kThreads), 0, s,
                           (const double*)H, n, ld, rowpart, L.ldp, st);
        hipLaunchKernelGGL(k_bounds_final<double>, dim3(nfb), dim3(kThreads), 0, s,
                           (const double*)H, n, ld, (const double*)rowpart, L.ldp, nsplit, bpart, st);
    } else {
        hipLaunchKernelGGL(k_bounds_partial<float>, dim3(nrb, nsplit), dim3(kThreads), 0, s,
                           (const float*)H, n, ld, rowpart, L.ldp, st);
        hipLaunchKernelGGL(k_bounds_final<float>, dim3(nfb), dim3(kThreads), 0, s,
                           (const float*)H, n, ld, (const double*)rowpart, L.ldp, nsplit, bpart, st);
    }
    return hipGetLastError();
}

hipError_t launch_init(const void* H, sp2_dtype dt, int n, int ld, const Layout& L, State* st,
                       double* x0, double* part, hipStream_t s) {
    const int nb = L.ldp / kBndTile;
    if (dt == SP2_F64)
        hipLaunchKernelGGL(k_init<double>, dim3(nb, nb), dim3(kThreads), 0, s, (const double*)H, n,
                           ld, L.ldp, x0, part, st);
    else
        hipLaunchKernelGGL(k_init<float>, dim3(nb, nb), dim3(kThreads), 0, s, (const float*)H, n, ld,
                           L.ldp, x0, part, st);
    return hipGetLastError();
}

template <typename T>
static void finalize_t(T* D, int n, int ld, const Layout& L, sp2_compute mode, const State* st,
                       const double* x0, const double* x1, const uint16_t* p0, const uint16_t* p1,
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
        default:
            hipLaunchKernelGGL((k_finalize<T, SP2_C_F64>), dim3(n), dim3(kThreads), 0, s, D, n, ld,
                               L.ldp, x0, x1, p0, p1, L.plane_stride, st);
    }
}

hipError_t launch_finalize(void* D, sp2_dtype dt, int n, int ld, const Layout& L, sp2_compute mode,
                           const State* st, const double* x0, const double* x1, const uint16_t* p0,
                           const uint16_t* p1, hipStream_t s) {
    if (dt == SP2_F64) finalize_t<double>((double*)D, n, ld, L, mode, st, x0, x1, p0, p1, s);
    else finalize_t<float>((float*)D, n, ld, L, mode, st, x0, x1, p0, p1, s);
    return hipGetLastError();
}

}  // namespace sp2
