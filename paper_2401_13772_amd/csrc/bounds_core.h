// bounds_core.h -- the tile-pair device code of the Gershgorin bounds and the
// initial iterate (Section "SP2 solver", first equation; bounds as in
// Section "Distributed matrices"), shared by the single-matrix kernels
// (bounds_init.hip) and the batched plan (sp2_batch.hip) so that both add in
// the same order.
#pragma once

#include "sp2_device.h"

namespace sp2 {

// LDS tile type of storage type T (FP32 storage: FP32 tiles).
template <typename T>
struct PairLds {
    typedef double type;
};
template <>
struct PairLds<float> {
    typedef float type;
};

// The lower tile pairs: block p handles tiles (I, J) and (J, I), I >= J
// (tri_tile numbering), so every element of H is read once.  The symmetric
// part Hs_ij = (H_ij + H_ji)/2 of the pair is formed from the two tiles in
// LDS.

// Loads tiles (I, J) -> sA and (J, I) -> sB (zero outside n x n) and reports
// a non-finite entry.  L, the LDS element type, is the storage type (FP32
// storage keeps FP32 tiles: half the LDS, twice the workgroups per CU, the
// same values once widened).
template <typename T, typename L>
__device__ inline void load_pair(const T* __restrict__ H, int n, int ld, int I, int J,
                                 L (*sA)[kBndTile + 1], L (*sB)[kBndTile + 1], int& bad) {
    constexpr int V = 16 / (int)sizeof(T);     // elements per 16-byte load
    constexpr int VPR = kBndTile / V;          // loads per tile row
    typedef T vec __attribute__((ext_vector_type(V)));
    const bool whole = (I + 1) * kBndTile <= n && (J + 1) * kBndTile <= n && (ld % V) == 0 &&
                       (reinterpret_cast<uintptr_t>(H) % 16) == 0;
    if (whole) {
        // interior pair: 16-byte loads, the same values as the element loop.
        // Every load of the thread is issued before the first LDS store, so
        // the block waits for one memory latency instead of one per trip.
        constexpr int IT = kBndTile * VPR / kThreads;   // loads per thread and tile
        static_assert(kBndTile * VPR % kThreads == 0, "tile must split evenly over the threads");
        vec a[IT], b[IT];
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int e = threadIdx.x + t * kThreads;
            const int rr = e / VPR, cv = (e % VPR) * V;
            a[t] = *(const vec*)(H + (size_t)(I * kBndTile + rr) * ld + J * kBndTile + cv);
            b[t] = *(const vec*)(H + (size_t)(J * kBndTile + rr) * ld + I * kBndTile + cv);
        }
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            const int e = threadIdx.x + t * kThreads;
            const int rr = e / VPR, cv = (e % VPR) * V;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                bad |= (int)!isfinite((double)a[t][v]) | (int)!isfinite((double)b[t][v]);
                sA[rr][cv + v] = (L)a[t][v];
                sB[rr][cv + v] = (L)b[t][v];
            }
        }
        return;
    }
    for (int e = threadIdx.x; e < kBndTile * kBndTile; e += kThreads) {
        const int rr = e >> 6, cc = e & 63;
        const int ra = I * kBndTile + rr, ca = J * kBndTile + cc;
        const int rb = J * kBndTile + rr, cb = I * kBndTile + cc;
        const T a = (ra < n && ca < n) ? H[(size_t)ra * ld + ca] : T(0);
        const T b = (rb < n && cb < n) ? H[(size_t)rb * ld + cb] : T(0);
        bad |= (int)!isfinite((double)a) | (int)!isfinite((double)b);
        sA[rr][cc] = (L)a;
        sB[rr][cc] = (L)b;
    }
}

// Gershgorin row partials of one tile pair.  rowpart[K * ldp + i] = sum over
// the 64 columns of column tile K of |Hs_ij|, j != i: rows of I from the
// columns of J, and (I != J) rows of J from the columns of I.  Four threads
// per row, 16 columns each, combined in a fixed pattern.
template <typename L>
__device__ inline void pair_row_partials(int n, int I, int J, L (*sA)[kBndTile + 1],
                                         L (*sB)[kBndTile + 1], double* __restrict__ rowpart,
                                         int ldp) {
    const int tid = threadIdx.x, r = tid >> 2, q = tid & 3;
    double acc = 0.0;
    const int gi = I * kBndTile + r;
    for (int j = 0; j < 16; ++j) {
        const int c = q * 16 + j, gj = J * kBndTile + c;
        const double hs = ((double)sA[r][c] + (double)sB[c][r]) / 2.0;
        if (gj != gi && gj < n && gi < n) acc += fabs(hs);
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (q == 0) rowpart[(size_t)J * ldp + gi] = acc;
    if (I != J) {
        // row gj = J*64 + r of Hs over the columns of I: Hs_{gj, I*64 + i}
        double acc2 = 0.0;
        const int gj = J * kBndTile + r;
        for (int i = 0; i < 16; ++i) {
            const int c = q * 16 + i, gi2 = I * kBndTile + c;
            const double hs = ((double)sA[c][r] + (double)sB[r][c]) / 2.0;
            if (gi2 < n && gj < n) acc2 += fabs(hs);
        }
        acc2 += __shfl_xor(acc2, 1, 64);
        acc2 += __shfl_xor(acc2, 2, 64);
        if (q == 0) rowpart[(size_t)I * ldp + gj] = acc2;
    }
}

// X_0 of one tile pair of the padded ldp x ldp FP64 buffer (zero outside
// n x n): tile (I, J) directly, tile (J, I) as its transpose through the FP64
// LDS tile sT (which may alias sA and sB: it is written only after both are
// read), so X_0 is bitwise symmetric.  The pair's trace and ||X_0||^2 (the
// off-diagonal pair counted twice) go to pairpart[2 p], [2 p + 1].
template <typename L>
__device__ inline void pair_x0(int n, int ldp, int I, int J, double emax, double width,
                               L (*sA)[kBndTile + 1], L (*sB)[kBndTile + 1], double (*sT)[kBndTile + 1],
                               double* __restrict__ X0, double* red, double* pairpart, unsigned p) {
    const int tid = threadIdx.x;
    double xv[kBndTile * kBndTile / kThreads];
    double trp = 0.0, fro = 0.0;
    const double wgt = (I == J) ? 1.0 : 2.0;
    int k = 0;
    for (int e = tid; e < kBndTile * kBndTile; e += kThreads, ++k) {
        const int rr = e >> 6, cc = e & 63;
        const int gi = I * kBndTile + rr, gj = J * kBndTile + cc;
        double x = 0.0;
        if (gi < n && gj < n) {
            const double hs = ((double)sA[rr][cc] + (double)sB[cc][rr]) / 2.0;
            const double num = (gi == gj) ? (emax - hs) : (0.0 - hs);
            x = num / width;
        }
        xv[k] = x;
        X0[(size_t)gi * ldp + gj] = x;
        fro += wgt * (x * x);
        if (gi == gj) trp += x;
    }
    trp = block_sum(trp, red);
    fro = block_sum(fro, red);
    if (tid == 0) {
        pairpart[2 * p + 0] = trp;
        pairpart[2 * p + 1] = fro;
    }
    if (I != J) {
        __syncthreads();
        k = 0;
        for (int e = tid; e < kBndTile * kBndTile; e += kThreads, ++k) sT[e >> 6][e & 63] = xv[k];
        __syncthreads();
        for (int e = tid; e < kBndTile * kBndTile; e += kThreads) {
            const int rr = e >> 6, cc = e & 63;
            X0[(size_t)(J * kBndTile + rr) * ldp + I * kBndTile + cc] = sT[cc][rr];
        }
    }
}

}  // namespace sp2
