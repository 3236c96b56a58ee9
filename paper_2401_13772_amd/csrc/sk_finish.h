// sk_finish.h -- the second kernel of a 128-tile SP2 step (FP64 or split
// operands): it completes the tiles that the step's stream-K remainder split
// over several workgroups and then takes the step's steering decision.
//
// The step kernel (k_syrk_f64_hyb, k_syrk_lp) leaves every split tile as FP64
// partial tiles in its scratch and every whole tile's sums (e^2, trace,
// ||X'||^2) in `part`; it uses no cross-workgroup fence or counter.  A kernel
// boundary orders its writes before this kernel's reads on every XCD, which an
// in-kernel hand-over can only get from agent-scope release/acquire fences
// (an L2 write-back and invalidate on each XCD, measured at tens of
// microseconds per step on MI355X).
//
// Grid: R * (BT / kFixRows) workgroups for R split tiles (one 8-row block of a
// tile each), or one workgroup when R = 0.  Each adds the tile's partials for its
// rows in workgroup order (the same order and operands as a single workgroup
// summing the whole tile), applies the SP2 update to its rows and to the
// mirrored columns, and stores its sums in `part` after the whole tiles'.
// The last workgroup to arrive (one cheap fence: this kernel's own writes are
// all that is dirty) adds `part` in index order and steers.
#pragma once

#include "syrk_f64_core.h"

namespace sp2 {

constexpr int kFixThreads = 256;

// Split of the stream-K remainder: R tiles of KT K-slices over G workgroups.
// Ranges of at least KT/16 slices go to the first Gs workgroups (by hardware
// block index); a range is shorter than a tile, so it touches at most two
// tiles and leaves at most two partials (slot 0: the range's first tile).
struct SkSplit {
    unsigned U, Gs, KT;
    __device__ SkSplit(unsigned R, unsigned KT_, unsigned G) : KT(KT_) {
        U = R * KT;
        const unsigned minr = KT >= 16 ? KT / 16u : 1u;
        Gs = (U / minr < G) ? (U / minr > 0 ? U / minr : 1u) : G;
    }
    // slices [u0, u1) of workgroup gr
    __device__ void range(unsigned gr, unsigned& u0, unsigned& u1) const {
        u0 = gr < Gs ? (U * gr) / Gs : U;
        u1 = gr < Gs ? (U * (gr + 1)) / Gs : U;
    }
    // workgroups ga..gb hold the slices of remainder tile r
    __device__ void owners(unsigned r, unsigned& ga, unsigned& gb) const {
        const unsigned ts = r * KT, te = ts + KT;
        ga = ((ts + 1) * Gs - 1) / U;
        gb = (te * Gs - 1) / U;
    }
    // partial slot of tile r in workgroup q: 0 if r is q's first tile
    __device__ unsigned slot(unsigned q, unsigned r) const { return ((U * q) / Gs / KT == r) ? 0u : 1u; }
};

// Eight consecutive elements of an iterate: split planes ...
template <int MODE>
struct PlaneIO {
    typedef typename Planes<MODE>::Elem E;
    typedef E v8 __attribute__((ext_vector_type(8)));
    const E* in;
    E* out;
    size_t pstride;
    int ldp;
    // eight columns j..j+7 of row i (j a multiple of 8: one plane slice)
    __device__ void load8(size_t i, size_t j, double (&x)[8]) const {
        const size_t g = plane_off<MODE>(i, j, ldp);
        v8 p[Planes<MODE>::NP];
#pragma unroll
        for (int q = 0; q < Planes<MODE>::NP; ++q) p[q] = *(const v8*)(in + q * pstride + g);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            E v[Planes<MODE>::NP];
#pragma unroll
            for (int q = 0; q < Planes<MODE>::NP; ++q) v[q] = p[q][k];
            x[k] = Planes<MODE>::decode(v);
        }
    }
    __device__ void store8(size_t i, size_t j, const double (&x)[8]) const {
        const size_t g = plane_off<MODE>(i, j, ldp);
        v8 p[Planes<MODE>::NP];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            E v[Planes<MODE>::NP];
            Planes<MODE>::encode(x[k], v);
#pragma unroll
            for (int q = 0; q < Planes<MODE>::NP; ++q) p[q][k] = v[q];
        }
#pragma unroll
        for (int q = 0; q < Planes<MODE>::NP; ++q) *(v8*)(out + q * pstride + g) = p[q];
    }
};

// ... or FP64.
struct F64IO {
    const double* in;
    double* out;
    int ldp;
    __device__ void load8(size_t i, size_t j, double (&x)[8]) const {
        const size_t g = i * (size_t)ldp + j;
        const d4 a = *(const d4*)(in + g), b = *(const d4*)(in + g + 4);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = a[k];
            x[k + 4] = b[k];
        }
    }
    __device__ void store8(size_t i, size_t j, const double (&x)[8]) const {
        const size_t g = i * (size_t)ldp + j;
        *(d4*)(out + g) = d4{x[0], x[1], x[2], x[3]};
        *(d4*)(out + g + 4) = d4{x[4], x[5], x[6], x[7]};
    }
};

// Sum in index order of the step's per-tile sums, then the steering.
__device__ inline void sk_steer(State* st, const double* part, unsigned entries, int grow, double* red) {
    double E = 0.0, TR = 0.0, F = 0.0;
    for (unsigned k = threadIdx.x; k < entries; k += kFixThreads) {
        E += part[4 * k + 0];
        TR += part[4 * k + 1];
        F += part[4 * k + 2];
    }
    E = group_sum<kFixThreads / 64>(E, red);
    TR = group_sum<kFixThreads / 64>(TR, red);
    F = group_sum<kFixThreads / 64>(F, red);
    if (threadIdx.x == 0) sp2_steer_thread0(st, E, TR, F, grow);
}

// LP: the kernel serves the split-operand phase (phase 1), else the FP64 one.
template <int BT, class IO, bool LP>
__global__ __launch_bounds__(kFixThreads) void k_sk_finish(IO io, int ldp, int T, int KE, State* st,
                                                           double* __restrict__ part,
                                                           const double* __restrict__ scratch,
                                                           unsigned G, int step) {
    constexpr int FB = BT / kFixRows;          // row blocks per tile
    constexpr int RUNS = BT / 8;               // 8-element runs per tile row
    static_assert(kFixRows == 8 && kFixRows * RUNS <= kFixThreads && BT <= kFixThreads,
                  "one run per thread for each pass");
    static_assert(kFixRows * BT / 2 == 2 * kFixThreads && BT * kFixRows / 2 == 2 * kFixThreads,
                  "two element pairs per thread for the rows and for the columns");
    __shared__ double Srow[kFixRows][BT];      // S rows r0..r0+7
    __shared__ double Scol[BT][kFixRows + 1];  // S columns r0..r0+7 (diagonal tiles)
    __shared__ double red[kFixThreads / 64];
    __shared__ int flag;

    if (st->done || st->iterations != step) return;
    if (LP != (st->phase == 1)) return;
    const int grow = st->grow;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const unsigned Dt = (ntiles / G) * G;
    const unsigned R = ntiles - Dt;
    if (R == 0) {                              // one workgroup: the step kernel's sums are visible
        sk_steer(st, part, Dt, grow, red);
        return;
    }
    const int tid = threadIdx.x;
    const unsigned r = blockIdx.x / FB;
    const int b = (int)(blockIdx.x % FB), r0 = b * kFixRows;
    const unsigned t = Dt + r;
    int ti, tj;
    grouped_tile(t, T, 8, ti, tj);
    const bool diag = (ti == tj);
    const SkSplit sk(R, (unsigned)(ldp / KE), G);
    unsigned ga, gb;
    sk.owners(r, ga, gb);
    const size_t tile_elems = (size_t)BT * BT;

    // S rows (and for a diagonal tile S columns) of this block: the partials
    // added in workgroup order, two element pairs per thread
    {
        d2 vr[2], vc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) vr[j] = vc[j] = d2{0.0, 0.0};
        for (unsigned q = ga; q <= gb; ++q) {
            const double* P = scratch + (2 * (size_t)q + sk.slot(q, r)) * tile_elems;
            d2 a[2], c[2] = {d2{0.0, 0.0}, d2{0.0, 0.0}};
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int p = tid + j * kFixThreads;
                a[j] = *(const d2*)(P + (size_t)(r0 + p / (BT / 2)) * BT + 2 * (p % (BT / 2)));
                if (diag) c[j] = *(const d2*)(P + (size_t)(p / 4) * BT + r0 + 2 * (p % 4));
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                vr[j] += a[j];
                if (diag) vc[j] += c[j];
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int p = tid + j * kFixThreads;
            Srow[p / (BT / 2)][2 * (p % (BT / 2))] = vr[j].x;
            Srow[p / (BT / 2)][2 * (p % (BT / 2)) + 1] = vr[j].y;
            if (diag) {
                Scol[p / 4][2 * (p % 4)] = vc[j].x;
                Scol[p / 4][2 * (p % 4) + 1] = vc[j].y;
            }
        }
    }
    __syncthreads();

    // threads 0..127: the block's rows (row rr, columns c0..c0+7);
    // threads 128..255: the mirrored columns (row c of tile row block tj,
    // columns r0..r0+7 of tile column block ti), off-diagonal tiles only
    double e2 = 0.0, trp = 0.0, fro = 0.0;
    const double wgt = diag ? 1.0 : 2.0;
    double x[8], xn[8];
    if (tid < kFixRows * RUNS) {
        const int rr = tid / RUNS, c0 = (tid % RUNS) * 8;
        const int rl = r0 + rr;                            // row inside the tile
        const size_t gi = (size_t)(ti * BT + rl), gj = (size_t)(tj * BT + c0);
        io.load8(gi, gj, x);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = c0 + k;
            // a diagonal tile takes its lower triangle's S for both halves
            const double sd = (diag && c > rl) ? Scol[c][rr] : Srow[rr][c];
            xn[k] = grow ? (2.0 * x[k] - sd) : sd;
            const double d = sd - x[k];
            e2 += wgt * (d * d);
            fro += wgt * (xn[k] * xn[k]);
            if (diag && c == rl) trp += xn[k];
        }
        io.store8(gi, gj, xn);
    } else if (!diag && tid - kFixRows * RUNS < BT) {
        const int c = tid - kFixRows * RUNS;
        const size_t gi = (size_t)(tj * BT + c), gj = (size_t)(ti * BT + r0);
        io.load8(gi, gj, x);                               // X is bitwise symmetric
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double sd = Srow[k][c];
            xn[k] = grow ? (2.0 * x[k] - sd) : sd;
        }
        io.store8(gi, gj, xn);
    }
    e2 = group_sum<kFixThreads / 64>(e2, red);
    trp = group_sum<kFixThreads / 64>(trp, red);
    fro = group_sum<kFixThreads / 64>(fro, red);
    if (tid == 0) {
        const size_t k = Dt + (size_t)r * FB + b;
        part[4 * k + 0] = e2;
        part[4 * k + 1] = trp;
        part[4 * k + 2] = fro;
    }
    if (!group_arrive_last(&st->ticket, gridDim.x, &flag)) return;
    sk_steer(st, part, Dt + R * FB, grow, red);
}

// grid of k_sk_finish for `tiles` tiles after a step kernel of G workgroups
inline unsigned sk_finish_grid(int tiles, int G, int bt) {
    const unsigned R = (unsigned)(tiles % G);
    return R ? R * (unsigned)(bt / kFixRows) : 1u;
}

}  // namespace sp2
