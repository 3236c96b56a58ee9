// sk_finish.h -- the kernels that end a 128-tile SP2 step (FP64 or split
// operands): k_step_finish completes the tiles that the step's stream-K
// remainder split over several workgroups, k_step_steer takes the step's
// steering decision.
//
// The step kernel (k_syrk_f64_hyb, k_syrk_lp) leaves every split tile as FP64
// partial tiles in its scratch and every whole tile's sums (e^2, trace,
// ||X'||^2) in `part`; it uses no cross-workgroup fence or counter.  Kernel
// boundaries order each kernel's writes before the next one's reads on every
// XCD, which an in-kernel hand-over can only get from agent-scope
// release/acquire fences (an L2 write-back and invalidate on each XCD,
// measured at about 20 microseconds per fence round on MI355X).
//
// k_step_finish: R * (BT / kFixRows) workgroups for R split tiles (one 8-row
// block of a tile each).  Each adds the tile's partials for its rows in
// workgroup order (the same order and operands as a single workgroup summing
// the whole tile), applies the SP2 update to its rows and to the mirrored
// columns, and stores its sums in `part` after the whole tiles'.
// k_step_steer: one workgroup adds `part` in index order and steers.
// Both serve whichever step ran (split-operand in phase 1, FP64 otherwise).
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
    struct Raw {
        v8 p[Planes<MODE>::NP];
    };
    // eight columns j..j+7 of row i (j a multiple of 8: one plane slice)
    __device__ Raw fetch(size_t i, size_t j) const {
        const size_t g = plane_off<MODE>(i, j, ldp);
        Raw r;
#pragma unroll
        for (int q = 0; q < Planes<MODE>::NP; ++q) r.p[q] = *(const v8*)(in + q * pstride + g);
        return r;
    }
    __device__ static void decode(const Raw& r, double (&x)[8]) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            E v[Planes<MODE>::NP];
#pragma unroll
            for (int q = 0; q < Planes<MODE>::NP; ++q) v[q] = r.p[q][k];
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
    struct Raw {
        d4 a, b;
    };
    __device__ Raw fetch(size_t i, size_t j) const {
        const size_t g = i * (size_t)ldp + j;
        return Raw{*(const d4*)(in + g), *(const d4*)(in + g + 4)};
    }
    __device__ static void decode(const Raw& r, double (&x)[8]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = r.a[k];
            x[k + 4] = r.b[k];
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

// One kFixRows-row block (blk) of split tile r of a step over T x T tiles of
// BT, whose stream-K remainder ran on G workgroups with K slices of KE
// elements.
template <int BT, class IO>
__device__ void sk_fix_block(const IO& io, int ldp, int T, int KE, unsigned G, unsigned blk, int grow,
                             double* __restrict__ part, const double* __restrict__ scratch) {
    constexpr int FB = BT / kFixRows;          // row blocks per tile
    constexpr int RUNS = BT / 8;               // 8-element runs per tile row
    static_assert(kFixRows == 8 && kFixRows * RUNS <= kFixThreads && BT <= kFixThreads,
                  "one run per thread for each pass");
    static_assert(kFixRows * BT / 2 == 2 * kFixThreads && BT * kFixRows / 2 == 2 * kFixThreads,
                  "two element pairs per thread for the rows and for the columns");
    __shared__ double Srow[kFixRows][BT];      // S rows r0..r0+7
    __shared__ double Scol[BT][kFixRows + 1];  // S columns r0..r0+7 (diagonal tiles)
    __shared__ double red[kFixThreads / 64];

    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const unsigned Dt = (ntiles / G) * G;
    const unsigned R = ntiles - Dt;
    const int tid = threadIdx.x;
    const unsigned r = blk / FB;
    const int b = (int)(blk % FB), r0 = b * kFixRows;
    const unsigned t = Dt + r;
    int ti, tj;
    grouped_tile(t, T, 8, ti, tj);
    const bool diag = (ti == tj);
    const SkSplit sk(R, (unsigned)(ldp / KE), G);
    unsigned ga, gb;
    sk.owners(r, ga, gb);
    const size_t tile_elems = (size_t)BT * BT;

    // this thread's run of X (rows, or the mirrored columns), fetched first so
    // that its latency overlaps the partial sums
    const bool rows = tid < kFixRows * RUNS;
    const bool mirror = !diag && !rows && tid - kFixRows * RUNS < BT;
    size_t gi = 0, gj = 0;
    if (rows) {
        gi = (size_t)(ti * BT + r0 + tid / RUNS);
        gj = (size_t)(tj * BT + (tid % RUNS) * 8);
    } else if (mirror) {
        gi = (size_t)(tj * BT + tid - kFixRows * RUNS);
        gj = (size_t)(ti * BT + r0);
    }
    typename IO::Raw xraw{};
    if (rows || mirror) xraw = io.fetch(gi, gj);

    // S rows (and for a diagonal tile S columns) of this block: the partials
    // added in workgroup order, two element pairs per thread; QB partials'
    // loads in flight at a time
    {
        constexpr int QB = 8;
        d2 vr[2], vc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) vr[j] = vc[j] = d2{0.0, 0.0};
        for (unsigned q0 = ga; q0 <= gb; q0 += QB) {
            d2 a[QB][2], c[QB][2];
#pragma unroll
            for (int u = 0; u < QB; ++u) {
                const unsigned q = q0 + u;
                if (q > gb) break;
                const double* P = scratch + (2 * (size_t)q + sk.slot(q, r)) * tile_elems;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int p = tid + j * kFixThreads;
                    a[u][j] = *(const d2*)(P + (size_t)(r0 + p / (BT / 2)) * BT + 2 * (p % (BT / 2)));
                    if (diag) c[u][j] = *(const d2*)(P + (size_t)(p / 4) * BT + r0 + 2 * (p % 4));
                }
            }
#pragma unroll
            for (int u = 0; u < QB; ++u) {
                if (q0 + u > gb) break;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    vr[j] += a[u][j];
                    if (diag) vc[j] += c[u][j];
                }
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
    if (rows) {
        const int rr = tid / RUNS, c0 = (tid % RUNS) * 8;
        const int rl = r0 + rr;                            // row inside the tile
        IO::decode(xraw, x);
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
    } else if (mirror) {
        const int c = tid - kFixRows * RUNS;
        IO::decode(xraw, x);                               // X is bitwise symmetric
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
    (void)R;
}

// The step shapes a solve may run: split-operand (T_lp 128-tiles a side,
// G_lp workgroups, K slices of KE_lp) and FP64 (T_f64 tiles a side, G_f64
// workgroups, kBK).  f64_small: the FP64 step is the 64-tile kernel, which
// finishes its split tiles itself (it has none when every tile gets its own
// workgroup) and leaves one sum per tile.
struct StepShape {
    int ldp;
    int T_lp, KE_lp, G_lp;
    int T_f64, G_f64, f64_small;
};

// Blocks of the split tiles of a step over T x T tiles on G workgroups.
__host__ __device__ inline unsigned sk_fix_blocks(int T, int G) {
    if (G <= 0) return 0;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    return (ntiles % (unsigned)G) * (unsigned)(kLpTile / kFixRows);
}

// Entries of `part` the step filled: whole tiles, then the split tiles' blocks.
__device__ inline unsigned sk_entries(int T, int G) {
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const unsigned R = ntiles % (unsigned)G;
    return ntiles - R + R * (unsigned)(kLpTile / kFixRows);
}

}  // namespace sp2
