// syrk_lp.hip -- one SP2 step with split-operand 16-bit products on the gfx950
// matrix cores (the low-precision phase of a mixed-precision solve).
//
// The iterate X (|x| <= 1) is held as 16-bit planes (see sp2_device.h):
// FP16 x2 (h + 2^-11 l'), BF16 x3 or BF16 x2.  S = X X^T is formed from the
// plane products with v_mfma_f32_16x16x32_{f16,bf16} in two parts:
//   * the leading term hi*hi.  Each K slice of 32 is one MFMA with a zero
//     accumulator input, so its FP32 rounding is that of a 32-term sum, and
//     the slice result is added into an FP64 accumulator.  One long FP32
//     accumulation over K = n instead rounds every slice against the O(|S|)
//     running sum, and that error grows with n (at n = 4096 it alone moves
//     the converged D by ~1e-6 rms);
//   * the correction terms hi*lo + lo*hi (+ the next order for BF16 x3), in
//     an FP32 accumulator of their own: they are 2^-11 (2^-8) of |S|, so
//     their FP32 rounding is far below the plane rounding of X'.
// S = HI_SCALE * acc64 + LO_SCALE * acc32.  The epilogue is the same SP2 update as the
// FP64 step (Section "SP2 solver": X' = X^2 or 2X - X^2 by the trace),
// evaluated in FP64 from the decoded X and S; it writes the planes of X'
// (they are the iterate during this phase: no FP64 copy is stored) and the
// per-tile e^2, trace and ||X'||^2.  The kernels launched after it complete
// the split tiles (k_step_finish) and steer (k_step_steer, sp2_steer_thread0).
//
// Design for CDNA4:
//   * 128 x 128 tiles of the lower block triangle, 8 wave64s each owning
//     64 x 32 (4 x 2 blocks of 16 x 16; FP64 + FP32 accumulators = 24 VGPRs
//     per block);
//   * operand panels go straight from global memory to LDS with the 16-byte
//     LDS-DMA load (global_load_lds_dwordx4): no staging registers.  The
//     planes are stored K-slice-tiled (plane_off), so a panel's slice is one
//     contiguous 8 KB block and each wave instruction reads 1 KiB = 16 rows x
//     64 B of whole 128-byte lines; a row's four 16-byte chunks are stored
//     XOR-swizzled by (row >> 1) & 3 so that the eight lanes a ds_read_b128
//     serves per cycle hit distinct banks;
//   * up to four K slices of 32 elements in LDS (three loading while one is
//     multiplied), one barrier per slice;
//   * the schedule of the 128-tile FP64 step: grouped raster, K-synchronous
//     data-parallel waves (the workgroups of one XCD share panels in L2) and
//     a stream-K remainder whose FP64 partial tiles k_step_finish adds in a
//     fixed order, run before the waves on even XCDs and after them on odd
//     ones.
#include "sk_finish.h"

namespace sp2 {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));
typedef long l1 __attribute__((ext_vector_type(1)));

// A K slice is 64 bytes of every row of a plane: 32 elements of the 16-bit
// formats, 64 of FP8.
constexpr int kSliceBytes = 64;

template <int BT_, int WM_, int WN_, int MODE_>
struct LpCfg {
    static constexpr int BT = BT_, WM = WM_, WN = WN_, MODE = MODE_;
    static constexpr int NT = 64 * WM * WN, NW = WM * WN;
    static constexpr int WTM = BT / WM, WTN = BT / WN;
    static constexpr int MI = WTM / 16, NI = WTN / 16;
    static constexpr int NP = Planes<MODE>::NP;
    typedef typename Planes<MODE>::Elem Elem;
    static constexpr int KE = kSliceBytes / (int)sizeof(Elem); // elements per K slice
    static constexpr int PANEL_BYTES = BT * kSliceBytes;       // one plane of one panel
    static constexpr int STAGE_BYTES = NP * 2 * PANEL_BYTES;
    static constexpr int CLD = BT + 1;                          // padded row of the LDS S tile (doubles)
    static constexpr size_t CTILE = (size_t)BT * CLD * sizeof(double);
    // K slices in flight: as many stages as fit beside nothing else (the S
    // tile of the epilogue reuses the same LDS), at most 4
    static constexpr int NS_FIT = (int)((160 * 1024) / STAGE_BYTES);
    static constexpr int NS = NS_FIT < 4 ? NS_FIT : 4;
    static_assert(NS >= 2, "two stages at least");
    static constexpr size_t LDS = (size_t)NS * STAGE_BYTES > CTILE ? (size_t)NS * STAGE_BYTES : CTILE;
    static constexpr int BLOCKS = PANEL_BYTES / 1024;           // 1 KiB LDS-DMA blocks per panel plane
    static constexpr int BPW = BLOCKS / NW;                     // ... per wave
    static_assert(BLOCKS % NW == 0, "panel must split evenly over the waves");
    static_assert(LDS + 256 <= 160 * 1024, "LDS budget of one CU (with the kernel's static LDS)");
};

// The product of one 16-byte fragment pair: 8 elements of each of the lane's
// rows for the 16-bit formats (one MFMA), 16 for FP8 (two MFMAs on the low
// and high 8 bytes; A and B use the same split of k, so the sum covers every
// k of the slice once).
template <int MODE>
__device__ __forceinline__ f4 mfma16(const uint4& a, const uint4& b, f4 c) {
    if constexpr (MODE == SP2_C_F16X2) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
    } else if constexpr (MODE == SP2_C_FP8) {
        const long alo = (long)(((unsigned long)a.y << 32) | a.x), ahi = (long)(((unsigned long)a.w << 32) | a.z);
        const long blo = (long)(((unsigned long)b.y << 32) | b.x), bhi = (long)(((unsigned long)b.w << 32) | b.z);
        c = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(alo, blo, c, 0, 0, 0);
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(ahi, bhi, c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8, a), __builtin_bit_cast(b8, b), c, 0, 0, 0);
    }
}

__device__ __forceinline__ int swz(int row) { return (row >> 1) & 3; }

// Issue the LDS-DMA loads of one K slice (all planes, both panels) into `stage`.
template <class C, bool DIAG>
__device__ __forceinline__ void lp_issue(const typename C::Elem* __restrict__ P, size_t pstride, int ldp,
                                         int rowA, int rowB, int k0, char* stage) {
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
    for (int p = 0; p < C::NP; ++p) {
#pragma unroll
        for (int q = 0; q < (DIAG ? 1 : 2); ++q) {
            const int prow0 = q ? rowB : rowA;
#pragma unroll
            for (int j = 0; j < C::BPW; ++j) {
                const int blk = w * C::BPW + j;
                const int row = blk * 16 + (lane >> 2);
                const int c = (lane & 3) ^ swz(row);
                // the K-slice-tiled plane: this slice of the panel's 128 rows is
                // one 8 KB block, 16 rows (1 KB) per wave instruction
                const typename C::Elem* src = P + p * pstride + ((size_t)(k0 / C::KE) * ldp + prow0 + row) * C::KE +
                                              c * (16 / (int)sizeof(typename C::Elem));
                char* dst = stage + (p * 2 + q) * C::PANEL_BYTES + blk * 1024;
                __builtin_amdgcn_global_load_lds((const void*)src,
                                                 (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
            }
        }
    }
}

// Wait until at most N of this wave's vector-memory loads are outstanding
// (loads complete in issue order, so the older stages are then in LDS).
template <int N>
__device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Stage kt is in LDS once at most `ahead` later stages are outstanding.
template <class C, bool DIAG>
__device__ __forceinline__ void lp_wait_stage(int ahead) {
    constexpr int L = C::NP * (DIAG ? 1 : 2) * C::BPW;   // LDS-DMA loads per stage and wave
    if (ahead >= 2) wait_vm<2 * L>();
    else if (ahead == 1) wait_vm<L>();
    else wait_vm<0>();
}

// K slices kt0..kt1-1 of tile (ti, tj): C::NS LDS stages, NS - 1 slices
// loading while one is multiplied.  Each iteration waits for its stage and
// passes one barrier, after which the stage consumed in the previous
// iteration is free for the slice NS - 1 ahead.
template <class C, bool DIAG>
__device__ __forceinline__ void lp_mainloop(const typename C::Elem* __restrict__ P, size_t pstride, int ldp,
                                            int ti, int tj, int kt0, int kt1, char* smem,
                                            d4 (&acc)[C::MI][C::NI], f4 (&accx)[C::MI][C::NI]) {
    static_assert(C::NS <= 4, "lp_wait_stage covers up to two stages ahead");
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const int rowA = ti * C::BT, rowB = tj * C::BT;
#pragma unroll
    for (int s = 0; s < C::NS - 1; ++s)
        if (kt0 + s < kt1) lp_issue<C, DIAG>(P, pstride, ldp, rowA, rowB, (kt0 + s) * C::KE, smem + s * C::STAGE_BYTES);
    // fragment addressing: row r of the wave's sub-tile, chunk c = lane >> 4
    int aoff[C::MI], boff[C::NI];
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi) {
        const int row = wm * C::WTM + mi * 16 + (lane & 15);
        aoff[mi] = row * 64 + (((lane >> 4) ^ swz(row)) << 4);
    }
#pragma unroll
    for (int ni = 0; ni < C::NI; ++ni) {
        const int row = wn * C::WTN + ni * 16 + (lane & 15);
        boff[ni] = row * 64 + (((lane >> 4) ^ swz(row)) << 4);
    }
    const f4 zero = {0.f, 0.f, 0.f, 0.f};
    // the leading term of the previous slice, promoted into FP64 one slice
    // late: its conversions and FP64 adds then never wait for an MFMA in
    // flight and overlap this slice's MFMAs (zero before the first slice:
    // adding +0.0 to the +0.0 accumulators changes no bit)
    f4 tl[C::MI][C::NI];
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) tl[mi][ni] = zero;
    int slot = 0;
    for (int kt = kt0; kt < kt1; ++kt) {
        const int ahead = (kt1 - 1 - kt) < (C::NS - 2) ? (kt1 - 1 - kt) : (C::NS - 2);
        lp_wait_stage<C, DIAG>(ahead);
        // a bare barrier: __syncthreads() would also wait for the later
        // stages' loads (its release fence drains every outstanding load)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kt + C::NS - 1 < kt1) {
            const int ls = (slot + C::NS - 1) % C::NS;
            lp_issue<C, DIAG>(P, pstride, ldp, rowA, rowB, (kt + C::NS - 1) * C::KE, smem + ls * C::STAGE_BYTES);
        }
        const char* S = smem + slot * C::STAGE_BYTES;
        slot = (slot + 1) % C::NS;
        uint4 af[C::NP][C::MI], bf[C::NP][C::NI];
#pragma unroll
        for (int p = 0; p < C::NP; ++p) {
            const char* pa = S + (p * 2 + 0) * C::PANEL_BYTES;
            const char* pb = DIAG ? pa : S + (p * 2 + 1) * C::PANEL_BYTES;
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi) af[p][mi] = *(const uint4*)(pa + aoff[mi]);
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) bf[p][ni] = *(const uint4*)(pb + boff[ni]);
        }
        // leading term: one slice per MFMA; the previous slice's goes to FP64
#pragma unroll
        for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) {
                const f4 t = tl[mi][ni];
                acc[mi][ni] += d4{(double)t[0], (double)t[1], (double)t[2], (double)t[3]};
                tl[mi][ni] = mfma16<C::MODE>(af[0][mi], bf[0][ni], zero);
            }
        // correction terms, smallest first, into the FP32 accumulator
        if constexpr (C::NP == 3) {
#pragma unroll
            for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < C::NI; ++ni) {
                    accx[mi][ni] = mfma16<C::MODE>(af[2][mi], bf[0][ni], accx[mi][ni]);
                    accx[mi][ni] = mfma16<C::MODE>(af[1][mi], bf[1][ni], accx[mi][ni]);
                    accx[mi][ni] = mfma16<C::MODE>(af[0][mi], bf[2][ni], accx[mi][ni]);
                }
        }
#pragma unroll
        for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) {
                accx[mi][ni] = mfma16<C::MODE>(af[1][mi], bf[0][ni], accx[mi][ni]);
                accx[mi][ni] = mfma16<C::MODE>(af[0][mi], bf[1][ni], accx[mi][ni]);
            }
    }
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) {
            const f4 t = tl[mi][ni];
            acc[mi][ni] += d4{(double)t[0], (double)t[1], (double)t[2], (double)t[3]};
        }
    __syncthreads();   // every wave is done with the stages before the LDS is reused
}

// Accumulators -> padded LDS tile S[BT][BT+1] (doubles), S = acc64 + LO_SCALE *
// acc32.  Accumulator layout of v_mfma_f32_16x16x32_{f16,bf16} (checked on
// gfx950): lane l holds column l%16 of the 16x16 block at rows 4*(l/16) + r,
// r = 0..3.
template <class C>
__device__ __forceinline__ void lp_acc_to_lds(const d4 (&acc)[C::MI][C::NI], const f4 (&accx)[C::MI][C::NI],
                                              double* Cs) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) {
            const int r0 = wm * C::WTM + mi * 16 + 4 * (lane >> 4);
            const int c = wn * C::WTN + ni * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                Cs[(r0 + r) * C::CLD + c] = Planes<C::MODE>::HI_SCALE * acc[mi][ni][r] +
                                            Planes<C::MODE>::LO_SCALE * (double)accx[mi][ni][r];
        }
}

// SP2 update of one finished tile held in LDS (Cs = S tile).  Each thread
// handles runs of 8 consecutive elements of a row, so every global plane
// access is one 16-byte vector.
//   pass A: the tile itself (rows of ti, columns of tj): X' from S and the
//           decoded X, the tile's e^2 / trace / ||X'||^2, the new planes;
//   pass B (off-diagonal tiles): the mirrored tile (rows of tj), from the
//           transposed LDS tile and X read at the mirrored place (the planes
//           are bitwise symmetric, so X' comes out bit-identical).
// Diagonal tiles take the lower triangle's S for both halves.  All plane
// loads of a pass are issued before the first is used, so a pass pays one
// memory latency rather than one per run.
template <class C>
__device__ __forceinline__ void lp_epilogue(const typename C::Elem* __restrict__ Pin,
                                            typename C::Elem* __restrict__ Pout,
                                            size_t pstride, int ldp, int ti, int tj, int grow,
                                            const double* Cs, double& e2, double& trp, double& fro) {
    constexpr int RUN = 8;
    constexpr int RUNS_PER_ROW = C::BT / RUN;
    constexpr int RPT = C::BT * RUNS_PER_ROW / C::NT;   // runs per thread and pass
    static_assert(C::BT * RUNS_PER_ROW % C::NT == 0, "runs must split evenly over the threads");
    const bool diag = (ti == tj);
    typedef typename C::Elem E;
    typedef E u16x8 __attribute__((ext_vector_type(8)));
    const double wgt = diag ? 1.0 : 2.0;
#pragma unroll 1
    for (int pass = 0; pass < (diag ? 1 : 2); ++pass) {
        const bool mirrored = pass == 1;
        const int rbase = (mirrored ? tj : ti) * C::BT;
        const int cbase = (mirrored ? ti : tj) * C::BT;
        u16x8 xin[RPT][C::NP];
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int q = threadIdx.x + j * C::NT;
            const int r = q / RUNS_PER_ROW, c0 = (q % RUNS_PER_ROW) * RUN;
            const size_t g = plane_off<C::MODE>((size_t)(rbase + r), (size_t)(cbase + c0), ldp);
#pragma unroll
            for (int p = 0; p < C::NP; ++p) xin[j][p] = *(const u16x8*)(Pin + p * pstride + g);
        }
        // one run per trip (the plane encoding is long code); the prefetched
        // runs shift down one register slot per trip
#pragma unroll 1
        for (int j = 0; j < RPT; ++j) {
            const int q = threadIdx.x + j * C::NT;
            const int r = q / RUNS_PER_ROW, c0 = (q % RUNS_PER_ROW) * RUN;
            const size_t g = plane_off<C::MODE>((size_t)(rbase + r), (size_t)(cbase + c0), ldp);
            u16x8 xout[C::NP];
#pragma unroll
            for (int k = 0; k < RUN; ++k) {
                const int c = c0 + k;
                // S at (row r, col c) of this pass's tile: transposed for the
                // mirrored tile and for the upper half of a diagonal tile
                const bool tr = mirrored || (diag && c > r);
                const double sd = Cs[tr ? c * C::CLD + r : r * C::CLD + c];
                E v[C::NP];
#pragma unroll
                for (int p = 0; p < C::NP; ++p) v[p] = xin[0][p][k];
                const double x = Planes<C::MODE>::decode(v);
                const double xn = grow ? (2.0 * x - sd) : sd;
                if (!mirrored) {
                    const double d = sd - x;
                    e2 += wgt * (d * d);
                    fro += wgt * (xn * xn);
                    if (diag && c == r) trp += xn;
                }
                E o[C::NP];
                Planes<C::MODE>::encode(xn, o);
#pragma unroll
                for (int p = 0; p < C::NP; ++p) xout[p][k] = o[p];
            }
#pragma unroll
            for (int p = 0; p < C::NP; ++p) *(u16x8*)(Pout + p * pstride + g) = xout[p];
#pragma unroll
            for (int jj = 0; jj + 1 < RPT; ++jj)
#pragma unroll
                for (int p = 0; p < C::NP; ++p) xin[jj][p] = xin[jj + 1][p];
        }
    }
}

// Stream-K split-operand step.  `step` is the index of the step this launch
// performs.  In the split-precision phase it does that step.  On the step
// where the loop has just handed over to the FP64 refinement (phase 2 with
// the iterate only in planes), it instead decodes the planes into the FP64
// iterate X that the FP64 step launched next reads.  Otherwise it returns at
// once.  No workgroup waits for another: the split tiles and the steering
// are k_step_finish's and k_step_steer's, launched after it.
template <class C>
__global__ __launch_bounds__(C::NT) void k_syrk_lp(const typename C::Elem* __restrict__ Pin,
                                                   typename C::Elem* __restrict__ Pout, size_t pstride,
                                                   double* __restrict__ X, int ldp, int T, State* st,
                                                   double* __restrict__ part,
                                                   double* __restrict__ scratch, int step) {
    extern __shared__ __attribute__((aligned(16))) char lsmem[];
    __shared__ double red[C::NW];

    if (st->done || st->iterations != step) return;
    const int phase = st->phase;
    if (phase == 2) {
        if (!st->stale) return;
        const size_t count = (size_t)ldp * ldp;
        for (size_t i = (size_t)blockIdx.x * C::NT + threadIdx.x; i < count; i += (size_t)gridDim.x * C::NT)
            X[i] = load_planes<C::MODE>(Pin, pstride, ldp, i / (size_t)ldp, i % (size_t)ldp);
        return;
    }
    if (phase != 1) return;
    const int grow = st->grow;
    const unsigned G = gridDim.x;
    const unsigned g = xcd_remap(blockIdx.x, G);
    const int KT = ldp / C::KE;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const unsigned waves = ntiles / G;
    const unsigned Dt = waves * G;
    const unsigned R = ntiles - Dt;
    const int tid = threadIdx.x;
    double* Cs = (double*)lsmem;       // the stage buffers are free after a main loop

    auto run = [&](int ti, int tj, int k0, int k1) {
        d4 acc[C::MI][C::NI];
        f4 accx[C::MI][C::NI];
#pragma unroll
        for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
            for (int ni = 0; ni < C::NI; ++ni) {
                acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
                accx[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
            }
        if (ti == tj) lp_mainloop<C, true>(Pin, pstride, ldp, ti, tj, k0, k1, lsmem, acc, accx);
        else lp_mainloop<C, false>(Pin, pstride, ldp, ti, tj, k0, k1, lsmem, acc, accx);
        lp_acc_to_lds<C>(acc, accx, Cs);
        __syncthreads();
    };
    auto finish = [&](unsigned t, int ti, int tj) {
        double e2 = 0.0, trp = 0.0, fro = 0.0;
        lp_epilogue<C>(Pin, Pout, pstride, ldp, ti, tj, grow, Cs, e2, trp, fro);
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
    // leaves its FP64 partial tile in slot 2g (the range's first tile) or
    // 2g + 1; k_step_finish adds them after this kernel.
    auto remainder = [&]() {
        if (R > 0) {
            const SkSplit sk(R, (unsigned)KT, G);
            // remainder owners by hardware block index: blocks are dealt round-robin
            // to the XCDs, so the owners spread over all of them
            const unsigned gr = blockIdx.x;
            unsigned u, u1;
            sk.range(gr, u, u1);
            int seg_no = 0;
            while (u < u1) {
                const unsigned r = u / (unsigned)KT;
                const int k0 = (int)(u - r * (unsigned)KT);
                const unsigned kend = (unsigned)k0 + (u1 - u);
                const int k1 = kend < (unsigned)KT ? (int)kend : KT;
                int ti, tj;
                grouped_tile(Dt + r, T, 8, ti, tj);
                run(ti, tj, k0, k1);
                u += (unsigned)(k1 - k0);
                d2* mine = (d2*)(scratch + (2 * (size_t)gr + seg_no++) * (size_t)C::BT * C::BT);
                for (int i = tid; i < C::BT * C::BT / 2; i += C::NT) {
                    const int e = 2 * i;
                    mine[i] = d2{Cs[(e / C::BT) * C::CLD + (e % C::BT)], Cs[(e / C::BT) * C::CLD + (e % C::BT) + 1]};
                }
                __syncthreads();   // the next main loop refills this LDS
            }
        }
    };
    auto waves_part = [&]() {
        // data-parallel waves over the grouped raster: the workgroups of one XCD
        // run their tiles' K slices in step and share row and column panels in L2
        for (unsigned w = 0; w < waves; ++w) {
            const unsigned t = w * G + g;
            int ti, tj;
            grouped_tile(t, T, 8, ti, tj);
            run(ti, tj, 0, KT);
            finish(t, ti, tj);
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

// The planes of the FP64 iterate, once, when the FP64 prefix hands over to the
// split-precision phase (at the start of step `step` = m0).
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_f64_to_planes(const double* __restrict__ X,
                                                            typename Planes<MODE>::Elem* __restrict__ Pout,
                                                            size_t pstride, int ldp,
                                                            size_t count, const State* st, int step) {
    if (st->done || st->iterations != step || st->phase != 1 || st->lp_steps != 0) return;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < count;
         i += (size_t)gridDim.x * kThreads)
        store_planes<MODE>(Pout, pstride, ldp, i / (size_t)ldp, i % (size_t)ldp, X[i]);
}

// Workgroups of the split-operand step: as many as are co-resident, at most
// L.lp_groups (the workspace holds 2 G partial 128-tiles).
template <class C>
static hipError_t lp_groups_cfg(const Layout& L, int* G) {
    static int per_cu = -1;
    static int cus = 0;
    if (per_cu < 0) {
        hipError_t e = hipFuncSetAttribute((const void*)k_syrk_lp<C>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS);
        if (e != hipSuccess) return e;
        int dev = 0, nb = 0;
        e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_syrk_lp<C>, C::NT, C::LDS);
        if (e != hipSuccess) return e;
        per_cu = nb < 1 ? 1 : nb;
    }
    int g = per_cu * cus;
    if (g > L.lp_groups) g = L.lp_groups;
    *G = g < 1 ? 1 : g;
    return hipSuccess;
}

template <class C>
static hipError_t launch_lp_cfg(const Layout& L, const void* Pin_, void* Pout_, double* X,
                                State* st, double* part, double* scratch, int step, hipStream_t s) {
    const typename C::Elem* Pin = (const typename C::Elem*)Pin_;
    typename C::Elem* Pout = (typename C::Elem*)Pout_;
    int G = 0;
    hipError_t e = lp_groups_cfg<C>(L, &G);
    if (e != hipSuccess) return e;
    const int T = L.ldp / C::BT;
    hipLaunchKernelGGL(k_syrk_lp<C>, dim3(G), dim3(C::NT), C::LDS, s, Pin, Pout, L.plane_stride, X,
                       L.ldp, T, st, part, scratch, step);
    return hipGetLastError();
}

// 8 waves of 64 x 32: two FP64 + one FP32 accumulator sets fit the VGPR budget
template <int MODE> using LpMain = LpCfg<kLpTile, 2, 4, MODE>;

hipError_t launch_syrk_lp(const Layout& L, sp2_compute mode, const void* Pin, void* Pout,
                          double* X, State* st, double* part, double* scratch, int step, hipStream_t s) {
    switch (mode) {
        case SP2_C_F16X2: return launch_lp_cfg<LpMain<SP2_C_F16X2>>(L, Pin, Pout, X, st, part, scratch, step, s);
        case SP2_C_BF16X3: return launch_lp_cfg<LpMain<SP2_C_BF16X3>>(L, Pin, Pout, X, st, part, scratch, step, s);
        case SP2_C_BF16X2: return launch_lp_cfg<LpMain<SP2_C_BF16X2>>(L, Pin, Pout, X, st, part, scratch, step, s);
        case SP2_C_FP8: return launch_lp_cfg<LpMain<SP2_C_FP8>>(L, Pin, Pout, X, st, part, scratch, step, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t lp_step_groups(const Layout& L, sp2_compute mode, int* G) {
    switch (mode) {
        case SP2_C_F16X2: return lp_groups_cfg<LpMain<SP2_C_F16X2>>(L, G);
        case SP2_C_BF16X3: return lp_groups_cfg<LpMain<SP2_C_BF16X3>>(L, G);
        case SP2_C_BF16X2: return lp_groups_cfg<LpMain<SP2_C_BF16X2>>(L, G);
        case SP2_C_FP8: return lp_groups_cfg<LpMain<SP2_C_FP8>>(L, G);
        default: return hipErrorInvalidValue;
    }
}

template <int MODE>
static void f64_to_planes_t(const Layout& L, const double* X, void* Pout, const State* st, int step, hipStream_t s) {
    const size_t count = (size_t)L.ldp * L.ldp;
    hipLaunchKernelGGL(k_f64_to_planes<MODE>, dim3(2048), dim3(kThreads), 0, s, X,
                       (typename Planes<MODE>::Elem*)Pout, L.plane_stride, L.ldp, count, st, step);
}

hipError_t launch_f64_to_planes(const Layout& L, sp2_compute mode, const double* X, void* Pout,
                                const State* st, int step, hipStream_t s) {
    switch (mode) {
        case SP2_C_F16X2: f64_to_planes_t<SP2_C_F16X2>(L, X, Pout, st, step, s); break;
        case SP2_C_BF16X3: f64_to_planes_t<SP2_C_BF16X3>(L, X, Pout, st, step, s); break;
        case SP2_C_BF16X2: f64_to_planes_t<SP2_C_BF16X2>(L, X, Pout, st, step, s); break;
        case SP2_C_FP8: f64_to_planes_t<SP2_C_FP8>(L, X, Pout, st, step, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sp2
