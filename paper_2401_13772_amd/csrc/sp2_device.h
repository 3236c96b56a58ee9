// sp2_device.h -- device helpers shared by the squaring kernels of libsp2.so:
// workgroup reductions, the stream-K tile numbering, the split-operand plane
// encodings and the device-side steering of the SP2 loop.
#pragma once

#include <hip/hip_fp8.h>

#include "sp2_internal.h"

namespace sp2 {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Map the hardware block index to a logical index so that each XCD gets a
// contiguous range (blocks b, b+8, b+16, ... run on the same XCD).
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

// Sum over the workgroup in a fixed order (wave sums, then waves 0..NW-1).
template <int NW>
__device__ inline double group_sum(double v, double* scratch) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    double r = scratch[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) r += scratch[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- split planes
// A value x (|x| <= 1 for SP2 iterates) is kept as a sum of 16-bit planes:
//   F16X2 : x ~ h + 2^-11 l',  h = fp16(x), l' = fp16((x - h) 2^11)
//           (Ootomo & Yokota's split-FP16 form: scaling the residual keeps it
//           out of FP16's subnormal range, ~22 significant bits for |x| down
//           to 2^-14 and an absolute quantum of 2^-35 below);
//   BF16X3: x ~ b1 + b2 + b3, each plane bf16 of the remainder (~24 bits);
//   BF16X2: x ~ b1 + b2                                      (~16 bits);
//   FP8X2 : two e4m3 planes with power-of-two scales (below)   (~8 bits).
// Products: the leading term hi*hi is accumulated apart from the correction
// terms (hi*lo + lo*hi, and for BF16X3 the next order), because it alone is
// O(|S|) and sets the FP32 rounding level; see syrk_lp.hip.  LO_SCALE is the
// factor that multiplies the correction sum.

template <int MODE> struct Planes;

// FP16 nearest-even rounding of a double in a few instructions: round to FP32
// first, then force the FP32 value to round-to-odd (truncate toward zero and
// set the last bit when the first rounding was inexact).  24 >= 11 + 2 bits,
// so the second rounding to FP16 is then the correctly rounded result of x
// (Boldo & Melquiond, rounding to odd, IEEE Trans. Computers 2008); the plain
// (_Float16)x conversion has no instruction on gfx950 and becomes ~40 integer
// instructions.  NaN and infinity pass through.
__device__ inline _Float16 f64_to_f16_rn(double x) {
    const float f = (float)x;
    const double fd = (double)f;
    unsigned b = __float_as_uint(f);
    if (fd != x) b = (fabs(fd) > fabs(x) ? b - 1u : b) | 1u;
    return (_Float16)__uint_as_float(b);
}

template <> struct Planes<SP2_C_F16X2> {
    static constexpr int NP = 2;
    static constexpr double HI_SCALE = 1.0;
    static constexpr double LO_SCALE = 1.0 / 2048.0;
    typedef uint16_t Elem;
    typedef _Float16 T;
    __device__ static inline void encode(double x, uint16_t* out) {
        const _Float16 h = f64_to_f16_rn(x);
        const _Float16 l = f64_to_f16_rn((x - (double)h) * 2048.0);
        out[0] = __builtin_bit_cast(uint16_t, h);
        out[1] = __builtin_bit_cast(uint16_t, l);
    }
    __device__ static inline double decode(const uint16_t* in) {
        return (double)__builtin_bit_cast(_Float16, in[0]) +
               (double)__builtin_bit_cast(_Float16, in[1]) * (1.0 / 2048.0);
    }
};

__device__ inline __bf16 to_bf16(double x) { return (__bf16)(float)x; }

template <> struct Planes<SP2_C_BF16X3> {
    static constexpr int NP = 3;
    static constexpr double HI_SCALE = 1.0;
    static constexpr double LO_SCALE = 1.0;
    typedef uint16_t Elem;
    typedef __bf16 T;
    __device__ static inline void encode(double x, uint16_t* out) {
        const __bf16 b1 = to_bf16(x);
        const double r1 = x - (double)(float)b1;
        const __bf16 b2 = to_bf16(r1);
        const __bf16 b3 = to_bf16(r1 - (double)(float)b2);
        out[0] = __builtin_bit_cast(uint16_t, b1);
        out[1] = __builtin_bit_cast(uint16_t, b2);
        out[2] = __builtin_bit_cast(uint16_t, b3);
    }
    __device__ static inline double decode(const uint16_t* in) {
        return ((double)(float)__builtin_bit_cast(__bf16, in[0]) +
                (double)(float)__builtin_bit_cast(__bf16, in[1])) +
               (double)(float)__builtin_bit_cast(__bf16, in[2]);
    }
};

template <> struct Planes<SP2_C_BF16X2> {
    static constexpr int NP = 2;
    static constexpr double HI_SCALE = 1.0;
    static constexpr double LO_SCALE = 1.0;
    typedef uint16_t Elem;
    typedef __bf16 T;
    __device__ static inline void encode(double x, uint16_t* out) {
        const __bf16 b1 = to_bf16(x);
        const __bf16 b2 = to_bf16(x - (double)(float)b1);
        out[0] = __builtin_bit_cast(uint16_t, b1);
        out[1] = __builtin_bit_cast(uint16_t, b2);
    }
    __device__ static inline double decode(const uint16_t* in) {
        return (double)(float)__builtin_bit_cast(__bf16, in[0]) +
               (double)(float)__builtin_bit_cast(__bf16, in[1]);
    }
};

// FP8X2: two OCP e4m3 planes with fixed power-of-two scales,
//   x ~ 2^-8 q0 + 2^-12 q1,  q0 = e4m3(2^8 x),  q1 = e4m3(2^12 (x - 2^-8 q0)).
// SP2 iterates satisfy |x| <= 1, so 2^8 x stays inside e4m3's range (448);
// e4m3 keeps 4 significant bits, so q1 takes the next 4 (~8 bits in all, a
// BF16X2-class representation).  Products q_i q_j carry 2^-(16 + 4(i+j)).
template <> struct Planes<SP2_C_FP8> {
    static constexpr int NP = 2;
    static constexpr double HI_SCALE = 1.0 / 65536.0;      // 2^-16
    static constexpr double LO_SCALE = 1.0 / 1048576.0;    // 2^-20
    typedef uint8_t Elem;
    __device__ static inline uint8_t to_e4m3(double v) {
        return (uint8_t)__hip_cvt_float_to_fp8((float)v, __HIP_SATFINITE, __HIP_E4M3);
    }
    __device__ static inline double from_e4m3(uint8_t q) {
        const __half_raw h = __hip_cvt_fp8_to_halfraw((__hip_fp8_storage_t)q, __HIP_E4M3);
        return (double)__builtin_bit_cast(_Float16, h.x);
    }
    __device__ static inline void encode(double x, uint8_t* out) {
        const uint8_t q0 = to_e4m3(x * 256.0);
        const double r = x - from_e4m3(q0) * (1.0 / 256.0);
        out[0] = q0;
        out[1] = to_e4m3(r * 4096.0);
    }
    __device__ static inline double decode(const uint8_t* in) {
        return from_e4m3(in[0]) * (1.0 / 256.0) + from_e4m3(in[1]) * (1.0 / 4096.0);
    }
};

// Plane storage is K-slice-tiled: the 64-byte slice s of every row (columns
// s KE .. s KE + KE - 1, KE = 64 / element bytes) is contiguous over the ldp
// rows, so the slice of a 128-row panel that one main-loop stage loads is a
// single 8 KB block (whole 128-byte lines, 1 KB per wave instruction) rather
// than 128 half lines one row apart:
//   offset(i, j) = ((j / KE) ldp + i) KE + j mod KE.
template <int MODE>
__device__ inline size_t plane_off(size_t i, size_t j, int ldp) {
    constexpr size_t KE = 64 / sizeof(typename Planes<MODE>::Elem);
    return ((j / KE) * (size_t)ldp + i) * KE + (j % KE);
}

// Write the planes of value x at element (i, j) (plane p lives at
// base + p * pstride).
template <int MODE>
__device__ inline void store_planes(typename Planes<MODE>::Elem* base, size_t pstride, int ldp, size_t i,
                                    size_t j, double x) {
    typename Planes<MODE>::Elem v[Planes<MODE>::NP];
    Planes<MODE>::encode(x, v);
    const size_t o = plane_off<MODE>(i, j, ldp);
#pragma unroll
    for (int p = 0; p < Planes<MODE>::NP; ++p) base[p * pstride + o] = v[p];
}

template <int MODE>
__device__ inline double load_planes(const typename Planes<MODE>::Elem* base, size_t pstride, int ldp, size_t i,
                                     size_t j) {
    typename Planes<MODE>::Elem v[Planes<MODE>::NP];
    const size_t o = plane_off<MODE>(i, j, ldp);
#pragma unroll
    for (int p = 0; p < Planes<MODE>::NP; ++p) v[p] = base[p * pstride + o];
    return Planes<MODE>::decode(v);
}

// ---------------------------------------------------------------- loop state
// Start of a solve (one thread).
__device__ inline void state_reset(State* st, int n, int n_occ, double tol, int max_iter, int m0) {
    st->emin = 0.0;
    st->emax = 0.0;
    st->tr = 0.0;
    st->fro2 = 0.0;
    st->idem = 0.0;
    st->tol = tol;
    st->nocc = (double)n_occ;
    st->n = n;
    st->max_iter = max_iter;
    st->grow = 0;
    st->done = 0;
    st->status = SP2_E_NOT_CONVERGED;
    st->iterations = 0;
    st->special = 0;
    st->bad = 0;
    st->ticket = 0;
    st->fp64_steps = 0;
    st->branch_mask[0] = 0;
    st->branch_mask[1] = 0;
    st->lp_mask[0] = 0;
    st->lp_mask[1] = 0;
    st->phase = 0;
    st->m0 = m0;
    st->lp_start = 0;
    st->lp_steps = 0;
    st->refine_steps = 0;
    st->max_refine = 8;
    st->stale = 0;
    st->pad0 = 0;
    st->lp_switch = 0.0;
    st->n_layers = 0;
    st->pad1 = 0;
    st->idem_fallback = 0.0;
    st->mu_mode = 0;
    st->pad2 = 0;
    st->mu = 0.0;
    st->xmu = 0.0;
    st->sp_slices = 0ull;
    st->sp_tiles = 0ull;
    st->restart_step = -1;
    st->restarted = 0;
    st->tr0 = 0.0;
}

// Start of a solve steered by a chemical potential mu (one thread): the
// density matrix is the projector on the eigenvalues below mu.
__device__ inline void state_reset_mu(State* st, int n, double mu, double tol, int max_iter) {
    state_reset(st, n, 0, tol, max_iter, 0);
    st->mu_mode = 1;
    st->mu = mu;
}

// Start of a learned-expansion solve: n_layers trained layers, then an SP2
// check step that accepts, continues with plain SP2 up to max_iter steps in
// all, or stops for a restart from H.
__device__ inline void state_reset_learned(State* st, int n, int n_occ, double tol, int max_iter,
                                           int n_layers, double idem_fallback) {
    state_reset(st, n, n_occ, tol, max_iter, 0);
    st->n_layers = n_layers;
    st->idem_fallback = idem_fallback;
    st->phase = n_layers > 0 ? 3 : 4;
}

// Coefficients of the update X' = al S + be X + ga I of a learned layer with
// f(x) = a x^2 + b x + c: the plain map when the trace is above n_occ, the
// particle-hole form I - f(I - X) = -a S + (2a + b) X + (1 - a - b - c) I
// otherwise (grow = 1, the branch SP2 sends to 2X - X^2).
__device__ inline void learned_update_coefs(const double* abc, int grow, double& al, double& be,
                                            double& ga) {
    const double a = abc[0], b = abc[1], c = abc[2];
    if (grow) {
        al = -a;
        be = 2.0 * a + b;
        ga = 1.0 - a - b - c;
    } else {
        al = a;
        be = b;
        ga = c;
    }
}

// After the bounds and X_0 sums (one thread): the trace decides the first
// branch; special occupations, non-finite input, a degenerate spectrum and
// max_iter == 0 end the solve before the first squaring.
__device__ inline void state_after_init(State* st, double t, double f) {
    st->tr = t;
    st->tr0 = t;
    st->fro2 = f;
    st->grow = (t - st->nocc <= 0.0) ? 1 : 0;
    const int nn = st->n;
    if (st->mu_mode) {
        // mu's image under X_0 = (emax I - H)/(emax - emin); eigenvalues above
        // x_mu (energies below mu) go to 1.  mu outside the Gershgorin
        // interval: every level lies on one side of it, D = 0 or I exactly.
        const double w = st->emax - st->emin;
        st->xmu = w > 0.0 ? (st->emax - st->mu) / w : 0.5;
        st->grow = st->xmu <= 0.5 ? 1 : 0;
        if (st->bad) {
            st->status = SP2_E_INVALID;
            st->done = 1;
        } else if (st->mu <= st->emin) {
            st->special = 1;
            st->status = SP2_OK;
            st->done = 1;
            st->tr = 0.0;
        } else if (st->mu >= st->emax) {
            st->special = 2;
            st->status = SP2_OK;
            st->done = 1;
            st->tr = (double)nn;
        } else if (st->max_iter == 0) {
            st->status = SP2_E_NOT_CONVERGED;
            st->done = 1;
        }
        st->ticket = 0;
        return;
    }
    if (st->bad) {
        st->status = SP2_E_INVALID;
        st->done = 1;
    } else if (st->nocc == 0.0) {
        st->special = 1;
        st->status = SP2_OK;
        st->done = 1;
        st->tr = 0.0;
    } else if (st->nocc == (double)nn) {
        st->special = 2;
        st->status = SP2_OK;
        st->done = 1;
        st->tr = (double)nn;
    } else if (!(st->emax > st->emin)) {
        st->status = SP2_E_DEGENERATE;
        st->done = 1;
    } else if (st->max_iter == 0) {
        st->status = SP2_E_NOT_CONVERGED;
        st->done = 1;
    }
    st->ticket = 0;
}

// ---------------------------------------------------------------- steering
// Run by one thread after step m (in the step's steering kernel, or in the
// last-arriving workgroup of a kernel that reduces by arrival), with the
// fixed-order sums E = ||S - X_m||^2, TR = tr X_{m+1}, F = ||X_{m+1}||^2.
//   phase 0: FP64 steps steered by the trace (plain SP2, or the FP64 prefix of
//            a mixed-precision solve, which hands over after m0 steps);
//   phase 1: split-precision steps steered by the trace, until the
//            idempotency no longer drops tenfold over two steps (the
//            rounding floor of the split products) -> phase 2;
//   phase 2: FP64 refinement: x^2 and 2x - x^2 alternate regardless of the
//            trace (a trace-steered continuation of a low-precision iterate
//            can square an eigenvalue at 1 + eps away from 1), until e <= tol.
__device__ __forceinline__ void sp2_steer_thread0(State* st, double E, double TR, double F, int grow) {
    const int m = st->iterations;
    const double e = sqrt(E);
    st->tr_hist[m] = st->tr;
    st->e_hist[m] = e;
    if (grow) st->branch_mask[m >> 6] |= 1ull << (m & 63);
    st->iterations = m + 1;
    st->tr = TR;
    st->fro2 = F;
    st->idem = e;
    int trace_grow = (TR - st->nocc <= 0.0) ? 1 : 0;
    if (st->mu_mode) {
        // follow mu's image through the map just applied; the next branch
        // pulls it back towards 1/2 (x_mu above 1/2: x^2, else 2x - x^2)
        const double x = st->xmu;
        const double xn = grow ? x * (2.0 - x) : x * x;
        st->xmu = xn;
        trace_grow = xn <= 0.5 ? 1 : 0;
    }
    const int phase = st->phase;
    if (phase == 0) {
        if (st->restarted) st->refine_steps = st->refine_steps + 1;   // SP2 from X_0 after the layers
        else st->fp64_steps = st->fp64_steps + 1;
        st->grow = trace_grow;
        // stagnation: no progress over two steps once every eigenvalue is
        // near 0 or 1.  Steered by mu, the branch follows mu's image, which
        // takes at most two equal branches in a row: levels on the side the
        // branch pushes away from 0 or 1 can grow for two steps before the
        // other branch squares their distance, so there the test spans three
        // steps and waits for e < 1e-3.
        const int stag_span = st->mu_mode ? 3 : 2;
        const double stag_below = st->mu_mode ? 1e-3 : 0.1;
        if (e <= st->tol) {
            st->done = 1;
            st->status = SP2_OK;
        } else if (m >= stag_span && m - stag_span >= st->restart_step &&
                   e >= st->e_hist[m - stag_span] && e < stag_below) {
            st->done = 1;
            st->status = SP2_E_STAGNATED;
        } else if (m + 1 >= st->max_iter) {
            st->done = 1;
            st->status = SP2_E_NOT_CONVERGED;
        } else if (st->m0 > 0 && m + 1 == st->m0) {
            st->phase = 1;
            st->lp_start = m + 1;
        }
    } else if (phase == 1) {
        st->lp_mask[m >> 6] |= 1ull << (m & 63);
        st->lp_steps = st->lp_steps + 1;
        st->grow = trace_grow;
        // the rounding floor: from below 0.1, e no longer drops tenfold over two
        // steps (below 0.1 a pair of exact steps takes e to ~0.4 e^2, so a
        // ratio above 1/10 means the rounding level has been reached: at
        // n = 4096 FP16x2, e goes 8.3e-3, 1.5e-5, 2.5e-5, 2.4e-6, 2.6e-6, ...).
        // The earlier value decides, so that a run-away from the floor (FP8 at
        // n = 16384: e = 0.087, 0.154, 0.302, 0.6, ... as levels just outside
        // [0, 1] are squared) hands over as well
        const bool floor_hit =
            (m - st->lp_start >= 2) && e >= 0.1 * st->e_hist[m - 2] && st->e_hist[m - 2] < 0.1;
        if (e <= st->tol) {
            st->done = 1;
            st->status = SP2_OK;
            st->stale = 1;
        } else if (floor_hit || e <= st->lp_switch) {
            st->phase = 2;
            st->stale = 1;
        } else if (m + 1 >= st->max_iter) {
            st->done = 1;
            st->status = SP2_E_NOT_CONVERGED;
            st->stale = 1;
        }
    } else if (phase == 3) {
        // trained layers: steered by the trace, no stop test but convergence
        st->fp64_steps = st->fp64_steps + 1;
        st->grow = trace_grow;
        if (e <= st->tol) {
            st->done = 1;
            st->status = SP2_OK;
        } else if (m + 1 >= st->n_layers) {
            st->phase = 4;
        }
    } else if (phase == 4) {
        // the SP2 check step: e is the idempotency of the last layer's output
        // X_L.  Accepted: done.  Close to a projector (e <= 0.3 bounds every
        // eigenvalue's |x^2 - x|, so x lies in [-0.242, 1.242]): one step of
        // the other branch pulls the check step's output into [0, 1] on the
        // same side of the middle (x^2 of [-0.242, 1.242] is [0, 1.542], and
        // 2y - y^2 of that is [0, 1] with 1.542 -> 0.707; 2x - x^2 gives
        // [-0.542, 1], and y^2 of that [0, 1] with -0.542 -> 0.293), after
        // which trace-steered SP2 steps are safe (they keep [0, 1]).
        // Otherwise the solve stops for a restart from H (SP2_E_FALLBACK).
        const double terr = fabs(TR - st->nocc);
        if (e <= st->idem_fallback && terr <= st->idem_fallback) {
            st->grow = trace_grow;
            st->done = 1;
            st->status = SP2_OK;
        } else if (e <= 0.3 && m + 2 < st->max_iter) {
            st->phase = 6;
            st->grow = grow ? 0 : 1;
        } else if (st->restart_step == -2 && m + 2 < st->max_iter) {
            // the plan keeps a copy of X_0: plain SP2 from it, in this run
            st->restart_step = m + 1;
            st->restarted = 1;
            st->phase = 0;
            st->tr = st->tr0;
            st->grow = (st->tr0 - st->nocc <= 0.0) ? 1 : 0;
        } else {
            st->done = 1;
            st->status = SP2_E_FALLBACK;
        }
    } else if (phase == 6) {
        // the pull-in step after the check: plain SP2 from here
        st->refine_steps = st->refine_steps + 1;
        st->phase = 5;
        st->grow = trace_grow;
        if (e <= st->tol) {
            st->done = 1;
            st->status = SP2_OK;
        }
    } else if (phase == 5) {
        // plain SP2 after the learned layers (the stop rule of phase 0)
        st->refine_steps = st->refine_steps + 1;
        st->grow = trace_grow;
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
    } else {
        st->stale = 0;
        st->refine_steps = st->refine_steps + 1;
        st->grow = grow ? 0 : 1;
        if (e <= st->tol) {
            st->done = 1;
            st->status = SP2_OK;
        } else if (st->refine_steps >= st->max_refine) {
            st->done = 1;
            st->status = SP2_E_STAGNATED;
        } else if (m + 1 >= st->max_iter) {
            st->done = 1;
            st->status = SP2_E_NOT_CONVERGED;
        }
    }
    st->ticket = 0;
}

}  // namespace sp2
