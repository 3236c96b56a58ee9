// sp2_device.h -- device helpers shared by the squaring kernels of libsp2.so:
// workgroup reductions, the stream-K tile numbering, the split-operand plane
// encodings and the device-side steering of the SP2 loop.
#pragma once

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

// True in every thread of the one workgroup that arrives last.
__device__ inline bool group_arrive_last(unsigned* ticket, unsigned nblocks, int* flag_lds) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(ticket, 1u);
        *flag_lds = (t == nblocks - 1);
    }
    __syncthreads();
    bool last = *flag_lds != 0;
    if (last) __threadfence();
    return last;
}

// ---------------------------------------------------------------- split planes
// A value x (|x| <= 1 for SP2 iterates) is kept as a sum of 16-bit planes:
//   F16X2 : x ~ h + l,        h = fp16(x), l = fp16(x - h)      (~6e-8 absolute)
//   BF16X3: x ~ b1 + b2 + b3, each plane bf16 of the remainder   (~24 bits)
//   BF16X2: x ~ b1 + b2                                        (~16 bits)
// Products use hi*hi + hi*lo + lo*hi (+ the next order for BF16X3); the
// dropped terms are below the FP32 accumulation error.

template <int MODE> struct Planes;

template <> struct Planes<SP2_C_F16X2> {
    static constexpr int NP = 2;
    typedef _Float16 T;
    __device__ static inline void encode(double x, uint16_t* out) {
        const _Float16 h = (_Float16)x;
        const _Float16 l = (_Float16)(x - (double)h);
        out[0] = __builtin_bit_cast(uint16_t, h);
        out[1] = __builtin_bit_cast(uint16_t, l);
    }
    __device__ static inline double decode(const uint16_t* in) {
        return (double)__builtin_bit_cast(_Float16, in[0]) + (double)__builtin_bit_cast(_Float16, in[1]);
    }
};

__device__ inline __bf16 to_bf16(double x) { return (__bf16)(float)x; }

template <> struct Planes<SP2_C_BF16X3> {
    static constexpr int NP = 3;
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

// Write the planes of value x at element offset `idx` (plane p lives at
// base + p * pstride).
template <int MODE>
__device__ inline void store_planes(uint16_t* base, size_t pstride, size_t idx, double x) {
    uint16_t v[Planes<MODE>::NP];
    Planes<MODE>::encode(x, v);
#pragma unroll
    for (int p = 0; p < Planes<MODE>::NP; ++p) base[p * pstride + idx] = v[p];
}

template <int MODE>
__device__ inline double load_planes(const uint16_t* base, size_t pstride, size_t idx) {
    uint16_t v[Planes<MODE>::NP];
#pragma unroll
    for (int p = 0; p < Planes<MODE>::NP; ++p) v[p] = base[p * pstride + idx];
    return Planes<MODE>::decode(v);
}

// ---------------------------------------------------------------- steering
// Run by one thread of the last-arriving workgroup after step m, with the
// fixed-order sums E = ||S - X_m||^2, TR = tr X_{m+1}, F = ||X_{m+1}||^2.
//   phase 0: FP64 steps steered by the trace (plain SP2, or the FP64 prefix of
//            a mixed-precision solve, which hands over after m0 steps);
//   phase 1: split-precision steps steered by the trace, until the
//            idempotency stops improving (the rounding floor of the split
//            products) -> phase 2;
//   phase 2: FP64 refinement: x^2 and 2x - x^2 alternate regardless of the
//            trace (a trace-steered continuation of a low-precision iterate
//            can square an eigenvalue at 1 + eps away from 1), until e <= tol.
__device__ inline void sp2_steer_thread0(State* st, double E, double TR, double F, int grow) {
    const int m = st->iterations;
    const double e = sqrt(E);
    st->tr_hist[m] = st->tr;
    st->e_hist[m] = e;
    if (grow) st->branch_mask[m >> 6] |= 1ull << (m & 63);
    st->iterations = m + 1;
    st->tr = TR;
    st->fro2 = F;
    st->idem = e;
    const int trace_grow = (TR - st->nocc <= 0.0) ? 1 : 0;
    const int phase = st->phase;
    if (phase == 0) {
        st->fp64_steps = st->fp64_steps + 1;
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
        } else if (st->m0 > 0 && m + 1 == st->m0) {
            st->phase = 1;
            st->lp_start = m + 1;
        }
    } else if (phase == 1) {
        st->lp_mask[m >> 6] |= 1ull << (m & 63);
        st->lp_steps = st->lp_steps + 1;
        st->grow = trace_grow;
        const bool floor_hit = (m - st->lp_start >= 2) && e >= st->e_hist[m - 2] && e < 0.1;
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
