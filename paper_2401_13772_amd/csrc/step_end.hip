// step_end.hip -- the kernels that end one SP2 step of the single-matrix
// solve, and their launch: k_step_finish completes the split tiles of the
// step's stream-K remainder (sk_fix_block of sk_finish.h), k_step_steer adds
// the step's per-tile sums and steers the next step.
#include "sk_finish.h"

namespace sp2 {

template <int MODE>
__global__ __launch_bounds__(kFixThreads) void k_step_finish(PlaneIO<MODE> lio, F64IO fio, StepShape sh,
                                                             const State* st, double* __restrict__ part,
                                                             const double* __restrict__ scratch, int step) {
    if (st->done || st->iterations != step) return;
    const bool lp = st->phase == 1;
    if (!lp && sh.f64_small) return;
    const int grow = st->grow;
    if (lp) {
        if (blockIdx.x >= sk_fix_blocks(sh.T_lp, sh.G_lp)) return;
        sk_fix_block<kLpTile>(lio, sh.ldp, sh.T_lp, sh.KE_lp, (unsigned)sh.G_lp, blockIdx.x, grow, part, scratch);
    } else {
        if (blockIdx.x >= sk_fix_blocks(sh.T_f64, sh.G_f64)) return;
        sk_fix_block<kLpTile>(fio, sh.ldp, sh.T_f64, kBK, (unsigned)sh.G_f64, blockIdx.x, grow, part, scratch);
    }
}

__global__ __launch_bounds__(kFixThreads) void k_step_steer(StepShape sh, State* st, const double* __restrict__ part,
                                                            int step) {
    __shared__ double red[kFixThreads / 64];
    if (st->done || st->iterations != step) return;
    const bool lp = st->phase == 1;
    const unsigned entries = lp ? sk_entries(sh.T_lp, sh.G_lp)
                                : sh.f64_small ? (unsigned)(sh.T_f64 * (sh.T_f64 + 1) / 2)
                                               : sk_entries(sh.T_f64, sh.G_f64);
    sk_steer(st, part, entries, st->grow, red);
}

template <int MODE>
static hipError_t step_end_t(const Layout& L, const StepShape& sh, const void* Pin, void* Pout, const double* X,
                             double* Y, State* st, double* part, const double* scratch, int step, hipStream_t s) {
    typedef typename Planes<MODE>::Elem E;
    const PlaneIO<MODE> lio{(const E*)Pin, (E*)Pout, L.plane_stride, L.ldp};
    const F64IO fio{X, Y, L.ldp};
    const unsigned lb = sk_fix_blocks(sh.T_lp, sh.G_lp), fb = sh.f64_small ? 0u : sk_fix_blocks(sh.T_f64, sh.G_f64);
    const unsigned grid = lb > fb ? lb : fb;
    if (grid > 0)
        hipLaunchKernelGGL(k_step_finish<MODE>, dim3(grid), dim3(kFixThreads), 0, s, lio, fio, sh, st, part,
                           scratch, step);
    hipLaunchKernelGGL(k_step_steer, dim3(1), dim3(kFixThreads), 0, s, sh, st, part, step);
    return hipGetLastError();
}

hipError_t launch_step_end(const Layout& L, sp2_compute mode, const void* Pin, void* Pout, const double* X,
                           double* Y, State* st, double* part, const double* scratch, int step,
                           hipStream_t s) {
    StepShape sh{};
    sh.ldp = L.ldp;
    hipError_t e = f64_step_groups(L, &sh.G_f64);
    if (e != hipSuccess) return e;
    sh.f64_small = L.bt != kLpTile;
    sh.T_f64 = L.ldp / L.bt;
    if (L.np > 0) {
        e = lp_step_groups(L, mode, &sh.G_lp);
        if (e != hipSuccess) return e;
        sh.T_lp = L.ldp / kLpTile;
        sh.KE_lp = 64 / L.pb;
    }
    switch (L.np > 0 ? mode : SP2_C_F16X2) {   // an FP64-only solve never reads planes
        case SP2_C_F16X2: return step_end_t<SP2_C_F16X2>(L, sh, Pin, Pout, X, Y, st, part, scratch, step, s);
        case SP2_C_BF16X3: return step_end_t<SP2_C_BF16X3>(L, sh, Pin, Pout, X, Y, st, part, scratch, step, s);
        case SP2_C_BF16X2: return step_end_t<SP2_C_BF16X2>(L, sh, Pin, Pout, X, Y, st, part, scratch, step, s);
        case SP2_C_FP8: return step_end_t<SP2_C_FP8>(L, sh, Pin, Pout, X, Y, st, part, scratch, step, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace sp2
