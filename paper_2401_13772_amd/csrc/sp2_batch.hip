// sp2_batch.hip -- the batched plan: many independent SP2 solves (the local
// subsystem solves of the paper's Section "Graph-based Divide electronic
// structure", one dense SP2 per part) in one hipGraph replay.
//
// Kernels (all grouped over the matrices of the plan):
//   k_batch_reset        loop state of every matrix;
//   k_batch_bounds_pair, k_batch_bounds_rows, k_batch_init_pair,
//   k_batch_init_final   Gershgorin bounds of (H + H^T)/2 and X_0 with its
//                        trace (Section "SP2 solver", first equation): the
//                        pair kernels one workgroup per (matrix, 64 x 64 tile
//                        pair), the others one per matrix, in the summation
//                        order of the single-matrix kernels;
//   k_batch_step<C>      one SP2 step of every matrix still running: one
//                        workgroup per (matrix, lower tile) item, the FP64 MFMA
//                        tile (operands by LDS-DMA) and fused epilogue of
//                        syrk_f64_core.h, per-tile sums, no cross-workgroup
//                        fence or counter;
//   k_batch_steer<C>     after each step, one workgroup per matrix: the
//                        matrix's tile sums in tile order and its steering
//                        (the kernel boundary orders the step's writes; an
//                        in-kernel arrival fence per item measured 3x the
//                        whole batched solve's time);
//   k_batch_finalize     D of every matrix, one workgroup per block of rows;
//   k_batch_info         the per-matrix sp2_info records.
// The plan captures reset, bounds/init, max_iter steps, finalize and info
// into one graph at creation; a run copies the caller's H/D pointers to the
// device, replays the graph and copies the infos back.  Steps of matrices
// that have stopped return at their first instruction, so the fixed graph
// needs no conditional nodes.
//
// Work placement: matrices are dealt to the 8 XCDs by a longest-processing-
// time rule on their per-step cost (~n^3), each XCD's items are kept
// contiguous in the grid (blocks are dispatched round-robin over XCDs, so a
// matrix's row panels stay in one XCD's L2), larger matrices first within an
// XCD, and the XCD ranges are padded to equal length with empty items.
//
// Tile shape: an autotuner times the grouped step kernel of each candidate
// tile shape on the plan's own size mix (X = 0 input, one step, best of
// several) and keeps the fastest; the choice is cached in a text file keyed by
// the device and the sorted size list.  Without a cache path the plan uses the
// single-matrix path's shape (64 x 64 tiles, 4 waves), so every matrix's D is
// bitwise equal to its sp2_density solve.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bounds_core.h"
#include "syrk_f64_core.h"

namespace sp2 {

struct BatchMat {
    const void* H;   // the caller's pointers, written by every run
    void* D;
    double* x0;
    double* x1;
    double* xk;        // learned plans: a kept copy of X_0 for the in-run restart (else null)
    double* part;
    double* rowpart;   // Gershgorin row partials, (ldp / 64) x ldp
    State* st;
    int n, ldp, n_occ, mu_mode;
    double mu;         // mu_mode: the chemical potential, written by every run
};

// ---------------------------------------------------------------- kernels

// n_layers < 0: plain SP2; otherwise the learned expansion (n_layers trained
// layers and the SP2 check step).
__global__ void k_batch_reset(BatchMat* mats, int batch, double tol, int max_iter, int n_layers,
                              double idem_fallback) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    if (mats[b].mu_mode) state_reset_mu(mats[b].st, mats[b].n, mats[b].mu, tol, max_iter);
    else if (n_layers < 0) state_reset(mats[b].st, mats[b].n, mats[b].n_occ, tol, max_iter, 0);
    else {
        state_reset_learned(mats[b].st, mats[b].n, mats[b].n_occ, tol, max_iter, n_layers, idem_fallback);
        if (mats[b].xk) mats[b].st->restart_step = -2;   // a rejected check restarts SP2 from X_0
    }
}

template <typename T>
__device__ inline double ld_hb(const T* H, size_t idx) { return (double)H[idx]; }

// The bounds and X_0 of every matrix in four grouped kernels, the work of
// k_bounds_pair / k_bounds_final / k_init_pair / k_init_final spread the same
// way: the pair kernels take one (matrix, tile pair) item per workgroup, the
// others one workgroup per matrix.  The pair partials, row sums and pair sums
// are the single-matrix kernels' and are added in the same order, so the
// plan's X_0 and bounds equal sp2_density's bit for bit.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_bounds_pair(const BatchMat* __restrict__ mats,
                                                                const int2* __restrict__ pairs) {
    typedef typename PairLds<T>::type L;
    __shared__ L sA[kBndTile][kBndTile + 1];
    __shared__ L sB[kBndTile][kBndTile + 1];
    const int2 it = pairs[blockIdx.x];
    const BatchMat M = mats[it.x];
    int I, J;
    tri_tile((unsigned)it.y, I, J);
    int bad = 0;
    load_pair((const T*)M.H, M.n, M.n, I, J, sA, sB, bad);
    __syncthreads();
    pair_row_partials(M.n, I, J, sA, sB, M.rowpart, M.ldp);
    if (bad) atomicOr(&M.st->bad, 1);
}

// Disc ends R_i (the column-tile partials in tile order) and emin / emax of
// one matrix per workgroup.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_bounds_rows(const BatchMat* __restrict__ mats) {
    __shared__ double red[2][4];
    const BatchMat M = mats[blockIdx.x];
    const T* __restrict__ H = (const T*)M.H;
    const int n = M.n, ldp = M.ldp, nb = ldp / kBndTile;
    const int tid = threadIdx.x;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = tid; i < n; i += kThreads) {
        double R = 0.0;
        for (int K = 0; K < nb; ++K) R += M.rowpart[(size_t)K * ldp + i];
        const double c = (double)H[(size_t)i * n + i];
        lo = fmin(lo, c - R);
        hi = fmax(hi, c + R);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
        red[0][w] = lo;
        red[1][w] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        M.st->emin = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
        M.st->emax = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
    }
}

// X_0 of one (matrix, tile pair) item per workgroup, with the pair's trace
// and ||X_0||^2 partials.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_init_pair(const BatchMat* __restrict__ mats,
                                                              const int2* __restrict__ pairs) {
    typedef typename PairLds<T>::type L;
    constexpr int kTileElems = kBndTile * (kBndTile + 1);
    constexpr int kRaw = sizeof(L) == sizeof(double) ? 2 * kTileElems : kTileElems;
    __shared__ double raw[kRaw];
    L (*sA)[kBndTile + 1] = (L (*)[kBndTile + 1])raw;
    L (*sB)[kBndTile + 1] = (L (*)[kBndTile + 1])((L*)raw + kTileElems);
    double (*sT)[kBndTile + 1] = (double (*)[kBndTile + 1])raw;
    __shared__ double red[4];
    const int2 it = pairs[blockIdx.x];
    const BatchMat M = mats[it.x];
    int I, J;
    tri_tile((unsigned)it.y, I, J);
    const double emax = M.st->emax, width = M.st->emax - M.st->emin;
    int bad = 0;
    load_pair((const T*)M.H, M.n, M.n, I, J, sA, sB, bad);
    __syncthreads();
    pair_x0(M.n, M.ldp, I, J, emax, width, sA, sB, sT, M.x0, red, M.part, (unsigned)it.y);
}

// tr X_0 and ||X_0||^2 of one matrix per workgroup (the pair partials in pair
// order), the start of its loop, and for learned plans the kept copy of X_0.
__global__ __launch_bounds__(kThreads) void k_batch_init_final(const BatchMat* __restrict__ mats) {
    __shared__ double red[4];
    const BatchMat M = mats[blockIdx.x];
    const int tid = threadIdx.x;
    const int nb = M.ldp / kBndTile;
    const int npairs = nb * (nb + 1) / 2;
    if (M.xk) {
        // keep X_0 for a restart after rejected learned layers (eight loads in
        // flight per thread)
        const size_t q = (size_t)M.ldp * M.ldp / 4;
        const d4* src = (const d4*)M.x0;
        d4* dst = (d4*)M.xk;
        constexpr int U = 8;
        size_t i = tid;
        for (; i + (U - 1) * kThreads < q; i += U * kThreads) {
            d4 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = src[i + u * kThreads];
#pragma unroll
            for (int u = 0; u < U; ++u) dst[i + u * kThreads] = v[u];
        }
        for (; i < q; i += kThreads) dst[i] = src[i];
    }
    double t = 0.0, f = 0.0;
    for (int k = tid; k < npairs; k += kThreads) {
        t += M.part[2 * k + 0];
        f += M.part[2 * k + 1];
    }
    t = block_sum(t, red);
    f = block_sum(f, red);
    if (tid == 0) state_after_init(M.st, t, f);
}

// One SP2 step of every running matrix.  items[b] = (matrix, lower tile) for
// logical block b (after the XCD renumbering); matrix -1 is padding.
// coef: 3 doubles per trained layer (a, b, c of f(x) = a x^2 + b x + c), read
// while a matrix is in its trained-layer phase.
template <class C>
__global__ __launch_bounds__(C::NT) void k_batch_step(const BatchMat* __restrict__ mats,
                                                      const int2* __restrict__ items,
                                                      const double* __restrict__ coef, int step) {
    extern __shared__ double smem[];
    __shared__ double red[C::NW];
    const int2 it = items[xcd_remap(blockIdx.x, gridDim.x)];
    if (it.x < 0) return;
    const BatchMat& M = mats[it.x];
    State* st = M.st;
    if (st->done || st->iterations != step || st->phase == 1) return;
    const int grow = st->grow;
    const int ldp = M.ldp;
    const double* X = (st->restart_step == step) ? M.xk : ((step & 1) ? M.x1 : M.x0);
    double* Y = (step & 1) ? M.x0 : M.x1;
    const int KT = ldp / kBK;
    const unsigned t = (unsigned)it.y;
    int ti, tj;
    tri_tile(t, ti, tj);
    d4 acc[C::MI][C::NI];
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    // operands by LDS-DMA (the same MFMAs in the same order as the
    // register-staged loop of the single-matrix kernel, so the same bits)
    static_assert(DmaLayout<C>::LDS <= C::LDS, "the launch's LDS holds the DMA stages");
    if (ti == tj) syrk_mainloop_dma<C, true>(X, ldp, ti, tj, 0, KT, (char*)smem, acc);
    else syrk_mainloop_dma<C, false>(X, ldp, ti, tj, 0, KT, (char*)smem, acc);
    double e2 = 0.0, trp = 0.0, fro = 0.0;
    if (st->phase == 3) {
        double al, be, ga;
        learned_update_coefs(coef + 3 * step, grow, al, be, ga);
        sp2_epilogue<C, true>(X, Y, ldp, ti, tj, grow, acc, e2, trp, fro, al, be, ga);
    } else {
        sp2_epilogue<C>(X, Y, ldp, ti, tj, grow, acc, e2, trp, fro);
    }
    e2 = group_sum<C::NW>(e2, red);
    trp = group_sum<C::NW>(trp, red);
    fro = group_sum<C::NW>(fro, red);
    const int tid = threadIdx.x;
    double* part = M.part;
    if (tid == 0) {
        part[4 * t + 0] = e2;
        part[4 * t + 1] = trp;
        part[4 * t + 2] = fro;
    }
}

// Steering of every matrix whose step `step` just ran: its tile sums in tile
// order, with the same threads and order as the single-matrix kernel's last
// workgroup (so a plan with that kernel's tile shape steers bit for bit like
// sp2_density).  grid = matrices.
template <class C>
__global__ __launch_bounds__(C::NT) void k_batch_steer(const BatchMat* __restrict__ mats, int step) {
    __shared__ double red[C::NW];
    const BatchMat& M = mats[blockIdx.x];
    State* st = M.st;
    if (st->done || st->iterations != step || st->phase == 1) return;
    const int T = M.ldp / C::BT;
    const unsigned ntiles = (unsigned)(T * (T + 1) / 2);
    const int tid = threadIdx.x;
    double E = 0.0, TR = 0.0, F = 0.0;
    for (unsigned k = tid; k < ntiles; k += C::NT) {
        E += M.part[4 * k + 0];
        TR += M.part[4 * k + 1];
        F += M.part[4 * k + 2];
    }
    E = group_sum<C::NW>(E, red);
    TR = group_sum<C::NW>(TR, red);
    F = group_sum<C::NW>(F, red);
    if (tid == 0) sp2_steer_thread0(st, E, TR, F, st->grow);
}

// D of every matrix: one (matrix, block of kFinRows rows) item per
// workgroup; a thread's elements of the block are all loaded before the first
// is stored.
constexpr int kFinRows = 8;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_batch_finalize(const BatchMat* __restrict__ mats,
                                                             const int2* __restrict__ rows) {
    const int2 it = rows[blockIdx.x];
    const BatchMat M = mats[it.x];
    const State* st = M.st;
    if (st->status < 0) return;
    const int special = st->special;
    const double* src = (st->iterations & 1) ? M.x1 : M.x0;
    T* D = (T*)M.D;
    const int n = M.n, i0 = it.y * kFinRows;
    const int cnt = (n - i0 < kFinRows ? n - i0 : kFinRows) * n;   // elements of the block, row by row
    auto put = [&](auto&& value) {
        constexpr int U = 16;
        for (int q0 = threadIdx.x; q0 < cnt; q0 += U * kThreads) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * kThreads;
                v[u] = q < cnt ? value(i0 + q / n, q % n) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int q = q0 + u * kThreads;
                if (q < cnt) D[(size_t)i0 * n + q] = (T)v[u];
            }
        }
    };
    if (special == 1) put([](int, int) { return 0.0; });
    else if (special == 2) put([](int i, int j) { return (i == j) ? 1.0 : 0.0; });
    else put([&](int i, int j) { return src[(size_t)i * M.ldp + j]; });
}

__global__ void k_batch_info(const BatchMat* __restrict__ mats, int batch, sp2_info* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const State* st = mats[b].st;
    sp2_info r;
    // a solve restarted from X_0 after rejected learned layers is reported
    // as a fallback (its D is that of the plain SP2 solve)
    r.status = (st->restarted && st->status == SP2_OK) ? SP2_E_FALLBACK : st->status;
    r.iterations = st->iterations;
    r.fp64_prefix_iters = st->fp64_steps;
    r.refine_steps = st->refine_steps;
    r.trace = st->tr;
    r.trace_error = st->mu_mode ? 0.0 : fabs(st->tr - st->nocc);
    r.idempotency = st->idem;
    r.emin = st->emin;
    r.emax = st->emax;
    r.branch_mask[0] = st->branch_mask[0];
    r.branch_mask[1] = st->branch_mask[1];
    out[b] = r;
}

// ---------------------------------------------------------------- tile shapes

using BCfg64 = SyrkCfg<64, 2, 2>;  // the single-matrix shape for n <= 2048
using BCfg32 = SyrkCfg<32, 1, 1>;  // one wave per 32 x 32 tile: 4x the items

constexpr int kNumCfg = 2;
constexpr int kCfgBT[kNumCfg] = {64, 32};
const char* const kCfgName[kNumCfg] = {"bt64w4", "bt32w1"};

template <class C>
hipError_t prepare_cfg() {
    return hipFuncSetAttribute((const void*)k_batch_step<C>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)C::LDS);
}

// One grouped step, then the steering of each of the nmats matrices.
hipError_t launch_batch_step(int cfg, const BatchMat* mats, int nmats, const int2* items, const double* coef,
                             int nblocks, int step, hipStream_t s) {
    if (cfg == 0) {
        hipLaunchKernelGGL(k_batch_step<BCfg64>, dim3(nblocks), dim3(BCfg64::NT), BCfg64::LDS, s, mats,
                           items, coef, step);
        hipLaunchKernelGGL(k_batch_steer<BCfg64>, dim3(nmats), dim3(BCfg64::NT), 0, s, mats, step);
    } else {
        hipLaunchKernelGGL(k_batch_step<BCfg32>, dim3(nblocks), dim3(BCfg32::NT), BCfg32::LDS, s, mats,
                           items, coef, step);
        hipLaunchKernelGGL(k_batch_steer<BCfg32>, dim3(nmats), dim3(BCfg32::NT), 0, s, mats, step);
    }
    return hipGetLastError();
}

}  // namespace sp2

// ---------------------------------------------------------------- the plan

struct sp2_plan {
    int batch = 0;
    sp2_dtype dtype = SP2_F64;
    sp2_compute compute = SP2_C_F64;
    double tol = 0.0;
    int max_iter = 0;
    int cfg = 0;
    int device = 0;
    std::vector<int> order;   // order[k] = caller index of the plan's k-th matrix
    std::vector<int> n;       // caller order
    void* dmem = nullptr;     // every device buffer of the plan, one allocation
    sp2::BatchMat* d_mats = nullptr;
    int2* d_items = nullptr;
    int nblocks = 0;
    int2* d_pairs = nullptr;          // (matrix, 64 x 64 tile pair) items of the bounds and X_0
    int npairs = 0;
    int2* d_rows = nullptr;           // (matrix, block of kFinRows rows) items of the finalize
    int nrows = 0;
    sp2_info* d_infos = nullptr;
    double* d_coef = nullptr;         // learned expansion: 3 per layer
    int n_layers = -1;                // -1: plain SP2
    double idem_fallback = 0.0;
    int mu_mode = 0;                  // 1: steered by a chemical potential per run
    sp2::BatchMat* h_mats = nullptr;  // pinned
    sp2_info* h_infos = nullptr;      // pinned
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char cfg_name[16] = {0};
};

namespace {

using namespace sp2;

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// Items of one tile shape: matrices dealt to the 8 XCDs by LPT on n^3, each
// XCD's items contiguous, larger matrices first, ranges padded to one length.
std::vector<int2> build_items(const std::vector<int>& ldp, int bt) {
    const int batch = (int)ldp.size();
    std::vector<int> idx(batch);
    for (int i = 0; i < batch; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return ldp[a] > ldp[b]; });
    std::vector<std::vector<int2>> xcd(8);
    std::vector<double> load(8, 0.0);
    for (int m : idx) {
        int best = 0;
        for (int x = 1; x < 8; ++x)
            if (load[x] < load[best]) best = x;
        const int T = ldp[m] / bt;
        const int tiles = T * (T + 1) / 2;
        load[best] += (double)tiles * ldp[m];
        for (int t = 0; t < tiles; ++t) xcd[best].push_back(make_int2(m, t));
    }
    size_t q = 0;
    for (auto& v : xcd) q = std::max(q, v.size());
    std::vector<int2> items;
    items.reserve(8 * q);
    for (auto& v : xcd) {
        items.insert(items.end(), v.begin(), v.end());
        for (size_t k = v.size(); k < q; ++k) items.push_back(make_int2(-1, 0));
    }
    return items;
}

std::string autotune_key(const std::vector<int>& n, sp2_compute compute) {
    std::vector<int> s(n);
    std::sort(s.begin(), s.end());
    unsigned long long h = 1469598103934665603ull;  // FNV-1a over the sorted sizes
    for (int v : s) {
        h ^= (unsigned)v;
        h *= 1099511628211ull;
    }
    hipDeviceProp_t p{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&p, dev);
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%s:%d:c%d:%016llx", p.gcnArchName, (int)n.size(), (int)compute, h);
    for (char* c = buf; *c; ++c)
        if (*c == ' ') *c = '_';
    return buf;
}

int cache_lookup(const char* path, const std::string& key) {
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char k[192], v[32];
    int found = -1;
    while (std::fscanf(f, "%191s %31s", k, v) == 2)
        if (key == k)
            for (int c = 0; c < kNumCfg; ++c)
                if (!std::strcmp(v, kCfgName[c])) found = c;
    std::fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, int cfg) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %s\n", key.c_str(), kCfgName[cfg]);
    std::fclose(f);
}

void plan_free(sp2_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->h_mats) (void)hipHostFree(p->h_mats);
    if (p->h_infos) (void)hipHostFree(p->h_infos);
    if (p->dmem) (void)hipFree(p->dmem);
    delete p;
}

// The launch sequence of one batched solve on stream s (captured into the graph).
hipError_t enqueue_solve(sp2_plan* p, hipStream_t s) {
    const int tb = 256;
    hipLaunchKernelGGL(k_batch_reset, dim3((p->batch + tb - 1) / tb), dim3(tb), 0, s, p->d_mats, p->batch,
                       p->tol, p->max_iter, p->n_layers, p->idem_fallback);
    if (p->dtype == SP2_F64) {
        hipLaunchKernelGGL(k_batch_bounds_pair<double>, dim3(p->npairs), dim3(kThreads), 0, s, p->d_mats,
                           p->d_pairs);
        hipLaunchKernelGGL(k_batch_bounds_rows<double>, dim3(p->batch), dim3(kThreads), 0, s, p->d_mats);
        hipLaunchKernelGGL(k_batch_init_pair<double>, dim3(p->npairs), dim3(kThreads), 0, s, p->d_mats,
                           p->d_pairs);
    } else {
        hipLaunchKernelGGL(k_batch_bounds_pair<float>, dim3(p->npairs), dim3(kThreads), 0, s, p->d_mats,
                           p->d_pairs);
        hipLaunchKernelGGL(k_batch_bounds_rows<float>, dim3(p->batch), dim3(kThreads), 0, s, p->d_mats);
        hipLaunchKernelGGL(k_batch_init_pair<float>, dim3(p->npairs), dim3(kThreads), 0, s, p->d_mats,
                           p->d_pairs);
    }
    hipLaunchKernelGGL(k_batch_init_final, dim3(p->batch), dim3(kThreads), 0, s, p->d_mats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int step = 0; step < p->max_iter; ++step) {
        e = launch_batch_step(p->cfg, p->d_mats, p->batch, p->d_items, p->d_coef, p->nblocks, step, s);
        if (e != hipSuccess) return e;
    }
    if (p->dtype == SP2_F64)
        hipLaunchKernelGGL(k_batch_finalize<double>, dim3(p->nrows), dim3(kThreads), 0, s, p->d_mats, p->d_rows);
    else
        hipLaunchKernelGGL(k_batch_finalize<float>, dim3(p->nrows), dim3(kThreads), 0, s, p->d_mats, p->d_rows);
    hipLaunchKernelGGL(k_batch_info, dim3((p->batch + tb - 1) / tb), dim3(tb), 0, s, p->d_mats, p->batch,
                       p->d_infos);
    return hipGetLastError();
}

// Time one grouped step of tile shape `cfg` on X = 0 (best of `reps`).
hipError_t time_cfg(sp2_plan* p, const std::vector<int2>& items, int2* d_items_tmp, int cfg,
                    hipStream_t s, float* best_ms) {
    hipError_t e = hipMemcpyAsync(d_items_tmp, items.data(), items.size() * sizeof(int2),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    *best_ms = 1e30f;
    const int tb = 256;
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
        hipLaunchKernelGGL(k_batch_reset, dim3((p->batch + tb - 1) / tb), dim3(tb), 0, s, p->d_mats,
                           p->batch, p->tol, 1, -1, 0.0);
        (void)hipEventRecord(a, s);
        e = launch_batch_step(cfg, p->d_mats, p->batch, d_items_tmp, p->d_coef, (int)items.size(), 0, s);
        (void)hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (rep > 0 && ms < *best_ms) *best_ms = ms;  // the first launch warms up
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
}

}  // namespace

namespace sp2 {

// The plan behind sp2_plan_create and the learned expansion's inference:
// n_layers < 0 is plain SP2; otherwise coef (3 per layer) are the trained
// layers, followed by the check step (bar idem_fallback) and plain SP2 steps
// up to max_iter steps in all.
int plan_create_impl(sp2_plan** plan, int batch, const int* n, const int* n_occ, sp2_dtype dtype,
                     sp2_compute compute, double tol, int max_iter, const char* autotune_cache,
                     const double* coef, int n_layers, double idem_fallback, int mu_mode) {
    if (!plan) return SP2_E_INVALID;
    *plan = nullptr;
    if (batch <= 0 || batch > SP2_PLAN_MAX_BATCH || !n || (!n_occ && !mu_mode)) return SP2_E_INVALID;
    if (mu_mode && n_layers >= 0) return SP2_E_INVALID;
    if (dtype != SP2_F64 && dtype != SP2_F32) return SP2_E_INVALID;
    if (!(tol > 0.0) || !(tol < 1e300) || max_iter < 0 || max_iter > SP2_MAX_ITER) return SP2_E_INVALID;
    if (n_layers >= 0 && (n_layers + 1 > max_iter || (n_layers > 0 && !coef) || !(idem_fallback > 0.0)))
        return SP2_E_INVALID;
    if (compute < SP2_C_F64 || compute > SP2_C_FP8) return SP2_E_INVALID;
    if (compute != SP2_C_F64) return SP2_E_UNSUPPORTED;
    for (int b = 0; b < batch; ++b)
        if (n[b] <= 0 || n[b] > SP2_PLAN_MAX_N || (!mu_mode && (n_occ[b] < 0 || n_occ[b] > n[b])))
            return SP2_E_INVALID;

    sp2_plan* p = new (std::nothrow) sp2_plan;
    if (!p) return SP2_E_HIP;
    p->batch = batch;
    p->dtype = dtype;
    p->compute = compute;
    p->tol = tol;
    p->max_iter = max_iter;
    p->n_layers = n_layers;
    p->idem_fallback = idem_fallback;
    p->mu_mode = mu_mode;
    p->n.assign(n, n + batch);
    if (hipGetDevice(&p->device) != hipSuccess) {
        plan_free(p);
        return SP2_E_HIP;
    }
    // plan order: larger matrices first (LPT by n^3; ties keep the caller order)
    p->order.resize(batch);
    for (int b = 0; b < batch; ++b) p->order[b] = b;
    std::stable_sort(p->order.begin(), p->order.end(), [&](int a, int c) { return n[a] > n[c]; });

    std::vector<int> ldp(batch);
    for (int k = 0; k < batch; ++k) ldp[k] = (int)align_up((size_t)n[p->order[k]], (size_t)kBndTile);
    // device layout: mats | infos | items (largest candidate) | states | parts | X0/X1 per matrix
    size_t max_items = 0;
    std::vector<std::vector<int2>> cand(kNumCfg);
    for (int c = 0; c < kNumCfg; ++c) {
        cand[c] = build_items(ldp, kCfgBT[c]);
        max_items = std::max(max_items, cand[c].size());
    }
    size_t off = 0;
    const size_t off_mats = off;  off = up256(off + batch * sizeof(BatchMat));
    const size_t off_infos = off; off = up256(off + batch * sizeof(sp2_info));
    const size_t off_items = off; off = up256(off + max_items * sizeof(int2));
    const size_t off_tune = off;  off = up256(off + max_items * sizeof(int2));
    // the bounds / X_0 pair items and the finalize row-block items, plan order
    std::vector<int2> pairs, rows;
    for (int k = 0; k < batch; ++k) {
        const int nb = ldp[k] / kBndTile;
        for (int q = 0; q < nb * (nb + 1) / 2; ++q) pairs.push_back(make_int2(k, q));
        const int nk = n[p->order[k]];
        for (int q = 0; q < (nk + kFinRows - 1) / kFinRows; ++q) rows.push_back(make_int2(k, q));
    }
    const size_t off_pairs = off; off = up256(off + pairs.size() * sizeof(int2));
    const size_t off_rows = off;  off = up256(off + rows.size() * sizeof(int2));
    const size_t off_st = off;    off = up256(off + batch * up256(sizeof(State)));
    const size_t off_coef = off;  off = up256(off + (size_t)3 * (n_layers > 0 ? n_layers : 1) * sizeof(double));
    std::vector<size_t> off_part(batch), off_x(batch), off_rp(batch);
    for (int k = 0; k < batch; ++k) {
        const int T32 = ldp[k] / 32;                 // the finest candidate tiling
        off_part[k] = off;
        off = up256(off + (size_t)4 * T32 * (T32 + 1) / 2 * sizeof(double));
        off_rp[k] = off;
        off = up256(off + (size_t)(ldp[k] / kBndTile) * ldp[k] * sizeof(double));
    }
    const int nbuf = n_layers >= 0 ? 3 : 2;   // learned plans keep X_0 too
    for (int k = 0; k < batch; ++k) {
        off_x[k] = off;
        off = up256(off + nbuf * (size_t)ldp[k] * ldp[k] * sizeof(double));
    }
    if (hipMalloc(&p->dmem, off) != hipSuccess ||
        hipHostMalloc((void**)&p->h_mats, batch * sizeof(BatchMat), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&p->h_infos, batch * sizeof(sp2_info), hipHostMallocDefault) != hipSuccess) {
        plan_free(p);
        return SP2_E_HIP;
    }
    char* base = (char*)p->dmem;
    p->d_mats = (BatchMat*)(base + off_mats);
    p->d_infos = (sp2_info*)(base + off_infos);
    p->d_items = (int2*)(base + off_items);
    int2* d_tune = (int2*)(base + off_tune);
    p->d_pairs = (int2*)(base + off_pairs);
    p->npairs = (int)pairs.size();
    p->d_rows = (int2*)(base + off_rows);
    p->nrows = (int)rows.size();
    p->d_coef = (double*)(base + off_coef);
    for (int k = 0; k < batch; ++k) {
        BatchMat& m = p->h_mats[k];
        m.H = nullptr;
        m.D = nullptr;
        m.st = (State*)(base + off_st + k * up256(sizeof(State)));
        m.part = (double*)(base + off_part[k]);
        m.rowpart = (double*)(base + off_rp[k]);
        m.x0 = (double*)(base + off_x[k]);
        m.x1 = m.x0 + (size_t)ldp[k] * ldp[k];
        m.xk = n_layers >= 0 ? m.x1 + (size_t)ldp[k] * ldp[k] : nullptr;
        m.n = n[p->order[k]];
        m.ldp = ldp[k];
        m.n_occ = mu_mode ? 0 : n_occ[p->order[k]];
        m.mu_mode = mu_mode;
        m.mu = 0.0;
    }
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = prepare_cfg<BCfg64>();
    if (e == hipSuccess) e = prepare_cfg<BCfg32>();
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_mats, p->h_mats, batch * sizeof(BatchMat),
                                            hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->d_rows, rows.data(), rows.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n_layers > 0)
        e = hipMemcpy(p->d_coef, coef, (size_t)3 * n_layers * sizeof(double), hipMemcpyHostToDevice);
    // zero iterates: the padding of X stays zero (x^2 and 2x - x^2 keep it)
    if (e == hipSuccess) e = hipMemsetAsync(base + off_x[0], 0, off - off_x[0], s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);

    // tile shape: cached, autotuned, or the single-matrix shape
    int cfg = 0;
    if (e == hipSuccess && autotune_cache) {
        const std::string key = autotune_key(p->n, compute);
        cfg = cache_lookup(autotune_cache, key);
        if (cfg < 0) {
            float best = 1e30f;
            cfg = 0;
            for (int c = 0; c < kNumCfg && e == hipSuccess; ++c) {
                float ms = 0.f;
                e = time_cfg(p, cand[c], d_tune, c, s, &ms);
                if (e == hipSuccess && ms < best) {
                    best = ms;
                    cfg = c;
                }
            }
            // the timing runs leave X_1 = 0 and the states dirty; a run resets both
            if (e == hipSuccess) cache_store(autotune_cache, key, cfg);
        }
    }
    p->cfg = cfg;
    std::snprintf(p->cfg_name, sizeof(p->cfg_name), "%s", kCfgName[cfg]);
    p->nblocks = (int)cand[cfg].size();
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_items, cand[cfg].data(), cand[cfg].size() * sizeof(int2),
                                            hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // capture the whole solve
    if (e == hipSuccess) e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = enqueue_solve(p, s);
        e = hipStreamEndCapture(s, &p->graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (s) (void)hipStreamDestroy(s);
    if (e != hipSuccess) {
        plan_free(p);
        return SP2_E_HIP;
    }
    *plan = p;
    return SP2_OK;
}

}  // namespace sp2

extern "C" {

int sp2_plan_create(sp2_plan** plan, int batch, const int* n, const int* n_occ, sp2_dtype dtype,
                    sp2_compute compute, double tol, int max_iter, const char* autotune_cache) {
    return sp2::plan_create_impl(plan, batch, n, n_occ, dtype, compute, tol, max_iter, autotune_cache,
                                 nullptr, -1, 0.0, 0);
}

int sp2_plan_run(sp2_plan* p, const void* const* H, void* const* D, void* hip_stream, sp2_info* infos) {
    return sp2::plan_run_impl(p, H, D, nullptr, hip_stream, infos);
}

const char* sp2_plan_config(const sp2_plan* p) { return p ? p->cfg_name : ""; }

int sp2_plan_destroy(sp2_plan* p) {
    if (!p) return SP2_E_INVALID;
    plan_free(p);
    return SP2_OK;
}

}  // extern "C"

namespace sp2 {

// One solve of every matrix of the plan.  mu (caller order) sets the chemical
// potential of each matrix of a plan made with mu_mode; it must be null
// otherwise.
int plan_run_impl(sp2_plan* p, const void* const* H, void* const* D, const double* mu, void* hip_stream,
                  sp2_info* infos) {
    if (!p || !H || !D) return SP2_E_INVALID;
    if ((mu != nullptr) != (p->mu_mode != 0)) return SP2_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SP2_E_HIP;
    if (dev != p->device) return SP2_E_INVALID;
    const size_t esz = p->dtype == SP2_F64 ? sizeof(double) : sizeof(float);
    for (int k = 0; k < p->batch; ++k) {
        const int b = p->order[k];
        if (!H[b] || !D[b]) return SP2_E_INVALID;
        const size_t bytes = (size_t)p->n[b] * p->n[b] * esz;
        const char* h = (const char*)H[b];
        const char* d = (const char*)D[b];
        if (h < d + bytes && d < h + bytes) return SP2_E_INVALID;
        if (mu && !std::isfinite(mu[b])) return SP2_E_INVALID;
        p->h_mats[k].H = H[b];
        p->h_mats[k].D = D[b];
        p->h_mats[k].mu = mu ? mu[b] : 0.0;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (hipMemcpyAsync(p->d_mats, p->h_mats, p->batch * sizeof(BatchMat), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipGraphLaunch(p->exec, s) != hipSuccess ||
        hipMemcpyAsync(p->h_infos, p->d_infos, p->batch * sizeof(sp2_info), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SP2_E_HIP;
    // the call's status: the most negative per-matrix status if any is
    // negative, else the largest (OK < NOT_CONVERGED < STAGNATED)
    int neg = 0, pos = SP2_OK;
    for (int k = 0; k < p->batch; ++k) {
        const sp2_info& r = p->h_infos[k];
        if (infos) infos[p->order[k]] = r;
        if (r.status < neg) neg = r.status;
        if (r.status > pos) pos = r.status;
    }
    return neg < 0 ? neg : pos;
}

}  // namespace sp2
