// sp2_graph.hip -- the graph-partitioned solver of the paper's Section
// "Graph-based Divide electronic structure" on one GPU: the thresholded
// adjacency of an auxiliary matrix G (the section's adjacency equation), core
// parts as regular segments of the index list, one-hop core-halo parts, the
// dense sub-matrix of H on every part solved by the batched plan, and the
// rows of each part's core nodes mapped back into D (the general solver
// routine listing: graph, partition, extract, solve, map back).
//
// Every part is solved at one chemical potential mu: its SP2 steps are
// steered by mu's image under the maps applied (State::mu_mode), so each
// part converges to the projector on its eigenvalues below mu, the
// zero-temperature Fermi-Dirac function the section applies part by part.
//
// Kernels:
//   k_graph_mask     membership bytes: part k x node j, from rows of G (reads
//                    G once, coalesced along j);
//   k_graph_compact  one workgroup per part: ascending node list, inverse map
//                    (position or -1), size and first core position;
//   k_graph_gather   the parts' sub-matrices of H into contiguous FP64
//                    buffers, one workgroup per gathered row;
//   k_graph_scatter  one workgroup per row of D: row i of the part whose core
//                    holds i, spread over the part's nodes, 0 elsewhere (no
//                    separate clearing pass).
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "sp2_internal.h"

namespace sp2 {

constexpr int kGraphThreads = 256;
constexpr int kCompactThreads = 1024;
constexpr int kGraphMaxN = 65536;
constexpr int kGraphMaxParts = 4096;

template <typename T>
__global__ __launch_bounds__(kGraphThreads) void k_graph_mask(const T* __restrict__ G, int n, int ld,
                                                              double tau, const int* __restrict__ seg,
                                                              unsigned char* __restrict__ mask) {
    const int k = blockIdx.y;
    const int j = blockIdx.x * kGraphThreads + threadIdx.x;
    if (j >= n) return;
    const int c0 = seg[k], c1 = seg[k + 1];
    int in = (j >= c0 && j < c1) ? 1 : 0;
    for (int l = c0; l < c1 && !in; ++l)
        in = (l != j && fabs((double)G[(size_t)l * ld + j]) >= tau) ? 1 : 0;
    mask[(size_t)k * n + j] = (unsigned char)in;
}

// meta[2k] = size of part k, meta[2k + 1] = position of its first core node.
__global__ __launch_bounds__(kCompactThreads) void k_graph_compact(const unsigned char* __restrict__ mask,
                                                                   int n, const int* __restrict__ seg,
                                                                   int* __restrict__ idx, int* __restrict__ inv,
                                                                   int* __restrict__ meta) {
    constexpr int NW = kCompactThreads / 64;
    __shared__ int wsum[NW];
    __shared__ int base_s, cpos_s;
    const int k = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const unsigned char* mk = mask + (size_t)k * n;
    const int first = seg[k];
    if (tid == 0) {
        base_s = 0;
        cpos_s = 0;
    }
    __syncthreads();
    for (int c = 0; c < n; c += kCompactThreads) {
        const int j = c + tid;
        const int f = (j < n) ? (int)mk[j] : 0;
        const unsigned long long b = __ballot(f);
        const int below = __popcll(b & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __popcll(b);
        __syncthreads();
        int off = base_s;
        for (int q = 0; q < w; ++q) off += wsum[q];
        if (j < n) {
            const int pos = f ? off + below : -1;
            if (f) idx[(size_t)k * n + pos] = j;
            inv[(size_t)k * n + j] = pos;
            if (j == first) cpos_s = pos;
        }
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            for (int q = 0; q < NW; ++q) t += wsum[q];
            base_s += t;
        }
        __syncthreads();
    }
    if (tid == 0) {
        meta[2 * k] = base_s;
        meta[2 * k + 1] = cpos_s;
    }
}

struct GatherRow {
    int part, row;
};

template <typename T>
__global__ __launch_bounds__(kGraphThreads) void k_graph_gather(const T* __restrict__ H, int ld, int n,
                                                                const int* __restrict__ idx,
                                                                const GatherRow* __restrict__ rows,
                                                                const int* __restrict__ size,
                                                                const size_t* __restrict__ off,
                                                                double* __restrict__ hbuf) {
    const GatherRow r = rows[blockIdx.x];
    const int s = size[r.part];
    const int* nodes = idx + (size_t)r.part * n;
    const T* src = H + (size_t)nodes[r.row] * ld;
    double* dst = hbuf + off[r.part] + (size_t)r.row * s;
    for (int b = threadIdx.x; b < s; b += kGraphThreads) dst[b] = (double)src[nodes[b]];
}

template <typename T>
__global__ __launch_bounds__(kGraphThreads) void k_graph_scatter(T* __restrict__ D, int ld, int n,
                                                                 const int* __restrict__ seg,
                                                                 const int* __restrict__ part_of,
                                                                 const int* __restrict__ inv,
                                                                 const int* __restrict__ meta,
                                                                 const size_t* __restrict__ off,
                                                                 const double* __restrict__ dbuf) {
    const int i = blockIdx.x;
    const int k = part_of[i];
    const int s = meta[2 * k];
    const int a = meta[2 * k + 1] + (i - seg[k]);
    const double* src = dbuf + off[k] + (size_t)a * s;
    const int* pk = inv + (size_t)k * n;
    T* dst = D + (size_t)i * ld;
    for (int j = threadIdx.x; j < n; j += kGraphThreads) {
        const int p = pk[j];
        dst[j] = (T)(p >= 0 ? src[p] : 0.0);
    }
}

}  // namespace sp2

struct sp2_graph {
    int n = 0, parts = 0, device = 0;
    std::vector<int> seg;          // parts + 1 segment starts
    std::vector<int> size;         // nodes per part
    std::vector<int> cpos;         // position of the first core node in each list
    std::vector<size_t> off;       // FP64 offset of each part's sub-matrix
    std::vector<const void*> hp;   // the plan's inputs and outputs
    std::vector<void*> dp;
    std::vector<double> mu;
    void* dmem = nullptr;          // seg | part_of | meta | off | idx | inv | mask | rows
    void* dbuf_mem = nullptr;      // sub-matrices of H and their density matrices
    int* d_seg = nullptr;
    int* d_part_of = nullptr;
    int* d_meta = nullptr;
    int* d_size = nullptr;
    size_t* d_off = nullptr;
    int* d_idx = nullptr;
    int* d_inv = nullptr;
    unsigned char* d_mask = nullptr;
    sp2::GatherRow* d_rows = nullptr;
    int nrows = 0;
    double* d_h = nullptr;
    double* d_d = nullptr;
    sp2_plan* plan = nullptr;
};

namespace {

void graph_free(sp2_graph* g) {
    if (!g) return;
    if (g->plan) (void)sp2_plan_destroy(g->plan);
    if (g->dbuf_mem) (void)hipFree(g->dbuf_mem);
    if (g->dmem) (void)hipFree(g->dmem);
    delete g;
}

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

extern "C" {

int sp2_graph_create(sp2_graph** graph, const void* G, int n, int ld, sp2_dtype dtype, double tau, int parts,
                     double tol, int max_iter, void* hip_stream) {
    using namespace sp2;
    if (!graph) return SP2_E_INVALID;
    *graph = nullptr;
    if (!G || n <= 0 || n > kGraphMaxN || ld < n || parts < 1 || parts > n || parts > kGraphMaxParts ||
        !(tau >= 0.0) || !std::isfinite(tau) || (dtype != SP2_F64 && dtype != SP2_F32))
        return SP2_E_INVALID;
    if (!(tol > 0.0) || !(tol < 1e300) || max_iter < 0 || max_iter > SP2_MAX_ITER) return SP2_E_INVALID;
    sp2_graph* g = new (std::nothrow) sp2_graph;
    if (!g) return SP2_E_HIP;
    g->n = n;
    g->parts = parts;
    if (hipGetDevice(&g->device) != hipSuccess) {
        graph_free(g);
        return SP2_E_HIP;
    }
    g->seg.resize(parts + 1);
    for (int k = 0; k <= parts; ++k) g->seg[k] = (int)(((long long)k * n) / parts);
    std::vector<int> part_of(n);
    for (int k = 0; k < parts; ++k)
        for (int i = g->seg[k]; i < g->seg[k + 1]; ++i) part_of[i] = k;

    const size_t pn = (size_t)parts * n;
    size_t o = 0;
    const size_t o_seg = o;   o = up256(o + (parts + 1) * sizeof(int));
    const size_t o_pof = o;   o = up256(o + n * sizeof(int));
    const size_t o_meta = o;  o = up256(o + 2 * (size_t)parts * sizeof(int));
    const size_t o_size = o;  o = up256(o + (size_t)parts * sizeof(int));
    const size_t o_off = o;   o = up256(o + (size_t)parts * sizeof(size_t));
    const size_t o_idx = o;   o = up256(o + pn * sizeof(int));
    const size_t o_inv = o;   o = up256(o + pn * sizeof(int));
    const size_t o_mask = o;  o = up256(o + pn);
    const size_t o_rows = o;  o = up256(o + (size_t)parts * SP2_PLAN_MAX_N * sizeof(GatherRow));
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMalloc(&g->dmem, o);
    if (e != hipSuccess) {
        graph_free(g);
        return SP2_E_HIP;
    }
    char* base = (char*)g->dmem;
    g->d_seg = (int*)(base + o_seg);
    g->d_part_of = (int*)(base + o_pof);
    g->d_meta = (int*)(base + o_meta);
    g->d_size = (int*)(base + o_size);
    g->d_off = (size_t*)(base + o_off);
    g->d_idx = (int*)(base + o_idx);
    g->d_inv = (int*)(base + o_inv);
    g->d_mask = (unsigned char*)(base + o_mask);
    g->d_rows = (GatherRow*)(base + o_rows);
    std::vector<int> meta(2 * (size_t)parts);
    e = hipMemcpyAsync(g->d_seg, g->seg.data(), (parts + 1) * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_part_of, part_of.data(), n * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        const dim3 grid((n + kGraphThreads - 1) / kGraphThreads, parts);
        if (dtype == SP2_F64)
            hipLaunchKernelGGL(k_graph_mask<double>, grid, dim3(kGraphThreads), 0, s, (const double*)G, n, ld, tau,
                               g->d_seg, g->d_mask);
        else
            hipLaunchKernelGGL(k_graph_mask<float>, grid, dim3(kGraphThreads), 0, s, (const float*)G, n, ld, tau,
                               g->d_seg, g->d_mask);
        hipLaunchKernelGGL(k_graph_compact, dim3(parts), dim3(kCompactThreads), 0, s, g->d_mask, n, g->d_seg,
                           g->d_idx, g->d_inv, g->d_meta);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(meta.data(), g->d_meta, meta.size() * sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        graph_free(g);
        return SP2_E_HIP;
    }
    g->size.resize(parts);
    g->cpos.resize(parts);
    g->off.resize(parts);
    size_t total = 0;
    int too_big = 0;
    for (int k = 0; k < parts; ++k) {
        g->size[k] = meta[2 * k];
        g->cpos[k] = meta[2 * k + 1];
        if (g->size[k] > SP2_PLAN_MAX_N) too_big = 1;
        g->off[k] = total;
        total += (size_t)g->size[k] * g->size[k];
    }
    if (too_big) {   // a part beyond the batched plan's size limit
        graph_free(g);
        return SP2_E_UNSUPPORTED;
    }
    std::vector<GatherRow> rows;
    rows.reserve(total / 64 + parts);
    for (int k = 0; k < parts; ++k)
        for (int a = 0; a < g->size[k]; ++a) rows.push_back(GatherRow{k, a});
    g->nrows = (int)rows.size();
    e = hipMalloc(&g->dbuf_mem, 2 * up256(total * sizeof(double)));
    if (e == hipSuccess) {
        g->d_h = (double*)g->dbuf_mem;
        g->d_d = (double*)((char*)g->dbuf_mem + up256(total * sizeof(double)));
        e = hipMemcpyAsync(g->d_rows, rows.data(), rows.size() * sizeof(GatherRow), hipMemcpyHostToDevice, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_size, g->size.data(), parts * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_off, g->off.data(), parts * sizeof(size_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        graph_free(g);
        return SP2_E_HIP;
    }
    const int st = plan_create_impl(&g->plan, parts, g->size.data(), nullptr, SP2_F64, SP2_C_F64, tol, max_iter,
                                    nullptr, nullptr, -1, 0.0, 1);
    if (st != SP2_OK) {
        graph_free(g);
        return st;
    }
    g->hp.resize(parts);
    g->dp.resize(parts);
    g->mu.resize(parts);
    for (int k = 0; k < parts; ++k) {
        g->hp[k] = g->d_h + g->off[k];
        g->dp[k] = g->d_d + g->off[k];
    }
    *graph = g;
    return SP2_OK;
}

int sp2_graph_parts(const sp2_graph* g, int* sizes, int* core_sizes) {
    if (!g) return SP2_E_INVALID;
    for (int k = 0; k < g->parts; ++k) {
        if (sizes) sizes[k] = g->size[k];
        if (core_sizes) core_sizes[k] = g->seg[k + 1] - g->seg[k];
    }
    return g->parts;
}

int sp2_graph_nodes(const sp2_graph* g, int part, int* nodes, int capacity) {
    if (!g || part < 0 || part >= g->parts) return SP2_E_INVALID;
    const int s = g->size[part];
    if (!nodes || capacity < s) return s;
    if (hipMemcpy(nodes, g->d_idx + (size_t)part * g->n, s * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return SP2_E_HIP;
    return s;
}

int sp2_graph_density(sp2_graph* g, const void* H, void* D, int ld, sp2_dtype dtype, double mu,
                      void* hip_stream, sp2_info* infos) {
    using namespace sp2;
    if (!g || !H || !D || ld < g->n || (dtype != SP2_F64 && dtype != SP2_F32) || !std::isfinite(mu))
        return SP2_E_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SP2_E_HIP;
    if (dev != g->device) return SP2_E_INVALID;
    const size_t esz = dtype == SP2_F64 ? sizeof(double) : sizeof(float);
    const size_t bytes = ((size_t)(g->n - 1) * ld + g->n) * esz;
    const char* h = (const char*)H;
    const char* d = (const char*)D;
    if (h < d + bytes && d < h + bytes) return SP2_E_INVALID;
    hipStream_t s = (hipStream_t)hip_stream;
    if (dtype == SP2_F64)
        hipLaunchKernelGGL(k_graph_gather<double>, dim3(g->nrows), dim3(kGraphThreads), 0, s, (const double*)H, ld,
                           g->n, g->d_idx, g->d_rows, g->d_size, g->d_off, g->d_h);
    else
        hipLaunchKernelGGL(k_graph_gather<float>, dim3(g->nrows), dim3(kGraphThreads), 0, s, (const float*)H, ld,
                           g->n, g->d_idx, g->d_rows, g->d_size, g->d_off, g->d_h);
    if (hipGetLastError() != hipSuccess) return SP2_E_HIP;
    std::fill(g->mu.begin(), g->mu.end(), mu);
    const int st = plan_run_impl(g->plan, g->hp.data(), g->dp.data(), g->mu.data(), hip_stream, infos);
    if (st == SP2_E_HIP || st == SP2_E_INVALID) return st;
    if (dtype == SP2_F64)
        hipLaunchKernelGGL(k_graph_scatter<double>, dim3(g->n), dim3(kGraphThreads), 0, s, (double*)D, ld, g->n,
                           g->d_seg, g->d_part_of, g->d_inv, g->d_meta, g->d_off, g->d_d);
    else
        hipLaunchKernelGGL(k_graph_scatter<float>, dim3(g->n), dim3(kGraphThreads), 0, s, (float*)D, ld, g->n,
                           g->d_seg, g->d_part_of, g->d_inv, g->d_meta, g->d_off, g->d_d);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) return SP2_E_HIP;
    return st;
}

int sp2_graph_destroy(sp2_graph* g) {
    if (!g) return SP2_E_INVALID;
    graph_free(g);
    return SP2_OK;
}

}  // extern "C"
