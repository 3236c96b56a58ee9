// sp2_cheb.hip -- the Chebyshev expansion of the Fermi operator (Section
// "Chebyshev polynomial expansion"): D = sum_{n < k m} c_n T_n(Hs), Hs the
// symmetric part of H scaled into [-1, 1] by its Gershgorin interval, c_n the
// Chebyshev coefficients of the Fermi-Dirac function at inverse temperature
// beta and chemical potential mu.  Evaluated in the Paterson-Stockmeyer form
// of the section's ansatz,
//   sum_n c_n T_n = S_0 + T_k (S_1 + T_k (S_2 + ... + T_k S_{m-1})),
//   S_j = sum_{i<k} d_{i,j} T_i,
// with T_2..T_k built level by level from the product identity
// T_a T_b = (T_{a+b} + T_{|a-b|})/2 (the section's T_2 = 2 T_1 T_1 - T_0,
// T_3 = 2 T_2 T_1 - T_1, T_4 = 2 T_2 T_2 - T_0, ...): every product of one
// level is independent of the others, so a level is one grouped launch (the
// concurrency the section obtains with several streams).  Then m - 1 Horner
// products, each fusing the sum S_j into its epilogue.  Matrix products:
// k - 1 + m - 1 for k m terms.
//
// All T_i are polynomials of Hs, so every product of two of them is symmetric:
// the product kernel computes the lower tiles only (64 x 64, 4 waves of
// v_mfma_f64_16x16x4f64, the register-staged LDS main loop of the SP2 step)
// and writes each tile and its mirror.
//
// Host side: c_n by the Chebyshev-Gauss rule with 4 k m nodes, and d_{i,j} by
// repeated division by T_k in the Chebyshev basis (T_t = 2 T_k T_{t-k} -
// T_{|2k-t|} moves the coefficient of T_t >= T_k into the quotient).
#include <cmath>
#include <cstring>
#include <vector>

#include "bounds_core.h"
#include "syrk_f64_core.h"

namespace sp2 {

constexpr int kChebMaxK = 64;   // terms of one S_j (the Horner epilogue reads all of them)

// One product C = al * A B + sum_t w[t] Z[t] + ga I (A, B, Z symmetric and
// commuting), or with al = 0 just the combination.
struct ChebProd {
    const double* A;
    const double* B;
    double* C;
    double al, ga;
    int nz, pad;
    const double* Z[kChebMaxK];
    double w[kChebMaxK];
};

using ChebCfg = SyrkCfg<64, 2, 2>;

// T_1 = (Hs - a I)/b for one tile pair (H read once, T_1 bitwise symmetric).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cheb_t1(const T* __restrict__ H, int n, int ld, int ldp,
                                                      const State* st, double* __restrict__ T1) {
    __shared__ double sA[kBndTile][kBndTile + 1];
    __shared__ double sB[kBndTile][kBndTile + 1];
    int I, J;
    tri_tile(blockIdx.x, I, J);
    const double a = (st->emax + st->emin) / 2.0, b = (st->emax - st->emin) / 2.0;
    int bad = 0;
    load_pair(H, n, ld, I, J, sA, sB, bad);
    __syncthreads();
    double xv[kBndTile * kBndTile / kThreads];
    int k = 0;
    for (int e = threadIdx.x; e < kBndTile * kBndTile; e += kThreads, ++k) {
        const int rr = e >> 6, cc = e & 63;
        const int gi = I * kBndTile + rr, gj = J * kBndTile + cc;
        double x = 0.0;
        if (gi < n && gj < n) {
            const double hs = (sA[rr][cc] + sB[cc][rr]) / 2.0;
            x = ((gi == gj) ? hs - a : hs) / b;
        }
        xv[k] = x;
        T1[(size_t)gi * ldp + gj] = x;
    }
    if (I != J) {
        __syncthreads();
        k = 0;
        for (int e = threadIdx.x; e < kBndTile * kBndTile; e += kThreads, ++k) sA[e >> 6][e & 63] = xv[k];
        __syncthreads();
        for (int e = threadIdx.x; e < kBndTile * kBndTile; e += kThreads) {
            const int rr = e >> 6, cc = e & 63;
            T1[(size_t)(J * kBndTile + rr) * ldp + I * kBndTile + cc] = sA[cc][rr];
        }
    }
}

// Grouped products: items[b] = (product, lower tile).  Zero padding stays
// zero (every term is zero there and ga multiplies the identity only inside
// n x n).
__global__ __launch_bounds__(ChebCfg::NT) void k_cheb_prod(const ChebProd* __restrict__ prods,
                                                           const int2* __restrict__ items, int n, int ldp) {
    using C = ChebCfg;
    __shared__ double smem[2 * 2 * C::BT * kLDK];
    const int2 it = items[blockIdx.x];
    const ChebProd& P = prods[it.x];
    int ti, tj;
    tri_tile((unsigned)it.y, ti, tj);
    d4 acc[C::MI][C::NI];
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) acc[mi][ni] = d4{0.0, 0.0, 0.0, 0.0};
    const int KT = ldp / kBK;
    if (P.al != 0.0) {
        double* sA = smem;
        double* sB = smem + 2 * C::BT * kLDK;
        if (P.A == P.B && ti == tj) syrk_mainloop2<C, true>(P.A, P.B, ldp, ti, tj, 0, KT, sA, sB, acc);
        else syrk_mainloop2<C, false>(P.A, P.B, ldp, ti, tj, 0, KT, sA, sB, acc);
    }
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w / C::WN, wn = w % C::WN;
    const bool diag = (ti == tj);
#pragma unroll
    for (int mi = 0; mi < C::MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < C::NI; ++ni) {
            const int gi0 = ti * C::BT + wm * C::WTM + mi * 16 + (lane >> 4);
            const int gj = tj * C::BT + wn * C::WTN + ni * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = gi0 + 4 * r;
                if (diag && gi < gj) continue;
                const size_t idx = (size_t)gi * ldp + gj;
                double v = P.al * acc[mi][ni][r];
                for (int t = 0; t < P.nz; ++t) v += P.w[t] * P.Z[t][idx];
                if (gi == gj && gi < n) v += P.ga;
                P.C[idx] = v;
                if (gi != gj) P.C[(size_t)gj * ldp + gi] = v;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
}

// D <- X (storage type of H) and the trace of X.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cheb_finalize(T* __restrict__ D, int n, int ld, int ldp,
                                                            const double* __restrict__ X, double* __restrict__ diag) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += kThreads) D[(size_t)i * ld + j] = (T)X[(size_t)i * ldp + j];
    if (threadIdx.x == 0) diag[i] = X[(size_t)i * ldp + i];
}

__global__ __launch_bounds__(kThreads) void k_cheb_trace(const double* __restrict__ diag, int n, State* st) {
    __shared__ double red[4];
    double t = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) t += diag[i];
    t = block_sum(t, red);
    if (threadIdx.x == 0) {
        st->tr = t;
        st->status = st->bad ? SP2_E_INVALID : SP2_OK;
        st->done = 1;
    }
}

// ---------------------------------------------------------------- host side

struct ChebLayout {
    int ldp, k;
    size_t off_state, off_part, off_rowpart, off_diag, off_prods, off_items, off_T, off_P, total;
    int max_prods, max_items;
};

inline ChebLayout cheb_layout(int n, int k) {
    ChebLayout L{};
    L.ldp = (int)align_up((size_t)n, 64);
    L.k = k;
    const int T = L.ldp / 64, nb = L.ldp / kBndTile;
    const int tiles = T * (T + 1) / 2;
    L.max_prods = 2 * k + 4;      // every product of every launch (k - 1 for T, m for Horner; m <= k + 4)
    L.max_items = L.max_prods * tiles;
    size_t off = 0;
    L.off_state = off;   off = align_up(off + sizeof(State), 256);
    L.off_part = off;    off = align_up(off + (size_t)nb * nb * 4 * sizeof(double), 256);
    L.off_rowpart = off; off = align_up(off + ((size_t)nb * L.ldp + 2 * (size_t)L.ldp) * sizeof(double), 256);
    L.off_diag = off;    off = align_up(off + (size_t)L.ldp * sizeof(double), 256);
    L.off_prods = off;   off = align_up(off + (size_t)L.max_prods * sizeof(ChebProd), 256);
    L.off_items = off;   off = align_up(off + (size_t)L.max_items * sizeof(int2), 256);
    L.off_T = off;       off = align_up(off + (size_t)k * L.ldp * L.ldp * sizeof(double), 256);   // T_1..T_k
    L.off_P = off;       off = align_up(off + 2 * (size_t)L.ldp * L.ldp * sizeof(double), 256);
    L.total = off;
    return L;
}

// c_0..c_{N-1} of 1/(1 + exp(bs (x - ms))) on [-1, 1], Chebyshev-Gauss rule.
static void gauss_coeffs(int N, double bs, double ms, std::vector<double>& c) {
    const int q = 4 * N;
    const double pi = 3.14159265358979323846;
    std::vector<double> f(q), th(q);
    for (int j = 0; j < q; ++j) {
        th[j] = pi * (j + 0.5) / q;
        const double t = bs * (std::cos(th[j]) - ms);
        f[j] = t > 0.0 ? std::exp(-t) / (1.0 + std::exp(-t)) : 1.0 / (1.0 + std::exp(t));
    }
    c.assign(N, 0.0);
    for (int nn = 0; nn < N; ++nn) {
        double s = 0.0;
        for (int j = 0; j < q; ++j) s += f[j] * std::cos(nn * th[j]);
        c[nn] = (nn == 0 ? 1.0 : 2.0) * s / q;
    }
}

// d[j][i] of the Paterson-Stockmeyer form (division by T_k, highest degree first).
static void ps_split(const std::vector<double>& c, int k, int m, std::vector<double>& d) {
    std::vector<double> a(c), q(c.size());
    d.assign((size_t)k * m, 0.0);
    int top = k * m - 1;
    for (int j = 0; j < m; ++j) {
        std::fill(q.begin(), q.end(), 0.0);
        for (int t = top; t >= k; --t) {
            const double v = a[t];
            a[t] = 0.0;
            if (t == k) {
                q[0] += v;
            } else {
                q[t - k] += 2.0 * v;
                a[std::abs(2 * k - t)] -= v;
            }
        }
        for (int i = 0; i < k && i <= top; ++i) d[(size_t)j * k + i] = a[i];
        top -= k;
        a = q;
    }
}

}  // namespace sp2

extern "C" {

size_t sp2_cheb_workspace_size(int n, int k) {
    if (n <= 0 || n > 32768 || k < 1 || k > sp2::kChebMaxK) return 0;
    return sp2::cheb_layout(n, k).total;
}

int sp2_cheb_density(const void* H, void* D, int n, int ld, sp2_dtype dtype, double mu, double beta, int k,
                     int m, void* workspace, size_t workspace_bytes, void* hip_stream, sp2_info* info) {
    using namespace sp2;
    if (info) *info = sp2_info{};
    auto fail = [&](int code) {
        if (info) info->status = code;
        return code;
    };
    if (!H || !D || n <= 0 || n > 32768 || ld < n || (dtype != SP2_F64 && dtype != SP2_F32)) return fail(SP2_E_INVALID);
    if (k < 1 || k > kChebMaxK || m < 1 || m > k + 4 || !(beta > 0.0) || !std::isfinite(beta) ||
        !std::isfinite(mu))
        return fail(SP2_E_INVALID);
    const ChebLayout L = cheb_layout(n, k);
    if (!workspace || workspace_bytes < L.total || (reinterpret_cast<uintptr_t>(workspace) % SP2_WORKSPACE_ALIGN))
        return fail(SP2_E_WORKSPACE);
    hipStream_t s = (hipStream_t)hip_stream;
    char* ws = (char*)workspace;
    State* st = (State*)(ws + L.off_state);
    double* part = (double*)(ws + L.off_part);
    double* rowpart = (double*)(ws + L.off_rowpart);
    double* diag = (double*)(ws + L.off_diag);
    ChebProd* d_prods = (ChebProd*)(ws + L.off_prods);
    int2* d_items = (int2*)(ws + L.off_items);
    auto Tm = [&](int i) { return (double*)(ws + L.off_T) + (size_t)(i - 1) * L.ldp * L.ldp; };   // T_1..T_k
    double* Pb[2] = {(double*)(ws + L.off_P), (double*)(ws + L.off_P) + (size_t)L.ldp * L.ldp};
    const int T = L.ldp / 64;
    const int tiles = T * (T + 1) / 2;

    // bounds (the SP2 kernels' tile-pair Gershgorin) and T_1
    Layout BL{};
    BL.n = n;
    BL.ldp = L.ldp;
    hipError_t e = launch_reset(st, n, 0, 1.0, 0, 0, nullptr, 0, s);
    if (e == hipSuccess) e = launch_bounds(H, dtype, n, ld, BL, st, rowpart, part, s);
    if (e != hipSuccess) return fail(SP2_E_HIP);
    // the bounds decide the scaling of mu and beta: read them back (one sync)
    State hst;
    if (hipMemcpyAsync(&hst, st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(SP2_E_HIP);
    if (hst.bad) return fail(SP2_E_INVALID);
    if (!(hst.emax > hst.emin)) return fail(SP2_E_DEGENERATE);
    const double a = (hst.emax + hst.emin) / 2.0, b = (hst.emax - hst.emin) / 2.0;
    const int npairs = (L.ldp / kBndTile) * (L.ldp / kBndTile + 1) / 2;
    if (dtype == SP2_F64)
        hipLaunchKernelGGL(k_cheb_t1<double>, dim3(npairs), dim3(kThreads), 0, s, (const double*)H, n, ld, L.ldp,
                           (const State*)st, Tm(1));
    else
        hipLaunchKernelGGL(k_cheb_t1<float>, dim3(npairs), dim3(kThreads), 0, s, (const float*)H, n, ld, L.ldp,
                           (const State*)st, Tm(1));

    std::vector<double> c, d;
    gauss_coeffs(k * m, beta * b, (mu - a) / b, c);
    ps_split(c, k, m, d);

    // host descriptors of every launch, copied into the workspace before each
    std::vector<std::vector<ChebProd>> launches;
    // T_t = 2 T_a T_b - T_{a-b}, a = ceil(t/2), b = floor(t/2), grouped by level
    std::vector<int> level(k + 1, 0);
    int nlev = 0;
    for (int t = 2; t <= k; ++t) {
        level[t] = level[(t + 1) / 2] + 1;
        nlev = level[t] > nlev ? level[t] : nlev;
    }
    for (int lv = 1; lv <= nlev; ++lv) {
        std::vector<ChebProd> ps;
        for (int t = 2; t <= k; ++t) {
            if (level[t] != lv) continue;
            const int ta = (t + 1) / 2, tb = t / 2;
            ChebProd p{};
            p.A = Tm(ta);
            p.B = Tm(tb);
            p.C = Tm(t);
            p.al = 2.0;
            if (ta == tb) {
                p.ga = -1.0;       // - T_0
            } else {
                p.nz = 1;
                p.Z[0] = Tm(1);    // - T_1
                p.w[0] = -1.0;
            }
            ps.push_back(p);
        }
        launches.push_back(ps);
    }
    // Horner: P = S_{m-1}; P <- S_j + T_k P for j = m-2 .. 0
    auto S_terms = [&](ChebProd& p, int j) {
        p.ga = d[(size_t)j * k + 0];     // d_{0,j} T_0
        p.nz = 0;
        for (int i = 1; i < k; ++i) {
            p.Z[p.nz] = Tm(i);
            p.w[p.nz] = d[(size_t)j * k + i];
            ++p.nz;
        }
    };
    int cur = 0;
    {
        ChebProd p{};
        p.al = 0.0;
        p.C = Pb[cur];
        S_terms(p, m - 1);
        launches.push_back({p});
    }
    for (int j = m - 2; j >= 0; --j) {
        ChebProd p{};
        p.A = Tm(k);
        p.B = Pb[cur];
        p.C = Pb[cur ^ 1];
        p.al = 1.0;
        S_terms(p, j);
        launches.push_back({p});
        cur ^= 1;
    }
    // every launch's descriptors and items go to their own slots in one copy,
    // then the launches run back to back
    std::vector<ChebProd> allp;
    std::vector<int2> alli;
    std::vector<int> p0(launches.size()), i0(launches.size()), icount(launches.size());
    for (size_t l = 0; l < launches.size(); ++l) {
        p0[l] = (int)allp.size();
        i0[l] = (int)alli.size();
        for (size_t q = 0; q < launches[l].size(); ++q) {
            allp.push_back(launches[l][q]);
            for (int t = 0; t < tiles; ++t) alli.push_back(make_int2((int)q, t));
        }
        icount[l] = (int)alli.size() - i0[l];
    }
    if ((int)allp.size() > L.max_prods || (int)alli.size() > L.max_items) return fail(SP2_E_INVALID);
    e = hipMemcpyAsync(d_prods, allp.data(), allp.size() * sizeof(ChebProd), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_items, alli.data(), alli.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail(SP2_E_HIP);
    for (size_t l = 0; l < launches.size(); ++l) {
        hipLaunchKernelGGL(k_cheb_prod, dim3((unsigned)icount[l]), dim3(ChebCfg::NT), 0, s, d_prods + p0[l],
                           d_items + i0[l], n, L.ldp);
        if ((e = hipGetLastError()) != hipSuccess) return fail(SP2_E_HIP);
    }
    if (dtype == SP2_F64)
        hipLaunchKernelGGL(k_cheb_finalize<double>, dim3(n), dim3(kThreads), 0, s, (double*)D, n, ld, L.ldp,
                           (const double*)Pb[cur], diag);
    else
        hipLaunchKernelGGL(k_cheb_finalize<float>, dim3(n), dim3(kThreads), 0, s, (float*)D, n, ld, L.ldp,
                           (const double*)Pb[cur], diag);
    hipLaunchKernelGGL(k_cheb_trace, dim3(1), dim3(kThreads), 0, s, (const double*)diag, n, st);
    if (hipMemcpyAsync(&hst, st, sizeof(State), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(SP2_E_HIP);
    if (info) {
        info->status = hst.status;
        info->iterations = (k - 1) + (m - 1);
        info->trace = hst.tr;
        info->emin = hst.emin;
        info->emax = hst.emax;
    }
    return hst.status;
}

}  // extern "C"
