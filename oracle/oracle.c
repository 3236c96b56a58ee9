/*
 * oracle.c -- plain, slow, obviously-correct FP64 CPU reference for SP2
 * density-matrix purification.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; it shares no code, header, table or constant with the
 * GPU path.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.
 *
 * What it computes (paper: Fattebert et al., "Hybrid programming-model
 * strategies for GPU offloading of electronic structure calculation kernels",
 * arXiv 2401.13772):
 *
 *   oracle_jacobi_dm     the definition of the zero-temperature density
 *                        matrix: eigen-decompose the symmetric H, then
 *                        D = sum over the n_occ lowest eigenpairs of v v^T
 *                        (Section "Single-particle density matrix ...",
 *                        Fermi-Dirac equation with beta -> infinity and mu in
 *                        the gap).  The eigen-decomposition is the textbook
 *                        cyclic-by-row Jacobi method.
 *   oracle_gershgorin    spectral bounds by Gershgorin circles (Section
 *                        "Distributed matrices"; used as emin/emax in the SP2
 *                        listing of Section "SP2 solver").
 *   oracle_sp2           the SP2 recursion of Section "SP2 solver" (the
 *                        equations for D_0 and D_{m+1}, and the listing's
 *                        branch rule), with plain triple-loop products.
 *   oracle_sp2_spectral  the same recursion applied to the eigenvalues of H
 *                        (a polynomial of H acts on each eigenvalue alone).
 *   oracle_sp2_step_entries  single entries of one SP2 step, for sampled
 *                        checks at sizes where the full loop is too slow.
 *   oracle_cheb_coeffs, oracle_cheb_density, oracle_cheb_ps_split
 *                        the Chebyshev expansion of the Fermi operator of
 *                        Section "Chebyshev polynomial expansion": the
 *                        coefficients c_n of the Fermi-Dirac function on the
 *                        spectrum scaled into [-1, 1], the serial recursion
 *                        T_{n+1} = 2 H T_n - T_{n-1} summed on the matrix,
 *                        and the coefficients d_{i,j} of the
 *                        Paterson-Stockmeyer form sum_j T_k^j S_j.
 *   oracle_learned_spectral, oracle_learned_matrix
 *                        a learned recursive expansion: a composition of
 *                        trained quadratic maps of the matrix (Section "GPU
 *                        friendly algorithms" describes the recursive
 *                        polynomial expansion as a product of layers, each a
 *                        low-order polynomial of the previous layer's output,
 *                        like a deep network).  Layer k maps
 *                        X -> f_k(X) = a_k X^2 + b_k X + c_k I when
 *                        tr X > n_occ and X -> I - f_k(I - X) otherwise (the
 *                        particle-hole form of the same map; with
 *                        (a, b, c) = (1, 0, 0) the two branches are SP2's X^2
 *                        and 2X - X^2).  On eigenvalues and on the matrix.
 *   oracle_sp2_thresh    SP2 with the listing's drop threshold tau: the
 *                        product and the 2X - X^2 update keep only entries
 *                        with |x| >= tau (the pruning of the sparse SP2 paths
 *                        of Section "Leveraging third-party libraries").
 *   oracle_mu_dm, oracle_graph_parts, oracle_graph_density
 *                        the graph-based divide solver of Section "Graph-based
 *                        Divide electronic structure": the thresholded
 *                        adjacency of an auxiliary matrix, core parts as
 *                        regular segments of the index list, core-halo parts,
 *                        the dense sub-problem of each part solved at a common
 *                        chemical potential (zero-temperature Fermi-Dirac, by
 *                        Jacobi), and the core rows mapped back into D.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   - H is used through its symmetric part Hs = (H + H^T)/2.
 *   - D_0 uses Gershgorin bounds (emin, emax) of Hs, computed in FP64.
 *   - The branch uses tr(X_m) taken before the squaring; the tie
 *     tr - n_occ == 0 takes X <- 2X - X^2 (the listing's "<=").
 *   - n_occ plays the role of the listing's number of electrons.
 *   - The convergence check elided in the listing is: e_m = ||X_m^2 - X_m||_F;
 *     stop after the update when e_m <= tol; stop as "stagnated" when
 *     m >= 2, e_m >= e_{m-2} and e_m < 0.1; otherwise stop at max_iter.
 *   - n_occ == 0 gives D = 0 and n_occ == n gives D = I with no iteration.
 *   - emax == emin with 0 < n_occ < n is degenerate (no unique D).
 *   - Thresholded SP2: an entry is dropped when |x| < tau (kept at
 *     equality), after the product and after 2X - X2; X_0 is kept whole; e
 *     is measured with the thresholded product.
 *   - Graph parts: each part's sub-problem is solved at one chemical
 *     potential mu shared by all parts (a part has no integer electron count
 *     of its own); only the rows of a part's core nodes are mapped back, so
 *     every row of D comes from exactly one part and D need not be exactly
 *     symmetric; the halo is one hop of the thresholded graph.
 *
 * Precision: IEEE double throughout.  Build with -ffp-contract=off so every
 * operation is rounded as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORACLE_OK = 0,
    ORACLE_NOT_CONVERGED = 1,
    ORACLE_STAGNATED = 2,
    ORACLE_INVALID = -1,
    ORACLE_DEGENERATE = -2,
    ORACLE_NOMEM = -5
};

typedef struct {
    int32_t status;
    int32_t iterations;
    double emin, emax;
    double trace;          /* trace of the returned D */
    double idempotency;    /* e of the last step taken: ||X_m^2 - X_m||_F */
    uint64_t branch_mask[2]; /* bit m set when step m used 2X - X^2 */
} oracle_sp2_result;

int oracle_version(void) { return 1; }

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int all_finite(const double* A, long count)
{
    for (long i = 0; i < count; ++i)
        if (!isfinite(A[i])) return 0;
    return 1;
}

/* Hs[i][j] = (H[i][j] + H[j][i]) / 2 */
static void symmetric_part(const double* H, int n, double* Hs)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            Hs[(long)i * n + j] = (H[(long)i * n + j] + H[(long)j * n + i]) / 2.0;
}

/* ---------------------------------------------------------------------- */
/* Gershgorin circles: every eigenvalue of Hs lies in some disc centred at  */
/* Hs_ii with radius R_i = sum_{j != i} |Hs_ij|.                            */
/* ---------------------------------------------------------------------- */
int oracle_gershgorin(const double* H, int n, double* emin, double* emax)
{
    if (n <= 0 || !H || !emin || !emax) return ORACLE_INVALID;
    if (!all_finite(H, (long)n * n)) return ORACLE_INVALID;
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < n; ++i) {
        double radius = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            radius += fabs((H[(long)i * n + j] + H[(long)j * n + i]) / 2.0);
        }
        double centre = H[(long)i * n + i];   /* (h + h)/2 == h exactly */
        if (centre - radius < lo) lo = centre - radius;
        if (centre + radius > hi) hi = centre + radius;
    }
    *emin = lo;
    *emax = hi;
    return ORACLE_OK;
}

/* D_0 = (emax I - Hs) / (emax - emin), one division per entry. */
void oracle_sp2_init(const double* H, int n, double emin, double emax, double* X0)
{
    double width = emax - emin;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double hs = (H[(long)i * n + j] + H[(long)j * n + i]) / 2.0;
            double a = (i == j) ? (emax - hs) : (0.0 - hs);
            X0[(long)i * n + j] = a / width;
        }
}

/* ---------------------------------------------------------------------- */
/* Cyclic-by-row Jacobi eigenvalue method for a symmetric matrix.           */
/* Each rotation J(p,q,theta) zeroes a_pq in J^T A J (the classical 2x2     */
/* symmetric Schur decomposition); sweeps repeat until the off-diagonal      */
/* mass is negligible.  On return w is ascending and column i of V (row-     */
/* major n x n) is the eigenvector of w[i].                                  */
/* ---------------------------------------------------------------------- */
int oracle_jacobi_eigh(const double* A_in, int n, double* w, double* V, int max_sweeps,
                       int* sweeps_out)
{
    if (n <= 0 || !A_in || !w || !V) return ORACLE_INVALID;
    if (!all_finite(A_in, (long)n * n)) return ORACLE_INVALID;
    double* a = (double*)malloc(sizeof(double) * (size_t)n * n);
    if (!a) return ORACLE_NOMEM;
    symmetric_part(A_in, n, a);
    for (long i = 0; i < (long)n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[(long)i * n + i] = 1.0;

    double fro2 = 0.0;
    for (long i = 0; i < (long)n * n; ++i) fro2 += a[i] * a[i];
    double thresh = 1e-15 * 1e-15 * fro2;

    int sweep = 0;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += 2.0 * a[(long)p * n + q] * a[(long)p * n + q];
        if (off <= thresh) break;
        int rotations = 0;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = a[(long)p * n + q];
                if (apq == 0.0) continue;
                double app = a[(long)p * n + p], aqq = a[(long)q * n + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* columns: A <- A J */
                for (int k = 0; k < n; ++k) {
                    double akp = a[(long)k * n + p], akq = a[(long)k * n + q];
                    a[(long)k * n + p] = c * akp - s * akq;
                    a[(long)k * n + q] = s * akp + c * akq;
                }
                /* rows: A <- J^T A */
                for (int k = 0; k < n; ++k) {
                    double apk = a[(long)p * n + k], aqk = a[(long)q * n + k];
                    a[(long)p * n + k] = c * apk - s * aqk;
                    a[(long)q * n + k] = s * apk + c * aqk;
                }
                a[(long)p * n + q] = 0.0;
                a[(long)q * n + p] = 0.0;
                /* eigenvectors: V <- V J */
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(long)k * n + p], vkq = V[(long)k * n + q];
                    V[(long)k * n + p] = c * vkp - s * vkq;
                    V[(long)k * n + q] = s * vkp + c * vkq;
                }
                ++rotations;
            }
        }
        if (rotations == 0) break;
    }
    if (sweeps_out) *sweeps_out = sweep;

    /* sort ascending (selection sort on the diagonal, permuting V's columns) */
    for (int i = 0; i < n; ++i) w[i] = a[(long)i * n + i];
    for (int i = 0; i < n - 1; ++i) {
        int best = i;
        for (int j = i + 1; j < n; ++j)
            if (w[j] < w[best]) best = j;
        if (best != i) {
            double tw = w[i]; w[i] = w[best]; w[best] = tw;
            for (int k = 0; k < n; ++k) {
                double tv = V[(long)k * n + i];
                V[(long)k * n + i] = V[(long)k * n + best];
                V[(long)k * n + best] = tv;
            }
        }
    }
    free(a);
    return ORACLE_OK;
}

/* D = sum_{i < n_occ} v_i v_i^T from the ascending eigenpairs of H.
 * w (length n) receives the eigenvalues; gap receives w[n_occ] - w[n_occ-1]
 * (0 when n_occ is 0 or n).  With 0 < n_occ < n and a gap at or below
 * 1e-8 (w[n-1] - w[0]) the occupied subspace is not determined by H (the
 * zero-temperature density matrix is then not unique): D, w and gap are
 * still written and the status is ORACLE_DEGENERATE. */
int oracle_jacobi_dm(const double* H, int n, int n_occ, double* D, double* w, double* gap,
                     int* sweeps)
{
    if (n <= 0 || n_occ < 0 || n_occ > n || !H || !D || !w) return ORACLE_INVALID;
    double* V = (double*)malloc(sizeof(double) * (size_t)n * n);
    if (!V) return ORACLE_NOMEM;
    int st = oracle_jacobi_eigh(H, n, w, V, 100, sweeps);
    if (st != ORACLE_OK) { free(V); return st; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n_occ; ++k) acc += V[(long)i * n + k] * V[(long)j * n + k];
            D[(long)i * n + j] = acc;
        }
    const double g = (n_occ > 0 && n_occ < n) ? w[n_occ] - w[n_occ - 1] : 0.0;
    if (gap) *gap = g;
    free(V);
    if (n_occ > 0 && n_occ < n && !(g > 1e-8 * (w[n - 1] - w[0]))) return ORACLE_DEGENERATE;
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* SP2 on the matrix                                                        */
/* ---------------------------------------------------------------------- */

/* S = X X (n x n, row-major), summing over k in increasing order. */
static void square(const double* X, double* S, int n, int nthreads)
{
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int i = 0; i < n; ++i) {
        double* Si = S + (long)i * n;
        for (int j = 0; j < n; ++j) Si[j] = 0.0;
        for (int k = 0; k < n; ++k) {
            double xik = X[(long)i * n + k];
            const double* Xk = X + (long)k * n;
            for (int j = 0; j < n; ++j) Si[j] += xik * Xk[j];
        }
    }
}

/* S = A B (n x n, row-major), summing over k in increasing order. */
static void square_pair(const double* A, const double* B, double* S, int n, int nthreads)
{
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int i = 0; i < n; ++i) {
        double* Si = S + (long)i * n;
        for (int j = 0; j < n; ++j) Si[j] = 0.0;
        for (int k = 0; k < n; ++k) {
            double aik = A[(long)i * n + k];
            const double* Bk = B + (long)k * n;
            for (int j = 0; j < n; ++j) Si[j] += aik * Bk[j];
        }
    }
}

static double trace_of(const double* X, int n)
{
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += X[(long)i * n + i];
    return t;
}

/*
 * Run SP2 on H.  D (n x n) receives the last iterate.  tr_hist / e_hist (may be
 * NULL, length >= max_iter) receive tr(X_m) and e_m per step.  nthreads sets the
 * OpenMP threads of the products (1 = serial).
 */
int oracle_sp2(const double* H, int n, int n_occ, double tol, int max_iter, int nthreads,
               double* D, oracle_sp2_result* res, double* tr_hist, double* e_hist)
{
    if (!res) return ORACLE_INVALID;
    memset(res, 0, sizeof(*res));
    if (n <= 0 || !H || !D || n_occ < 0 || n_occ > n || !(tol > 0.0) || max_iter < 0) {
        res->status = ORACLE_INVALID;
        return ORACLE_INVALID;
    }
    double emin, emax;
    int st = oracle_gershgorin(H, n, &emin, &emax);
    if (st != ORACLE_OK) { res->status = st; return st; }
    res->emin = emin;
    res->emax = emax;

    long nn = (long)n * n;
    if (n_occ == 0 || n_occ == n) {
        for (long i = 0; i < nn; ++i) D[i] = 0.0;
        if (n_occ == n)
            for (int i = 0; i < n; ++i) D[(long)i * n + i] = 1.0;
        res->trace = (double)n_occ;
        res->status = ORACLE_OK;
        return ORACLE_OK;
    }
    if (!(emax > emin)) { res->status = ORACLE_DEGENERATE; return ORACLE_DEGENERATE; }

    double* X = (double*)malloc(sizeof(double) * (size_t)nn);
    double* S = (double*)malloc(sizeof(double) * (size_t)nn);
    double* e = (double*)malloc(sizeof(double) * (size_t)(max_iter > 0 ? max_iter : 1));
    if (!X || !S || !e) { free(X); free(S); free(e); res->status = ORACLE_NOMEM; return ORACLE_NOMEM; }

    oracle_sp2_init(H, n, emin, emax, X);
    int status = ORACLE_NOT_CONVERGED;
    int m;
    for (m = 0; m < max_iter; ++m) {
        double tr = trace_of(X, n);
        square(X, S, n, nthreads);
        double e2 = 0.0;
        for (long i = 0; i < nn; ++i) {
            double d = S[i] - X[i];
            e2 += d * d;
        }
        e[m] = sqrt(e2);
        int grow = (tr - (double)n_occ <= 0.0);   /* tie goes to 2X - X^2 */
        if (grow) {
            for (long i = 0; i < nn; ++i) X[i] = 2.0 * X[i] - S[i];
            if (m < 128) res->branch_mask[m / 64] |= (uint64_t)1 << (m % 64);
        } else {
            for (long i = 0; i < nn; ++i) X[i] = S[i];
        }
        if (tr_hist) tr_hist[m] = tr;
        if (e_hist) e_hist[m] = e[m];
        res->idempotency = e[m];
        if (e[m] <= tol) { status = ORACLE_OK; ++m; break; }
        if (m >= 2 && e[m] >= e[m - 2] && e[m] < 0.1) { status = ORACLE_STAGNATED; ++m; break; }
    }
    res->iterations = m;
    res->status = status;
    memcpy(D, X, sizeof(double) * (size_t)nn);
    res->trace = trace_of(D, n);
    free(X); free(S); free(e);
    return status;
}

/*
 * The same recursion on eigenvalues: x_i = (emax - lambda_i)/(emax - emin);
 * tr = sum x_i; e = sqrt(sum (x_i^2 - x_i)^2); x_i <- 2x_i - x_i^2 or x_i^2.
 * emin/emax are passed in so the caller can use the matrix's Gershgorin
 * bounds.  x_out (length n, may be NULL) receives the final x_i.
 */
int oracle_sp2_spectral(const double* lambda, int n, int n_occ, double emin, double emax,
                        double tol, int max_iter, double* x_out, oracle_sp2_result* res,
                        double* tr_hist, double* e_hist)
{
    if (!res) return ORACLE_INVALID;
    memset(res, 0, sizeof(*res));
    if (n <= 0 || !lambda || n_occ < 0 || n_occ > n || !(tol > 0.0) || max_iter < 0) {
        res->status = ORACLE_INVALID;
        return ORACLE_INVALID;
    }
    res->emin = emin;
    res->emax = emax;
    if (n_occ == 0 || n_occ == n) {
        if (x_out)
            for (int i = 0; i < n; ++i) x_out[i] = (n_occ == n) ? 1.0 : 0.0;
        res->trace = (double)n_occ;
        res->status = ORACLE_OK;
        return ORACLE_OK;
    }
    if (!(emax > emin)) { res->status = ORACLE_DEGENERATE; return ORACLE_DEGENERATE; }
    double* x = (double*)malloc(sizeof(double) * (size_t)n);
    double* e = (double*)malloc(sizeof(double) * (size_t)(max_iter > 0 ? max_iter : 1));
    if (!x || !e) { free(x); free(e); res->status = ORACLE_NOMEM; return ORACLE_NOMEM; }
    for (int i = 0; i < n; ++i) x[i] = (emax - lambda[i]) / (emax - emin);
    int status = ORACLE_NOT_CONVERGED;
    int m;
    for (m = 0; m < max_iter; ++m) {
        double tr = 0.0, e2 = 0.0;
        for (int i = 0; i < n; ++i) tr += x[i];
        for (int i = 0; i < n; ++i) {
            double d = x[i] * x[i] - x[i];
            e2 += d * d;
        }
        e[m] = sqrt(e2);
        int grow = (tr - (double)n_occ <= 0.0);
        for (int i = 0; i < n; ++i) {
            double sq = x[i] * x[i];
            x[i] = grow ? 2.0 * x[i] - sq : sq;
        }
        if (grow && m < 128) res->branch_mask[m / 64] |= (uint64_t)1 << (m % 64);
        if (tr_hist) tr_hist[m] = tr;
        if (e_hist) e_hist[m] = e[m];
        res->idempotency = e[m];
        if (e[m] <= tol) { status = ORACLE_OK; ++m; break; }
        if (m >= 2 && e[m] >= e[m - 2] && e[m] < 0.1) { status = ORACLE_STAGNATED; ++m; break; }
    }
    res->iterations = m;
    res->status = status;
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += x[i];
    res->trace = t;
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)n);
    free(x); free(e);
    return status;
}

/*
 * Entries (I[t], J[t]) of one SP2 step applied to X (n x n, row-major):
 * (X X)_ij if grow == 0, else 2 X_ij - (X X)_ij.  The sum over k runs in
 * increasing k, as in the full product above.
 */
void oracle_sp2_step_entries(const double* X, int n, int grow, const int* I, const int* J,
                             int count, double* out)
{
    for (int t = 0; t < count; ++t) {
        int i = I[t], j = J[t];
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += X[(long)i * n + k] * X[(long)k * n + j];
        out[t] = grow ? 2.0 * X[(long)i * n + j] - s : s;
    }
}

/* ---------------------------------------------------------------------- */
/* Learned recursive expansion                                             */
/* ---------------------------------------------------------------------- */

/* One layer on a scalar: f(x) = a x^2 + b x + c, or 1 - f(1 - x). */
static double learned_map(double x, const double* abc, int particle_hole)
{
    double a = abc[0], b = abc[1], c = abc[2];
    if (!particle_hole) return a * (x * x) + b * x + c;
    double y = 1.0 - x;
    return 1.0 - (a * (y * y) + b * y + c);
}

/*
 * The learned expansion on eigenvalues: x_i = (emax - lambda_i)/(emax - emin),
 * then n_layers layers (coef: 3 per layer), each taking the particle-hole
 * form when tr - n_occ <= 0 (the trace is taken before the layer, as in SP2).
 * x_out (n) receives the final x_i; branch_mask (2 words, may be NULL) the
 * branch of every layer; tr_hist (n_layers, may be NULL) the traces.
 */
int oracle_learned_spectral(const double* lambda, int n, int n_occ, double emin, double emax,
                            const double* coef, int n_layers, double* x_out, uint64_t* branch_mask,
                            double* tr_hist)
{
    if (n <= 0 || !lambda || !x_out || !coef || n_occ < 0 || n_occ > n || n_layers < 0 ||
        n_layers > 128)
        return ORACLE_INVALID;
    if (!(emax > emin)) return ORACLE_DEGENERATE;
    if (branch_mask) branch_mask[0] = branch_mask[1] = 0;
    for (int i = 0; i < n; ++i) x_out[i] = (emax - lambda[i]) / (emax - emin);
    for (int k = 0; k < n_layers; ++k) {
        double tr = 0.0;
        for (int i = 0; i < n; ++i) tr += x_out[i];
        int ph = (tr - (double)n_occ <= 0.0);
        if (tr_hist) tr_hist[k] = tr;
        if (ph && branch_mask) branch_mask[k / 64] |= (uint64_t)1 << (k % 64);
        for (int i = 0; i < n; ++i) x_out[i] = learned_map(x_out[i], coef + 3 * k, ph);
    }
    return ORACLE_OK;
}

/*
 * The learned expansion on the matrix H (n x n): Gershgorin bounds, X_0 as in
 * SP2, then each layer literally as written above (S = X X or (I-X)(I-X) by
 * the triple loop, then the combination).  D receives X after the last layer.
 */
int oracle_learned_matrix(const double* H, int n, int n_occ, const double* coef, int n_layers,
                          int nthreads, double* D, uint64_t* branch_mask)
{
    if (n <= 0 || !H || !D || !coef || n_occ < 0 || n_occ > n || n_layers < 0 || n_layers > 128)
        return ORACLE_INVALID;
    double emin, emax;
    int st = oracle_gershgorin(H, n, &emin, &emax);
    if (st != ORACLE_OK) return st;
    if (!(emax > emin)) return ORACLE_DEGENERATE;
    long nn = (long)n * n;
    double* X = (double*)malloc(sizeof(double) * (size_t)nn);
    double* Y = (double*)malloc(sizeof(double) * (size_t)nn);
    double* S = (double*)malloc(sizeof(double) * (size_t)nn);
    if (!X || !Y || !S) { free(X); free(Y); free(S); return ORACLE_NOMEM; }
    if (branch_mask) branch_mask[0] = branch_mask[1] = 0;
    oracle_sp2_init(H, n, emin, emax, X);
    for (int k = 0; k < n_layers; ++k) {
        const double a = coef[3 * k], b = coef[3 * k + 1], c = coef[3 * k + 2];
        double tr = trace_of(X, n);
        int ph = (tr - (double)n_occ <= 0.0);
        if (ph && branch_mask) branch_mask[k / 64] |= (uint64_t)1 << (k % 64);
        if (!ph) {
            square(X, S, n, nthreads);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    long q = (long)i * n + j;
                    X[q] = a * S[q] + b * X[q] + (i == j ? c : 0.0);
                }
        } else {
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    long q = (long)i * n + j;
                    Y[q] = (i == j ? 1.0 : 0.0) - X[q];
                }
            square(Y, S, n, nthreads);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    long q = (long)i * n + j;
                    X[q] = (i == j ? 1.0 : 0.0) - (a * S[q] + b * Y[q] + (i == j ? c : 0.0));
                }
        }
    }
    memcpy(D, X, sizeof(double) * (size_t)nn);
    free(X); free(Y); free(S);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Chebyshev expansion of the Fermi operator                               */
/* ---------------------------------------------------------------------- */

/* Fermi-Dirac occupation 1 / (1 + exp(t)), evaluated without overflow. */
static double fermi(double t)
{
    if (t > 0.0) { double e = exp(-t); return e / (1.0 + e); }
    return 1.0 / (1.0 + exp(t));
}

/*
 * c_0..c_L of f(x) = 1/(1 + exp(bs (x - ms))) on [-1, 1] (bs, ms: the inverse
 * temperature and chemical potential in the scaled variable), by the
 * Chebyshev-Gauss rule with q nodes:
 *   c_n = (2 - [n == 0]) / q * sum_{j<q} f(cos t_j) cos(n t_j),
 *   t_j = pi (j + 1/2) / q.
 */
int oracle_cheb_coeffs(int L, double bs, double ms, int q, double* c)
{
    if (L < 0 || q < L + 1 || !c) return ORACLE_INVALID;
    const double pi = 3.14159265358979323846;
    for (int n = 0; n <= L; ++n) {
        double acc = 0.0;
        for (int j = 0; j < q; ++j) {
            double t = pi * (j + 0.5) / q;
            acc += fermi(bs * (cos(t) - ms)) * cos(n * t);
        }
        c[n] = (n == 0 ? 1.0 : 2.0) * acc / q;
    }
    return ORACLE_OK;
}

/*
 * D = sum_{n<=L} c_n T_n(Hs) with Hs = (H - a I)/b, a and b the centre and
 * half width of the Gershgorin interval, by the serial recursion
 * T_{n+1} = 2 Hs T_n - T_{n-1} (triple-loop products).  mu and beta in the
 * units of H; q nodes for the coefficients (q >= L + 1).  coef (may be NULL,
 * length L + 1) receives c_n; bounds (may be NULL) a and b.
 */
int oracle_cheb_density(const double* H, int n, int L, double beta, double mu, int q, int nthreads,
                        double* D, double* coef, double* bounds)
{
    if (n <= 0 || !H || !D || L < 0 || q < L + 1 || !(beta > 0.0)) return ORACLE_INVALID;
    double emin, emax;
    int st = oracle_gershgorin(H, n, &emin, &emax);
    if (st != ORACLE_OK) return st;
    if (!(emax > emin)) return ORACLE_DEGENERATE;
    const double a = (emax + emin) / 2.0, b = (emax - emin) / 2.0;
    if (bounds) { bounds[0] = a; bounds[1] = b; }
    long nn = (long)n * n;
    double* c = (double*)malloc(sizeof(double) * (size_t)(L + 1));
    double* Hs = (double*)malloc(sizeof(double) * (size_t)nn);
    double* Tm = (double*)malloc(sizeof(double) * (size_t)nn);   /* T_{k-1} */
    double* T = (double*)malloc(sizeof(double) * (size_t)nn);    /* T_k */
    double* Tn = (double*)malloc(sizeof(double) * (size_t)nn);   /* T_{k+1} */
    if (!c || !Hs || !Tm || !T || !Tn) {
        free(c); free(Hs); free(Tm); free(T); free(Tn);
        return ORACLE_NOMEM;
    }
    oracle_cheb_coeffs(L, beta * b, (mu - a) / b, q, c);
    if (coef) memcpy(coef, c, sizeof(double) * (size_t)(L + 1));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            long p = (long)i * n + j;
            double hs = (H[p] + H[(long)j * n + i]) / 2.0;
            Hs[p] = ((i == j ? hs - a : hs)) / b;
            Tm[p] = (i == j) ? 1.0 : 0.0;           /* T_0 */
            T[p] = Hs[p];                           /* T_1 */
            D[p] = c[0] * Tm[p];
        }
    if (L >= 1)
        for (long p = 0; p < nn; ++p) D[p] += c[1] * T[p];
    for (int k = 1; k < L; ++k) {
        square_pair(Hs, T, Tn, n, nthreads);
        for (long p = 0; p < nn; ++p) {
            Tn[p] = 2.0 * Tn[p] - Tm[p];
            D[p] += c[k + 1] * Tn[p];
        }
        double* t = Tm; Tm = T; T = Tn; Tn = t;
    }
    free(c); free(Hs); free(Tm); free(T); free(Tn);
    return ORACLE_OK;
}

/*
 * The Paterson-Stockmeyer form: given c_0..c_{k m - 1}, the d_{i,j}
 * (i < k, j < m; d[j * k + i]) with sum_n c_n T_n = sum_j T_k^j S_j,
 * S_j = sum_{i<k} d_{i,j} T_i.  By repeated division by T_k in the
 * Chebyshev basis: for the highest remaining degree t >= k,
 * T_t = 2 T_k T_{t-k} - T_{|2k - t|} (T_k T_0 = T_k for t = k) moves the
 * coefficient of T_t into the quotient; what remains below k is S_j.
 */
int oracle_cheb_ps_split(const double* c, int k, int m, double* d)
{
    if (!c || !d || k < 1 || m < 1) return ORACLE_INVALID;
    int N = k * m;
    double* a = (double*)malloc(sizeof(double) * (size_t)N);
    double* qt = (double*)malloc(sizeof(double) * (size_t)N);
    if (!a || !qt) { free(a); free(qt); return ORACLE_NOMEM; }
    memcpy(a, c, sizeof(double) * (size_t)N);
    int deg = N - 1;
    for (int j = 0; j < m; ++j) {
        for (int t = 0; t < N; ++t) qt[t] = 0.0;
        for (int t = deg; t >= k; --t) {
            double v = a[t];
            a[t] = 0.0;
            if (t == k) {
                qt[0] += v;
            } else {
                qt[t - k] += 2.0 * v;
                int r = 2 * k - t;
                if (r < 0) r = -r;
                a[r] -= v;
            }
        }
        for (int i = 0; i < k; ++i) d[j * k + i] = (i <= deg) ? a[i] : 0.0;
        deg -= k;
        for (int t = 0; t < N; ++t) a[t] = qt[t];
    }
    free(a); free(qt);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Graph-partitioned density matrix (Section "Graph-based Divide          */
/* electronic structure": the adjacency equation, core and core-halo      */
/* partitions, sub-matrix extraction and map-back of the general solver   */
/* routine listing)                                                         */
/* ---------------------------------------------------------------------- */

/* Zero-temperature density matrix at a given chemical potential: the
 * Fermi-Dirac function with beta -> infinity is 1 below mu and 0 above, so
 * D = sum over the eigenpairs with w_i < mu of v_i v_i^T.  The eigenvalues
 * go to w.  An eigenvalue within 1e-8 (w[n-1] - w[0]) of mu leaves D
 * undetermined: D is still written and the status is ORACLE_DEGENERATE. */
int oracle_mu_dm(const double* H, int n, double mu, double* D, double* w)
{
    if (n <= 0 || !H || !D || !w || !isfinite(mu)) return ORACLE_INVALID;
    double* V = (double*)malloc(sizeof(double) * (size_t)n * n);
    if (!V) return ORACLE_NOMEM;
    int st = oracle_jacobi_eigh(H, n, w, V, 100, NULL);
    if (st != ORACLE_OK) { free(V); return st; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int k = 0; k < n; ++k)
                if (w[k] < mu) acc += V[(long)i * n + k] * V[(long)j * n + k];
            D[(long)i * n + j] = acc;
        }
    free(V);
    const double width = w[n - 1] - w[0];
    for (int k = 0; k < n; ++k)
        if (fabs(w[k] - mu) <= 1e-8 * width) return ORACLE_DEGENERATE;
    return ORACLE_OK;
}

/* First node of core part k when n nodes are cut into `parts` regular
 * segments of the index list: floor(k n / parts). */
static int segment_start(int k, int n, int parts)
{
    return (int)(((long)k * n) / parts);
}

/* Membership of the core-halo parts: in_part[k * n + j] = 1 when node j is
 * in part k.  Core part k is the k-th regular segment of the index list.
 * The graph's adjacency is A_lj = 1 when |G_lj| >= tau and l != j; the part
 * adds to its core every node j with A_lj = 1 for a core node l. */
int oracle_graph_parts(const double* G, int n, double tau, int parts, unsigned char* in_part)
{
    if (!G || !in_part || n <= 0 || parts < 1 || parts > n || !(tau >= 0.0)) return ORACLE_INVALID;
    for (int k = 0; k < parts; ++k) {
        unsigned char* row = in_part + (long)k * n;
        for (int j = 0; j < n; ++j) row[j] = 0;
        const int c0 = segment_start(k, n, parts), c1 = segment_start(k + 1, n, parts);
        for (int l = c0; l < c1; ++l) {
            row[l] = 1;                                   /* the core node */
            for (int j = 0; j < n; ++j)
                if (j != l && fabs(G[(long)l * n + j]) >= tau) row[j] = 1;   /* its neighbours */
        }
    }
    return ORACLE_OK;
}

/* The graph-based density matrix: for every part, the sub-matrix h of H on
 * the part's nodes (ascending node order), its density matrix at chemical
 * potential mu (oracle_mu_dm), and the rows of the part's core nodes mapped
 * back into D (row l of D gets h's row for l, spread over the part's nodes;
 * every other entry of that row is 0).  sizes[k] = nodes in part k.
 * Returns ORACLE_DEGENERATE if any part's sub-problem is degenerate. */
int oracle_graph_density(const double* H, const double* G, int n, double tau, int parts, double mu,
                         double* D, int* sizes)
{
    if (!H || !G || !D || n <= 0 || parts < 1 || parts > n || !(tau >= 0.0) || !isfinite(mu))
        return ORACLE_INVALID;
    unsigned char* in_part = (unsigned char*)malloc((size_t)parts * n);
    int* nodes = (int*)malloc(sizeof(int) * (size_t)n);
    if (!in_part || !nodes) { free(in_part); free(nodes); return ORACLE_NOMEM; }
    int st = oracle_graph_parts(G, n, tau, parts, in_part);
    for (long p = 0; p < (long)n * n; ++p) D[p] = 0.0;
    int degenerate = 0;
    for (int k = 0; k < parts && st == ORACLE_OK; ++k) {
        int s = 0;
        for (int j = 0; j < n; ++j)
            if (in_part[(long)k * n + j]) nodes[s++] = j;
        if (sizes) sizes[k] = s;
        double* h = (double*)malloc(sizeof(double) * (size_t)s * s);
        double* d = (double*)malloc(sizeof(double) * (size_t)s * s);
        double* w = (double*)malloc(sizeof(double) * (size_t)s);
        if (!h || !d || !w) { free(h); free(d); free(w); st = ORACLE_NOMEM; break; }
        for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b) h[(long)a * s + b] = H[(long)nodes[a] * n + nodes[b]];
        int r = oracle_mu_dm(h, s, mu, d, w);
        if (r == ORACLE_DEGENERATE) degenerate = 1;
        else if (r != ORACLE_OK) st = r;
        const int c0 = segment_start(k, n, parts), c1 = segment_start(k + 1, n, parts);
        for (int a = 0; a < s; ++a) {
            const int l = nodes[a];
            if (l < c0 || l >= c1) continue;              /* halo rows are not kept */
            for (int b = 0; b < s; ++b) D[(long)l * n + nodes[b]] = d[(long)a * s + b];
        }
        free(h); free(d); free(w);
    }
    free(in_part); free(nodes);
    if (st != ORACLE_OK) return st;
    return degenerate ? ORACLE_DEGENERATE : ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Thresholded SP2 (the drop threshold tau of the SP2 listing: the product */
/* and the update keep only entries with |x| >= tau, the pruning the       */
/* sparse solvers of Section "Leveraging third-party libraries" apply)     */
/* ---------------------------------------------------------------------- */

/* Entry kept by the drop rule; *margin tracks the closest call,
 * | |v| - tau | / max(|v|, tau), over every decision with tau > 0. */
static double drop_small(double v, double tau, double* margin)
{
    if (tau > 0.0) {
        double a = fabs(v);
        double m = fabs(a - tau) / (a > tau ? a : tau);
        if (m < *margin) *margin = m;
        if (a < tau) return 0.0;
    }
    return v;
}

/* SP2 as in the listing with a drop threshold: X2 = drop(X X); the update is
 * X = drop(2 X - X2) or X = X2; X_0 is not thresholded (the listing forms it
 * by copy, shift and scale).  e_m = ||X2 - X_m||_F with the thresholded X2;
 * branch, stop rule and special cases as oracle_sp2 (tau = 0 is oracle_sp2).
 * margin (may be NULL) receives the closest drop decision (see drop_small);
 * 1 when no decision was taken. */
int oracle_sp2_thresh(const double* H, int n, int n_occ, double tol, int max_iter, double tau,
                      int nthreads, double* D, oracle_sp2_result* res, double* margin)
{
    if (!res) return ORACLE_INVALID;
    memset(res, 0, sizeof(*res));
    double mg = 1.0;
    if (margin) *margin = 1.0;
    if (n <= 0 || !H || !D || n_occ < 0 || n_occ > n || !(tol > 0.0) || max_iter < 0 || !(tau >= 0.0)) {
        res->status = ORACLE_INVALID;
        return ORACLE_INVALID;
    }
    double emin, emax;
    int st = oracle_gershgorin(H, n, &emin, &emax);
    if (st != ORACLE_OK) { res->status = st; return st; }
    res->emin = emin;
    res->emax = emax;
    long nn = (long)n * n;
    if (n_occ == 0 || n_occ == n) {
        for (long i = 0; i < nn; ++i) D[i] = 0.0;
        if (n_occ == n)
            for (int i = 0; i < n; ++i) D[(long)i * n + i] = 1.0;
        res->trace = (double)n_occ;
        res->status = ORACLE_OK;
        return ORACLE_OK;
    }
    if (!(emax > emin)) { res->status = ORACLE_DEGENERATE; return ORACLE_DEGENERATE; }
    double* X = (double*)malloc(sizeof(double) * (size_t)nn);
    double* S = (double*)malloc(sizeof(double) * (size_t)nn);
    double* e = (double*)malloc(sizeof(double) * (size_t)(max_iter > 0 ? max_iter : 1));
    if (!X || !S || !e) { free(X); free(S); free(e); res->status = ORACLE_NOMEM; return ORACLE_NOMEM; }
    oracle_sp2_init(H, n, emin, emax, X);
    int status = ORACLE_NOT_CONVERGED;
    int m;
    for (m = 0; m < max_iter; ++m) {
        double tr = trace_of(X, n);
        square(X, S, n, nthreads);
        for (long i = 0; i < nn; ++i) S[i] = drop_small(S[i], tau, &mg);
        double e2 = 0.0;
        for (long i = 0; i < nn; ++i) {
            double d = S[i] - X[i];
            e2 += d * d;
        }
        e[m] = sqrt(e2);
        int grow = (tr - (double)n_occ <= 0.0);
        if (grow) {
            for (long i = 0; i < nn; ++i) X[i] = drop_small(2.0 * X[i] - S[i], tau, &mg);
            if (m < 128) res->branch_mask[m / 64] |= (uint64_t)1 << (m % 64);
        } else {
            for (long i = 0; i < nn; ++i) X[i] = S[i];
        }
        res->idempotency = e[m];
        if (e[m] <= tol) { status = ORACLE_OK; ++m; break; }
        if (m >= 2 && e[m] >= e[m - 2] && e[m] < 0.1) { status = ORACLE_STAGNATED; ++m; break; }
    }
    res->iterations = m;
    res->status = status;
    memcpy(D, X, sizeof(double) * (size_t)nn);
    res->trace = trace_of(D, n);
    if (margin) *margin = mg;
    free(X); free(S); free(e);
    return status;
}
