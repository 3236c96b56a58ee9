"""Pins for the FP64 CPU oracle (no GPU).

The oracle is checked against things other than itself: hand-derived closed
forms (tests/golden), a third-party eigensolver (LAPACK through NumPy),
exact invariants of projectors, brute force on diagonal inputs, and
equivariances of the density matrix.  Each test names the plausible oracle
mistake it would catch.
"""
import numpy as np
import pytest

import golden
from tbgen import diagonal_hamiltonian, gapped_random_hamiltonian, make_tb_hamiltonian, two_level_hamiltonian


def fro_rms(A):
    return np.linalg.norm(A) / np.sqrt(A.shape[0])


def lapack_dm(H, n_occ):
    w, V = np.linalg.eigh(H)
    return V[:, :n_occ] @ V[:, :n_occ].T, w


# --------------------------------------------------------------------------- bounds

def test_gershgorin_hand_3x3(oracle_lib):
    g = golden.load("gershgorin_3x3.txt")
    lo, hi = oracle_lib.gershgorin(g["H"])
    assert lo == g["emin"] and hi == g["emax"]          # catches a dropped |.| or a wrong row/col


def test_gershgorin_symmetric_part(oracle_lib):
    g = golden.load("gershgorin_nonsym_2x2.txt")
    lo, hi = oracle_lib.gershgorin(g["H"])
    assert (lo, hi) == (g["emin"], g["emax"])           # catches reading H instead of (H+H^T)/2
    r = oracle_lib.sp2(g["H"], int(g["n_occ"]))
    assert np.abs(r.D - g["D"]).max() < 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gershgorin_contains_spectrum(oracle_lib, seed):
    H = make_tb_hamiltonian(64, seed).H
    lo, hi = oracle_lib.gershgorin(H)
    w = np.linalg.eigvalsh(H)
    assert lo <= w[0] and w[-1] <= hi
    # exact for a diagonal matrix: the discs have radius 0
    Hd = diagonal_hamiltonian(17, seed)
    lo, hi = oracle_lib.gershgorin(Hd)
    assert lo == np.diag(Hd).min() and hi == np.diag(Hd).max()


def test_init_matches_hand_values(oracle_lib):
    g = golden.load("dm_2x2_tie.txt")
    X0 = oracle_lib.sp2_init(g["H"], g["emin"], g["emax"])
    assert np.array_equal(X0, g["X0"])                   # catches a sign/shift error in D_0
    assert np.trace(X0) == 1.0


# --------------------------------------------------------------------------- Jacobi

@pytest.mark.parametrize("n,seed", [(5, 0), (33, 1), (64, 2)])
def test_jacobi_against_lapack(oracle_lib, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    A = A + A.T
    w, V, sweeps = oracle_lib.jacobi_eigh(A)
    wl = np.linalg.eigvalsh(A)
    scale = np.abs(wl).max()
    assert np.abs(w - wl).max() <= 1e-13 * scale * n
    assert np.abs(V.T @ V - np.eye(n)).max() < 1e-13 * n
    assert np.abs(A @ V - V * w).max() < 1e-12 * scale * n
    assert sweeps < 30


def test_jacobi_dm_closed_form_2x2(oracle_lib):
    g = golden.load("dm_2x2_tie.txt")
    D, w, gap = oracle_lib.jacobi_dm(g["H"], 1)
    assert np.abs(w - g["eigenvalues"]).max() < 1e-14
    assert np.abs(D - g["D"]).max() < 1e-15
    assert gap == pytest.approx(10.0)


@pytest.mark.parametrize("seed", range(6))
def test_jacobi_dm_random_2x2_closed_form(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    a, b, c = rng.normal(size=3) * [3, 2, 3]
    H = np.array([[a, b], [b, c]])
    lp = (a + c) / 2 + np.sqrt(((a - c) / 2) ** 2 + b * b)
    lm = (a + c) / 2 - np.sqrt(((a - c) / 2) ** 2 + b * b)
    Dexact = (lp * np.eye(2) - H) / (lp - lm)
    D, _, _ = oracle_lib.jacobi_dm(H, 1)
    assert np.abs(D - Dexact).max() < 1e-13
    r = oracle_lib.sp2(H, 1)
    assert r.status == 0
    assert np.abs(r.D - Dexact).max() < 1e-10


@pytest.mark.parametrize("n,seed", [(64, 3), (128, 4)])
def test_jacobi_dm_matches_lapack_projector(oracle_lib, n, seed):
    inst = make_tb_hamiltonian(n, seed)
    D, w, gap = oracle_lib.jacobi_dm(inst.H, inst.n_occ)
    Dl, wl = lapack_dm(inst.H, inst.n_occ)
    assert fro_rms(D - Dl) < 1e-12
    assert gap == pytest.approx(0.5, abs=1e-9)


# --------------------------------------------------------------------------- SP2

def test_tie_goes_to_grow_branch(oracle_lib):
    """tr X0 == n_occ exactly: the listing's "<=" takes 2X - X^2 first."""
    g = golden.load("dm_2x2_tie.txt")
    r = oracle_lib.sp2(g["H"], 1, max_iter=1)
    assert r.status == 1 and r.iterations == 1
    assert r.branches() == [int(g["first_branch"])]
    assert r.tr_hist[0] == 1.0
    rs, x = oracle_lib.sp2_spectral(g["eigenvalues"], 1, g["emin"], g["emax"], max_iter=1)
    assert rs.branches() == [1]
    assert np.abs(x - g["x_after_first_step"]).max() < 1e-15
    full = oracle_lib.sp2(g["H"], 1)
    assert full.status == 0 and np.abs(full.D - g["D"]).max() < 1e-10


@pytest.mark.parametrize("n,seed", [(32, 0), (64, 1), (128, 2), (256, 0)])
def test_sp2_matches_jacobi_dm(oracle_lib, n, seed):
    inst = make_tb_hamiltonian(n, seed)
    D, w, gap = oracle_lib.jacobi_dm(inst.H, inst.n_occ)
    r = oracle_lib.sp2(inst.H, inst.n_occ, tol=1e-10)
    assert r.status == 0
    assert 20 <= r.iterations <= 45
    assert fro_rms(r.D - D) < 1e-10


@pytest.mark.parametrize("n,seed", [(64, 5), (128, 6)])
def test_sp2_invariants(oracle_lib, n, seed):
    inst = make_tb_hamiltonian(n, seed)
    H = inst.H
    r = oracle_lib.sp2(H, inst.n_occ)
    D = r.D
    wl = np.linalg.eigvalsh(H)
    assert np.abs(D - D.T).max() < 1e-13
    assert np.linalg.norm(D @ D - D) < 1e-9
    assert abs(np.trace(D) - inst.n_occ) < 1e-9
    assert np.linalg.norm(H @ D - D @ H) / np.sqrt(n) < 1e-8
    assert np.trace(D @ H) == pytest.approx(wl[: inst.n_occ].sum(), rel=1e-11)
    wd = np.linalg.eigvalsh(D)
    assert np.abs(wd[: n - inst.n_occ]).max() < 1e-9 and np.abs(wd[n - inst.n_occ:] - 1).max() < 1e-9


@pytest.mark.parametrize("n,k", [(16, 5), (40, 20), (64, 9)])
def test_two_level_system(oracle_lib, n, k):
    H, P = two_level_hamiltonian(n, k, alpha=-1.3, beta=2.1, seed=n + k)
    r = oracle_lib.sp2(H, k)
    assert r.status == 0
    assert np.abs(r.D - P).max() < 1e-9
    D, _, _ = oracle_lib.jacobi_dm(H, k)
    assert np.abs(D - P).max() < 1e-12
    # the spectral recursion needs only the two levels with their multiplicities
    lam = np.array([-1.3] * k + [2.1] * (n - k))
    rs, _ = oracle_lib.sp2_spectral(lam, k, r.emin, r.emax)
    assert rs.iterations == r.iterations


@pytest.mark.parametrize("n,seed", [(7, 0), (31, 1), (100, 2)])
def test_diagonal_brute_force_and_bitwise(oracle_lib, n, seed):
    Hd = diagonal_hamiltonian(n, seed)
    d = np.diag(Hd)
    n_occ = n // 3 + 1
    r = oracle_lib.sp2(Hd, n_occ)
    assert r.status == 0
    want = np.zeros(n)
    want[np.argsort(d)[:n_occ]] = 1.0                    # brute force: the n_occ lowest levels
    assert np.abs(np.diag(r.D) - want).max() < 1e-9
    assert np.count_nonzero(r.D - np.diag(np.diag(r.D))) == 0
    # SP2 acts entrywise on a diagonal matrix: the spectral recursion over the
    # diagonal (same order, same bounds) must agree bit for bit
    rs, x = oracle_lib.sp2_spectral(d, n_occ, r.emin, r.emax)
    assert rs.iterations == r.iterations and rs.branch_mask == r.branch_mask
    assert np.array_equal(x, np.diag(r.D))


@pytest.mark.parametrize("n,seed", [(64, 7), (128, 8), (256, 9)])
def test_spectral_predicts_matrix_steering(oracle_lib, n, seed):
    inst = make_tb_hamiltonian(n, seed)
    r = oracle_lib.sp2(inst.H, inst.n_occ)
    w = np.linalg.eigvalsh(inst.H)
    rs, _ = oracle_lib.sp2_spectral(w, inst.n_occ, r.emin, r.emax)
    assert rs.iterations == r.iterations
    trm, trs = np.asarray(r.tr_hist), np.asarray(rs.tr_hist)
    assert np.abs(trm - trs).max() <= 1e-9 * n
    decided = np.abs(trm - inst.n_occ) > 1e-9 * n
    bm, bs = np.array(r.branches()), np.array(rs.branches())
    assert np.array_equal(bm[decided], bs[decided])
    assert np.abs(np.asarray(r.e_hist)[:-3] - np.asarray(rs.e_hist)[:-3]).max() < 1e-8


def test_equivariances(oracle_lib):
    inst = make_tb_hamiltonian(64, 11)
    H, k = inst.H, inst.n_occ
    D = oracle_lib.sp2(H, k).D
    rng = np.random.default_rng(0)
    p = rng.permutation(64)
    Dp = oracle_lib.sp2(H[np.ix_(p, p)], k).D
    assert np.abs(Dp - D[np.ix_(p, p)]).max() < 1e-9    # catches index mix-ups
    assert np.abs(oracle_lib.sp2(H + 3.7 * np.eye(64), k).D - D).max() < 1e-9
    assert np.abs(oracle_lib.sp2(2.5 * H, k).D - D).max() < 1e-9
    Dph = oracle_lib.sp2(-H, 64 - k).D                   # particle-hole symmetry
    assert np.abs(Dph - (np.eye(64) - D)).max() < 1e-9


def test_special_and_error_cases(oracle_lib):
    H = make_tb_hamiltonian(16, 3).H
    r0 = oracle_lib.sp2(H, 0)
    assert r0.status == 0 and r0.iterations == 0 and not r0.D.any()
    rn = oracle_lib.sp2(H, 16)
    assert rn.status == 0 and np.array_equal(rn.D, np.eye(16))
    assert oracle_lib.sp2(2.0 * np.eye(8), 3).status == oracle_lib.DEGENERATE
    Hn = H.copy()
    Hn[3, 5] = np.nan
    assert oracle_lib.sp2(Hn, 8).status == oracle_lib.INVALID
    r1 = oracle_lib.sp2(H, 8, max_iter=1)
    assert r1.status == oracle_lib.NOT_CONVERGED and r1.iterations == 1
    # a tolerance below the rounding floor ends on the stagnation rule
    rs = oracle_lib.sp2(H, 8, tol=1e-300)
    assert rs.status == oracle_lib.STAGNATED
    assert np.linalg.norm(rs.D @ rs.D - rs.D) < 1e-12
    assert oracle_lib.sp2(H, 8, tol=0.0).status == oracle_lib.INVALID


def test_step_entries_match_library_matmul(oracle_lib):
    inst = make_tb_hamiltonian(48, 2)
    lo, hi = oracle_lib.gershgorin(inst.H)
    X = oracle_lib.sp2_init(inst.H, lo, hi)
    rng = np.random.default_rng(1)
    I = rng.integers(0, 48, 50)
    J = rng.integers(0, 48, 50)
    S = X @ X
    for grow in (0, 1):
        got = oracle_lib.sp2_step_entries(X, grow, I, J)
        want = (2 * X - S if grow else S)[I, J]
        assert np.abs(got - want).max() < 1e-14


# --------------------------------------------------------------------------- learned expansion

def test_learned_hand_three_levels(oracle_lib):
    g = golden.load("learned_3level.txt")
    x, br, tr = oracle_lib.learned_spectral(g["lambda"], int(g["n_occ"]), g["emin"], g["emax"],
                                            g["coef"])
    # exact dyadic values: catches a swapped branch, a wrong sign in the
    # particle-hole form or a coefficient applied to the wrong power
    assert br == [int(v) for v in g["branches"]]
    assert np.array_equal(x, g["x_final"])
    x1, _, _ = oracle_lib.learned_spectral(g["lambda"], 1, g["emin"], g["emax"], g["coef"][:3])
    assert np.array_equal(x1, g["x_after_layer0"])


@pytest.mark.parametrize("seed", [0, 1])
def test_learned_with_sp2_coefficients_is_sp2(oracle_lib, seed):
    """(a, b, c) = (1, 0, 0) in every layer is SP2 truncated after that many steps."""
    inst = make_tb_hamiltonian(128, seed=seed)
    w = np.linalg.eigvalsh(inst.H)
    lo, hi = oracle_lib.gershgorin(inst.H)
    L = 20
    x, br, tr = oracle_lib.learned_spectral(w, inst.n_occ, lo, hi, np.tile([1.0, 0.0, 0.0], L))
    ref, xs = oracle_lib.sp2_spectral(w, inst.n_occ, lo, hi, tol=1e-300, max_iter=L)
    assert br == ref.branches()
    assert np.allclose(tr, ref.tr_hist, rtol=0, atol=1e-10)
    assert np.abs(x - xs).max() < 1e-11


def test_learned_matrix_equals_spectral_form(oracle_lib):
    """Every layer is a polynomial of H, so D = V diag(p(x_i)) V^T with V from
    LAPACK; catches a layer applied to the wrong matrix (X vs I - X) or a
    missing identity term."""
    rng = np.random.default_rng(4)
    inst = make_tb_hamiltonian(64, seed=6)
    coef = np.column_stack([1.0 + 0.3 * rng.standard_normal(6), 0.2 * rng.standard_normal(6),
                            0.05 * rng.standard_normal(6)])
    D, br = oracle_lib.learned_matrix(inst.H, inst.n_occ, coef)
    w, V = np.linalg.eigh(inst.H)
    lo, hi = oracle_lib.gershgorin(inst.H)
    x, brs, _ = oracle_lib.learned_spectral(w, inst.n_occ, lo, hi, coef)
    assert br == brs
    assert np.abs(D - (V * x) @ V.T).max() < 1e-10


def test_learned_particle_hole_symmetry(oracle_lib):
    """-H with n - n_occ occupied maps x -> 1 - x and swaps the branches, so
    D(-H, n - n_occ) = I - D(H, n_occ)."""
    rng = np.random.default_rng(8)
    inst = make_tb_hamiltonian(48, seed=2)
    coef = np.column_stack([1.0 + 0.2 * rng.standard_normal(5), 0.1 * rng.standard_normal(5),
                            0.02 * rng.standard_normal(5)])
    D, br = oracle_lib.learned_matrix(inst.H, inst.n_occ, coef)
    Dm, brm = oracle_lib.learned_matrix(-inst.H, 48 - inst.n_occ, coef)
    assert [1 - b for b in br] == brm
    assert np.abs(Dm - (np.eye(48) - D)).max() < 1e-10


# --------------------------------------------------------------------------- Chebyshev expansion

def test_cheb_coeffs_match_library_interpolant(oracle_lib):
    """The Chebyshev-Gauss coefficients equal NumPy's Chebyshev interpolant of
    the same function at the same nodes (a wrong node, weight or the factor 2
    on n > 0 fails)."""
    from numpy.polynomial import chebyshev as C
    L, bs, ms = 40, 12.0, 0.1
    c = oracle_lib.cheb_coeffs(L, bs, ms, q=L + 1)
    f = lambda x: 1.0 / (1.0 + np.exp(bs * (x - ms)))
    ref = C.chebinterpolate(f, L)
    assert np.abs(c - ref).max() < 1e-13


def test_cheb_series_converges_to_fermi_function(oracle_lib):
    from numpy.polynomial import chebyshev as C
    bs, ms = 30.0, -0.2
    x = np.linspace(-1, 1, 201)
    f = 1.0 / (1.0 + np.exp(bs * (x - ms)))
    errs = [np.abs(C.chebval(x, oracle_lib.cheb_coeffs(L, bs, ms)) - f).max() for L in (20, 60, 200)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-9


@pytest.mark.parametrize("k,m", [(1, 5), (4, 4), (5, 3), (8, 9)])
def test_ps_split_reproduces_series(oracle_lib, k, m):
    """sum_j T_k(x)^j S_j(x) equals the series at random points (a wrong
    remainder index in the division by T_k fails)."""
    from numpy.polynomial import chebyshev as C
    rng = np.random.default_rng(k * 10 + m)
    c = rng.standard_normal(k * m)
    d = oracle_lib.cheb_ps_split(c, k, m)
    x = rng.uniform(-1, 1, 50)
    Tk = C.chebval(x, np.eye(k + 1)[k])
    val = np.zeros_like(x)
    for j in reversed(range(m)):
        val = C.chebval(x, d[j]) + Tk * val
    assert np.abs(val - C.chebval(x, c)).max() < 1e-11


def test_cheb_density_is_fermi_operator(oracle_lib):
    """On the matrix: V diag(sum c_n T_n(x_i)) V^T (LAPACK V) equals the serial
    recursion, and it equals the Fermi operator V diag(f(eps_i)) V^T to the
    series' own approximation error."""
    from numpy.polynomial import chebyshev as C
    inst = make_tb_hamiltonian(64, seed=13, gap=1.0)
    w, V = np.linalg.eigh(inst.H)
    mu = 0.5 * (w[31] + w[32])
    beta = 0.5                                           # 1/eV; ~35 in the scaled variable
    D, c, (a, b) = oracle_lib.cheb_density(inst.H, 200, beta=beta, mu=mu)
    lo, hi = oracle_lib.gershgorin(inst.H)
    assert a == (hi + lo) / 2 and b == (hi - lo) / 2
    spec = C.chebval((w - a) / b, c)
    assert np.abs(D - (V * spec) @ V.T).max() < 1e-10
    fermi = 1.0 / (1.0 + np.exp(beta * (w - mu)))
    assert np.abs(spec - fermi).max() < 1e-10
    assert np.abs(D - (V * fermi) @ V.T).max() < 1e-9


def test_jacobi_dm_flags_a_vanishing_gap(oracle_lib):
    """Two equal levels straddling the Fermi level: any unit vector in their
    span is a valid occupied state, so the oracle reports the case as
    degenerate rather than returning one of them as the answer; a gap of
    1e-6 of the width is still resolved."""
    H = np.diag([-1.0, 0.5, 0.5, 2.0])
    with pytest.raises(oracle_lib.DegenerateError):
        oracle_lib.jacobi_dm(H, 2)
    H2 = np.diag([-1.0, 0.5, 0.5 + 3e-6, 2.0])
    D, w, gap = oracle_lib.jacobi_dm(H2, 2)
    assert np.allclose(D, np.diag([1.0, 1.0, 0.0, 0.0]), atol=1e-12) and abs(gap - 3e-6) < 1e-12


# ---------------------------------------------------------------- graph solver

def test_graph_parts_hand_worked_chain(oracle_lib):
    """Core-halo membership of a 6-node graph worked by hand at three
    thresholds; an asymmetric entry pins that the halo follows row l of the
    adjacency (node o joins when A_lo = 1 for a core node l)."""
    g = golden.load("graph_chain6.txt")
    n, parts = g["n"], int(g["parts"])
    G = g["G"].reshape(n, n)
    for key in ("a", "b", "c"):
        got = oracle_lib.graph_parts(G, g["tau_" + key], parts)
        want = g["parts_" + key].reshape(parts, n).astype(bool)
        assert np.array_equal(got, want), key


def test_mu_dm_special_cases(oracle_lib):
    """Diagonal H: D = diag(w < mu); a 2x2 closed form; mu at an eigenvalue
    is reported degenerate."""
    H = diagonal_hamiltonian(9, seed=4)
    D, w = oracle_lib.mu_dm(H, 0.3)
    assert np.array_equal(np.diag(D), (np.diag(H) < 0.3).astype(float))
    assert np.abs(D - np.diag(np.diag(D))).max() == 0.0
    # [[a, c], [c, b]]: occupied eigenvector (cos t, sin t) with tan 2t = 2c/(a-b)
    a, b, c = 1.0, -0.5, 0.4
    t = 0.5 * np.arctan2(2 * c, a - b) + np.pi / 2      # the lower eigenvector
    v = np.array([np.cos(t), np.sin(t)])
    D2, w2 = oracle_lib.mu_dm(np.array([[a, c], [c, b]]), 0.0)
    assert np.allclose(D2, np.outer(v, v), atol=1e-14)
    with pytest.raises(oracle_lib.DegenerateError):
        oracle_lib.mu_dm(np.diag([-1.0, 0.0, 1.0]), 0.0)


def test_graph_density_zero_threshold_is_the_full_solve(oracle_lib):
    """tau = 0 joins every pair of nodes: every part is the whole matrix and
    the mapped-back rows assemble the full density matrix."""
    H, _ = gapped_random_hamiltonian(24, 11, gap=1.0, seed=3)
    D, sizes = oracle_lib.graph_density(H, 0.0, 4, 0.0)
    Dfull, _ = oracle_lib.mu_dm(H, 0.0)
    assert list(sizes) == [24] * 4
    assert np.abs(D - Dfull).max() < 1e-13


def test_graph_density_decoupled_blocks_are_exact(oracle_lib):
    """H block-diagonal on the core segments: each part is its own block and
    the result is the exact density matrix; the parts' sizes are the cores."""
    rng = np.random.default_rng(9)
    n, parts = 30, 3
    H = np.zeros((n, n))
    st = oracle_lib.segment_starts(n, parts)
    for k in range(parts):
        m = st[k + 1] - st[k]
        A = rng.standard_normal((m, m))
        H[st[k]:st[k + 1], st[k]:st[k + 1]] = A + A.T
    D, sizes = oracle_lib.graph_density(H, 1e-12, parts, 0.05)
    Dfull, _ = oracle_lib.mu_dm(H, 0.05)
    assert list(sizes) == [10, 10, 10]
    assert np.abs(D - Dfull).max() < 1e-13


def test_graph_density_local_model(oracle_lib):
    """The local gapped model (n = 256): each part's mapped-back rows are the
    rows of the projector of its sub-matrix (LAPACK), the error against the
    full projector shrinks as the threshold drops, and the occupation of the
    assembled D is n/2."""
    from tbgen import make_local_hamiltonian
    inst = make_local_hamiltonian(256, seed=2)
    H, n, parts = inst.H, 256, 4
    Dfull, _ = oracle_lib.mu_dm(H, inst.mu)
    errs = []
    for tau in (0.3, 0.1, 0.03):
        D, sizes = oracle_lib.graph_density(H, tau, parts, inst.mu)
        member = oracle_lib.graph_parts(H, tau, parts)
        assert list(sizes) == list(member.sum(1))
        st = oracle_lib.segment_starts(n, parts)
        for k in range(parts):
            nodes = np.nonzero(member[k])[0]
            w, V = np.linalg.eigh(H[np.ix_(nodes, nodes)])
            P = V[:, w < inst.mu] @ V[:, w < inst.mu].T
            core = np.arange(st[k], st[k + 1])
            want = np.zeros((core.size, n))
            want[:, nodes] = P[np.searchsorted(nodes, core)]
            assert np.abs(D[core] - want).max() < 1e-11
        errs.append(np.linalg.norm(D - Dfull) / n)
        assert abs(np.trace(D) - n / 2) < 0.05 * n
    assert errs[0] > errs[1] > errs[2]


# ---------------------------------------------------------------- thresholded SP2

def test_sp2_thresh_zero_threshold_is_sp2(oracle_lib):
    """tau = 0 never drops an entry: the thresholded loop is plain SP2, bit
    for bit (iterations, branches, D)."""
    inst = make_tb_hamiltonian(64, seed=12)
    a = oracle_lib.sp2(inst.H, inst.n_occ)
    b = oracle_lib.sp2_thresh(inst.H, inst.n_occ, 0.0)
    assert a.iterations == b.iterations and a.branch_mask == b.branch_mask
    assert np.array_equal(a.D, b.D) and b.margin == 1.0


def test_sp2_thresh_hand_worked_2x2(oracle_lib):
    """H = [[-1, 0.01], [0.01, 1]], n_occ = 1, tau = 0.01, worked by hand:
    Gershgorin [-1.01, 1.01], X_0 = (1.01 I - H)/2.02 has trace 1 (a tie:
    2X - X^2) and off-diagonal -0.01/2.02; the product's off-diagonal
    x01 (x00 + x11) = -0.01/2.02 is dropped, and so is 2 x01 - 0 =
    -0.0099 < tau.  X is diagonal from then on and converges to diag(1, 0)
    (the exact projector has off-diagonal entries of about -0.005)."""
    H = np.array([[-1.0, 0.01], [0.01, 1.0]])
    r = oracle_lib.sp2_thresh(H, 1, 0.01)
    assert r.status == 0 and r.branches()[0] == 1
    assert np.abs(r.D - np.diag([1.0, 0.0])).max() < 1e-9
    assert r.D[0, 1] == 0.0 and r.D[1, 0] == 0.0
    exact = oracle_lib.sp2(H, 1)
    assert abs(exact.D[0, 1] + 0.005) < 2e-4


def test_sp2_thresh_error_follows_tau(oracle_lib):
    """On the local model the thresholded D approaches plain SP2's as tau
    falls.  Dropping entries puts a floor of about tau under the idempotency,
    so with tol = 1e-10 the loop ends by the stagnation rule, at e of order
    tau; the entries dropped shrink with tau."""
    from tbgen import make_local_hamiltonian
    inst = make_local_hamiltonian(128, seed=5)
    ref = oracle_lib.sp2(inst.H, inst.n_occ)
    errs, zeros = [], []
    for tau in (1e-3, 1e-5, 1e-7):
        r = oracle_lib.sp2_thresh(inst.H, inst.n_occ, tau, nthreads=4)
        assert r.status == oracle_lib.STAGNATED and r.idempotency < 100 * tau
        errs.append(np.linalg.norm(r.D - ref.D) / np.sqrt(128))
        zeros.append(int((r.D == 0).sum()))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6
    assert zeros[0] > zeros[1] > zeros[2]
