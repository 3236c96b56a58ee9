"""GPU parity: the HIP SP2 path (through the C ABI) against the FP64 CPU oracle.

Tolerances.  The FP64 path and the oracle run the same recursion in IEEE
double with different summation orders, so they agree to rounding noise
amplified by the loop: we require |D_gpu - D_oracle| rms <= 1e-11 and the
error against the eigenvector definition <= 1e-10 rms (the stop tolerance is
1e-10 on ||X^2 - X||_F).  The accuracy bar of the method is 1e-6 rms; these
bars are four orders tighter.  Iteration counts must be equal, and branches
equal wherever |tr - n_occ| > 1e-9 n (elsewhere both choices are correct up
to rounding).
"""
import numpy as np
import pytest

from tbgen import (diagonal_hamiltonian, gapped_random_hamiltonian, make_tb_hamiltonian,
                   two_level_hamiltonian)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_13772_amd as m
    return m


def rms(A):
    return float(np.linalg.norm(A) / np.sqrt(A.shape[0]))


def run_gpu(sp2, H, n_occ, **kw):
    print(f"[gpu] sp2_density n={H.shape[0]} n_occ={n_occ} dtype={H.dtype} {kw}", flush=True)
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda()
    D, info = sp2.sp2_density(Ht, n_occ, **kw)
    torch.cuda.synchronize()
    return D.cpu().numpy().astype(np.float64), info


def check_against_oracle(sp2, oracle_lib, H, n_occ, jacobi=True):
    n = H.shape[0]
    Dg, info = run_gpu(sp2, H, n_occ)
    ref = oracle_lib.sp2(H.astype(np.float64), n_occ, tol=1e-10)
    assert info.status == ref.status == 0, (info, ref.status)
    assert info.iterations == ref.iterations
    lo, hi = oracle_lib.gershgorin(H.astype(np.float64))
    assert info.emin == pytest.approx(lo, rel=1e-13, abs=1e-13)
    assert info.emax == pytest.approx(hi, rel=1e-13, abs=1e-13)
    tr = np.asarray(ref.tr_hist)
    decided = np.abs(tr - n_occ) > 1e-9 * n
    assert np.array_equal(np.array(info.branches())[decided], np.array(ref.branches())[decided])
    tol_d = 1e-11 if H.dtype == np.float64 else 1e-7
    assert rms(Dg - ref.D) <= tol_d
    if jacobi:
        Dj, _, _ = oracle_lib.jacobi_dm(H.astype(np.float64), n_occ)
        assert rms(Dg - Dj) <= (1e-10 if H.dtype == np.float64 else 1e-7)
    assert abs(info.trace - n_occ) < 1e-8
    return Dg, info, ref


@pytest.mark.parametrize("n", [4, 16, 64, 128, 256])
def test_tb_fp64_matches_oracle(sp2, oracle_lib, n):
    inst = make_tb_hamiltonian(n, seed=n, gap=0.5)
    check_against_oracle(sp2, oracle_lib, inst.H, inst.n_occ, jacobi=n <= 256)


@pytest.mark.parametrize("n,n_occ", [(2, 1), (3, 1), (37, 18), (100, 61), (127, 64), (129, 40),
                                     (191, 95), (255, 128), (257, 100)])
def test_ragged_sizes_fp64(sp2, oracle_lib, n, n_occ):
    H, _ = gapped_random_hamiltonian(n, n_occ, gap=0.8, seed=n)
    check_against_oracle(sp2, oracle_lib, H, n_occ, jacobi=n <= 200)


@pytest.mark.parametrize("n", [128, 260])
def test_tb_fp32_storage(sp2, oracle_lib, n):
    inst = make_tb_hamiltonian(n, seed=7, gap=0.5, dtype=np.float32)
    Dg, info, ref = check_against_oracle(sp2, oracle_lib, inst.H, inst.n_occ, jacobi=False)


def test_golden_2x2_tie(sp2):
    import golden
    g = golden.load("dm_2x2_tie.txt")
    Dg, info = run_gpu(sp2, g["H"], 1)
    assert info.status == 0
    assert info.branches()[0] == 1                     # tr X0 == 1 exactly: tie -> 2X - X^2
    assert (info.emin, info.emax) == (g["emin"], g["emax"])
    assert np.abs(Dg - g["D"]).max() < 1e-10
    D1, i1 = run_gpu(sp2, g["H"], 1, max_iter=1)
    assert i1.status == 1 and i1.iterations == 1
    w = np.linalg.eigvalsh(D1)
    assert np.abs(np.sort(w) - np.sort(g["x_after_first_step"])).max() < 1e-15


@pytest.mark.parametrize("n", [7, 64, 150])
def test_diagonal_bitwise(sp2, oracle_lib, n):
    """SP2 on a diagonal H is entrywise: GPU and oracle must agree bit for bit."""
    Hd = diagonal_hamiltonian(n, seed=n)
    n_occ = n // 3 + 1
    Dg, info = run_gpu(sp2, Hd, n_occ)
    ref = oracle_lib.sp2(Hd, n_occ)
    assert info.status == ref.status == 0
    assert info.iterations == ref.iterations
    assert info.branch_mask == ref.branch_mask
    assert np.array_equal(Dg, ref.D)


def test_two_level(sp2, oracle_lib):
    H, P = two_level_hamiltonian(96, 30, alpha=-2.0, beta=1.5, seed=3)
    Dg, info = run_gpu(sp2, H, 30)
    ref = oracle_lib.sp2(H, 30)
    assert info.iterations == ref.iterations and info.status == 0
    assert np.abs(Dg - P).max() < 1e-9


def test_history_matches_oracle(sp2, oracle_lib):
    inst = make_tb_hamiltonian(128, seed=21)
    Ht = torch.from_numpy(inst.H).cuda()
    ws = sp2.alloc_workspace(128)
    D, info = sp2.sp2_density(Ht, inst.n_occ, workspace=ws)
    tr, e = sp2.sp2_history(ws)
    ref = oracle_lib.sp2(inst.H, inst.n_occ)
    assert len(tr) == info.iterations == ref.iterations
    assert np.abs(tr - ref.tr_hist).max() < 1e-9 * 128
    big = np.asarray(ref.e_hist) > 1e-6
    assert np.allclose(e[big], np.asarray(ref.e_hist)[big], rtol=1e-9)


def test_special_cases(sp2):
    inst = make_tb_hamiltonian(64, seed=2)
    D0, i0 = run_gpu(sp2, inst.H, 0)
    assert i0.status == 0 and i0.iterations == 0 and not D0.any()
    Dn, iN = run_gpu(sp2, inst.H, 64)
    assert iN.status == 0 and np.array_equal(Dn, np.eye(64))
    # H = c I with 0 < n_occ < n has no unique density matrix; D stays untouched
    Hc = torch.full((16, 16), 0.0, dtype=torch.float64, device="cuda")
    Hc.fill_diagonal_(3.0)
    Dt = torch.full((16, 16), 7.0, dtype=torch.float64, device="cuda")
    _, ic = sp2.sp2_density(Hc, 5, D=Dt)
    assert ic.status == sp2.E_DEGENERATE and bool((Dt == 7.0).all())
    Hn = torch.from_numpy(inst.H).cuda()
    Hn[3, 9] = float("nan")
    Dt = torch.full((64, 64), 7.0, dtype=torch.float64, device="cuda")
    _, inan = sp2.sp2_density(Hn, 32, D=Dt)
    assert inan.status == sp2.E_INVALID and bool((Dt == 7.0).all())
    D1, i1 = run_gpu(sp2, inst.H, 32, max_iter=1)
    assert i1.status == sp2.NOT_CONVERGED and i1.iterations == 1
    Dm0, im0 = run_gpu(sp2, inst.H, 32, max_iter=0)
    assert im0.status == sp2.NOT_CONVERGED and im0.iterations == 0
    Ds, ist = run_gpu(sp2, inst.H, 32, tol=1e-300)
    assert ist.status == sp2.STAGNATED
    assert np.linalg.norm(Ds @ Ds - Ds) < 1e-11


def test_leading_dimension_and_determinism(sp2, oracle_lib):
    inst = make_tb_hamiltonian(96, seed=4)
    big = torch.zeros((96, 131), dtype=torch.float64, device="cuda")
    big[:, :96] = torch.from_numpy(inst.H).cuda()
    big[:, 96:] = float("nan")                         # never read: outside the n x n view
    Hv = big[:, :96]
    D1, i1 = sp2.sp2_density(Hv, inst.n_occ)
    D2, i2 = sp2.sp2_density(Hv, inst.n_occ)
    assert D1.stride(0) == 131
    assert i1.status == 0 and torch.equal(D1, D2)      # bitwise reproducible
    ref = oracle_lib.sp2(inst.H, inst.n_occ)
    assert rms(D1.cpu().numpy() - ref.D) < 1e-11


def test_one_step_sampled_entries(sp2, oracle_lib):
    """X_1 at a size spanning many tiles, checked entry by entry."""
    inst = make_tb_hamiltonian(1028, seed=5, dtype=np.float32)
    H64 = inst.H.astype(np.float64)
    D1, i1 = run_gpu(sp2, H64, inst.n_occ, max_iter=1)
    lo, hi = oracle_lib.gershgorin(H64)
    X0 = oracle_lib.sp2_init(H64, lo, hi)
    grow = int(np.trace(X0) - inst.n_occ <= 0)
    assert i1.branches() == [grow]
    rng = np.random.default_rng(0)
    I = rng.integers(0, 1028, 4000)
    J = rng.integers(0, 1028, 4000)
    want = oracle_lib.sp2_step_entries(X0, grow, I, J)
    assert np.abs(D1[I, J] - want).max() < 1e-14


def _oracle_threads():
    import os
    return max(1, min(16, len(os.sched_getaffinity(0))))


def test_bt128_full_solve_matches_oracle(sp2, oracle_lib):
    """n = 2052: the 128 x 128-tile squaring kernel (8 waves) with its fused
    epilogue sums and device steering, over a whole solve, against the oracle
    (paper: Section "SP2 solver", recursion and listing): iteration count,
    every branch, the trace and idempotency histories, info.idempotency and D."""
    n = 2052
    inst = make_tb_hamiltonian(n, seed=31, gap=0.5)
    print(f"[gpu] bt128 full solve n={n}", flush=True)
    Ht = torch.from_numpy(inst.H).cuda()
    ws = sp2.alloc_workspace(n)
    D, info = sp2.sp2_density(Ht, inst.n_occ, workspace=ws)
    tr, e = sp2.sp2_history(ws)
    Dg = D.cpu().numpy()
    ref = oracle_lib.sp2(inst.H, inst.n_occ, tol=1e-10, nthreads=_oracle_threads())
    assert info.status == ref.status == 0
    assert info.iterations == ref.iterations == len(tr)
    lo, hi = oracle_lib.gershgorin(inst.H)
    assert info.emin == pytest.approx(lo, rel=1e-13) and info.emax == pytest.approx(hi, rel=1e-13)
    # the branch is decided wherever the trace is not at n_occ to rounding
    # (on the converged last step it is, and either branch is then correct)
    decided = np.abs(np.asarray(ref.tr_hist) - inst.n_occ) > 1e-9 * n
    assert decided[:-1].all()
    assert np.array_equal(np.array(info.branches())[decided], np.array(ref.branches())[decided])
    assert np.abs(tr - ref.tr_hist).max() <= 1e-9 * n
    big = np.asarray(ref.e_hist) > 1e-6
    assert np.allclose(e[big], np.asarray(ref.e_hist)[big], rtol=1e-9)
    assert info.idempotency == pytest.approx(ref.idempotency, rel=0.5, abs=2e-11)
    assert info.idempotency <= 1e-10
    assert rms(Dg - ref.D) <= 1e-11
    assert abs(info.trace - ref.trace) <= 1e-9
    assert np.array_equal(Dg, Dg.T)


def test_split_tiles_three_steps_match_oracle(sp2, oracle_lib):
    """n = 3000: more 128 x 128 tiles than co-resident workgroups, so the
    stream-K schedule splits tiles between two workgroups.  Three whole steps
    (squaring, update, trace and norm sums, branch decisions) against the
    oracle, entry by entry."""
    n = 3000
    inst = make_tb_hamiltonian(n, seed=12, gap=0.5)
    print(f"[gpu] split tiles three steps n={n}", flush=True)
    Ht = torch.from_numpy(inst.H).cuda()
    ws = sp2.alloc_workspace(n)
    D, info = sp2.sp2_density(Ht, inst.n_occ, max_iter=3, workspace=ws)
    tr, e = sp2.sp2_history(ws)
    Dg = D.cpu().numpy()
    ref = oracle_lib.sp2(inst.H, inst.n_occ, max_iter=3, nthreads=_oracle_threads())
    assert info.status == ref.status == sp2.NOT_CONVERGED
    assert info.iterations == ref.iterations == 3
    assert info.branches() == ref.branches()
    assert np.abs(tr - ref.tr_hist).max() <= 1e-10 * n
    assert np.allclose(e, ref.e_hist, rtol=1e-12)
    assert np.abs(Dg - ref.D).max() <= 1e-13
    assert np.array_equal(Dg, Dg.T)
