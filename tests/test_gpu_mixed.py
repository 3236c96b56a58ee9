"""GPU parity of the mixed-precision schedule (split-operand 16-bit products).

Bars.  The method's accuracy bar is rms |D - D_ref| <= 1e-6 against the
eigenvector definition of D (the oracle's Jacobi projector, or LAPACK at sizes
the Jacobi oracle is too slow for); F16X2 and BF16X3 must meet it with the
automatic FP64 prefix.  BF16X2 (16-bit operands) cannot: its test reports the
floor it reaches and checks convergence of the FP64 refinement and a loose
1e-3.

A single split-operand step is checked entry by entry against the oracle's
FP64 step: operands are represented to ~2^-22 relative (F16X2 hi + lo, BF16X3
three planes) and products accumulate in FP32, so we bound the entry error by
2^-18 * sum_k |x_ik||x_kj| + 1e-9 (well above the rounding level, far below
any indexing or layout error, which is O(1)).
"""
import numpy as np
import pytest

from tbgen import gapped_random_hamiltonian, make_tb_hamiltonian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MODES = ["f16x2", "bf16x3"]


@pytest.fixture(scope="module")
def sp2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_13772_amd as m
    return m


def rms(A):
    return float(np.linalg.norm(A) / np.sqrt(A.shape[0]))


def solve(sp2, H, n_occ, **kw):
    print(f"[gpu] mixed n={H.shape[0]} {kw}", flush=True)
    Ht = torch.from_numpy(np.ascontiguousarray(H)).cuda()
    D, info = sp2.sp2_density(Ht, n_occ, **kw)
    torch.cuda.synchronize()
    return D.cpu().numpy().astype(np.float64), info


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [128, 256])
def test_mixed_meets_accuracy_bar(sp2, oracle_lib, mode, n):
    inst = make_tb_hamiltonian(n, seed=100 + n)
    D, info = solve(sp2, inst.H, inst.n_occ, compute=mode)
    Dj, w, _ = oracle_lib.jacobi_dm(inst.H, inst.n_occ)
    assert info.status == 0, info
    assert info.fp64_prefix_iters >= 1
    assert 1 <= info.refine_steps <= 8
    assert info.iterations > info.fp64_prefix_iters + info.refine_steps   # split steps happened
    assert info.idempotency <= 1e-10
    assert abs(info.trace - inst.n_occ) < 1e-8
    assert rms(D - Dj) <= 1e-6
    assert np.abs(D - D.T).max() == 0.0


@pytest.mark.parametrize("n,n_occ", [(200, 77), (257, 128), (384, 200)])
def test_mixed_ragged(sp2, oracle_lib, n, n_occ):
    H, _ = gapped_random_hamiltonian(n, n_occ, gap=1.0, seed=n)
    D, info = solve(sp2, H, n_occ, compute="f16x2")
    w, V = np.linalg.eigh(H)
    Dref = V[:, :n_occ] @ V[:, :n_occ].T
    assert info.status == 0
    assert rms(D - Dref) <= 1e-6


def test_bf16x2_reports_its_floor(sp2, oracle_lib):
    inst = make_tb_hamiltonian(256, seed=3)
    D, info = solve(sp2, inst.H, inst.n_occ, compute="bf16x2")
    Dj, _, _ = oracle_lib.jacobi_dm(inst.H, inst.n_occ)
    err = rms(D - Dj)
    print(f"[gpu] bf16x2 floor: rms |D - D_jacobi| = {err:.3e}", flush=True)
    assert info.status in (0, 2)
    assert err <= 1e-3


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [256, 1028])
def test_single_split_step_entries(sp2, oracle_lib, mode, n):
    """m0 = 1, max_iter = 2: one FP64 step, then one split-operand step."""
    inst = make_tb_hamiltonian(n, seed=7)
    H = inst.H
    D2, info = solve(sp2, H, inst.n_occ, compute=mode, fp64_prefix_iters=1, max_iter=2)
    assert info.status == 1 and info.iterations == 2 and info.fp64_prefix_iters == 1
    r1 = oracle_lib.sp2(H, inst.n_occ, max_iter=1)
    X1 = r1.D
    grow = int(np.trace(X1) - inst.n_occ <= 0)
    assert info.branches() == [r1.branches()[0], grow]
    rng = np.random.default_rng(2)
    I = np.concatenate([rng.integers(0, n, 3000), np.arange(n), np.arange(n)])
    J = np.concatenate([rng.integers(0, n, 3000), np.arange(n), np.arange(n)[::-1]])
    want = oracle_lib.sp2_step_entries(X1, grow, I, J)
    absX = np.abs(X1)
    bound = 2.0 ** -18 * np.einsum("tk,tk->t", absX[I], absX[J]) + 1e-9
    assert np.all(np.abs(D2[I, J] - want) <= bound)
    assert np.array_equal(D2, D2.T)


@pytest.mark.parametrize("mode", ["f16x2", "bf16x3", "fp8"])
def test_split_step_entries_every_tile_split(sp2, oracle_lib, mode):
    """n = 2176 (17 x 17 tiles of 128, 153 lower tiles): fewer tiles than the
    step kernels' workgroups, so every tile of the FP64 step and of the
    split-operand step is a stream-K remainder tile, finished by the step-end
    kernel from its workgroups' FP64 partials (planes of 2 bytes or, for FP8,
    1 byte).  One FP64 step, then one split-operand step, entry by entry,
    including whole tile rows at the tile edges."""
    n = 2176
    inst = make_tb_hamiltonian(n, seed=5)
    D2, info = solve(sp2, inst.H, inst.n_occ, compute=mode, fp64_prefix_iters=1, max_iter=2)
    assert info.status == 1 and info.iterations == 2 and info.fp64_prefix_iters == 1
    r1 = oracle_lib.sp2(inst.H, inst.n_occ, max_iter=1)
    X1 = r1.D
    grow = int(np.trace(X1) - inst.n_occ <= 0)
    assert info.branches() == [r1.branches()[0], grow]
    rng = np.random.default_rng(4)
    edge = np.concatenate([np.arange(120, 136), np.arange(n - 16, n)])
    I = np.concatenate([rng.integers(0, n, 3000), np.repeat(edge, 64), np.arange(n)])
    J = np.concatenate([rng.integers(0, n, 3000), np.tile(rng.integers(0, n, 64), edge.size), np.arange(n)[::-1]])
    want = oracle_lib.sp2_step_entries(X1, grow, I, J)
    absX = np.abs(X1)
    scale, floor = (2.0 ** -6, 1e-6) if mode == "fp8" else (2.0 ** -18, 1e-9)
    bound = scale * np.einsum("tk,tk->t", absX[I], absX[J]) + floor
    assert np.all(np.abs(D2[I, J] - want) <= bound)
    assert np.array_equal(D2, D2.T)


@pytest.mark.parametrize("mode", MODES)
def test_mixed_fullsize_split_tiles(sp2, mode):
    """n = 4096, FP32 storage: the bench workload, stream-K split tiles in both
    the FP64 and the split-operand kernels."""
    inst = make_tb_hamiltonian(4096, seed=0, dtype=np.float32)
    Ht = torch.from_numpy(inst.H).cuda()
    print(f"[gpu] mixed fullsize {mode}", flush=True)
    D, info = sp2.sp2_density(Ht, inst.n_occ, compute=mode)
    assert info.status == 0, info
    w, V = np.linalg.eigh(inst.H.astype(np.float64))
    Dref = torch.from_numpy(V[:, :2048] @ V[:, :2048].T).cuda()
    err = float(torch.linalg.norm(D.double() - Dref)) / 64.0
    assert err <= 1e-6
    D2, _ = sp2.sp2_density(Ht, inst.n_occ, compute=mode)
    assert torch.equal(D, D2)


def test_mixed_special_cases(sp2):
    inst = make_tb_hamiltonian(64, seed=2)
    D0, i0 = solve(sp2, inst.H, 0, compute="f16x2")
    assert i0.status == 0 and not D0.any()
    Dn, iN = solve(sp2, inst.H, 64, compute="f16x2")
    assert iN.status == 0 and np.array_equal(Dn, np.eye(64))
    # a max_iter that ends inside the split phase returns the decoded planes
    D, info = solve(sp2, inst.H, 32, compute="f16x2", fp64_prefix_iters=3, max_iter=6)
    assert info.status == 1 and info.iterations == 6
    assert np.isfinite(D).all() and np.array_equal(D, D.T)


def test_fp8_reports_its_floor(sp2, oracle_lib):
    """Two e4m3 planes (~8 bits): the FP64 prefix and refinement converge, and
    the subspace error is reported (a BF16X2-class floor, far above 1e-6)."""
    inst = make_tb_hamiltonian(256, seed=3)
    D, info = solve(sp2, inst.H, inst.n_occ, compute="fp8")
    Dj, _, _ = oracle_lib.jacobi_dm(inst.H, inst.n_occ)
    err = rms(D - Dj)
    print(f"[gpu] fp8 floor: rms |D - D_jacobi| = {err:.3e}", flush=True)
    assert info.status in (0, 2)
    assert info.idempotency < 1e-6
    assert err <= 1e-2


@pytest.mark.parametrize("n", [256, 1028])
def test_single_fp8_step_entries(sp2, oracle_lib, n):
    """One FP64 step, then one FP8X2 step, entry by entry: operands carry ~2^-8
    relative, so the bound is 2^-6 sum_k |x_ik||x_kj| + 1e-6 (an indexing or
    layout error is O(1))."""
    inst = make_tb_hamiltonian(n, seed=7)
    D2, info = solve(sp2, inst.H, inst.n_occ, compute="fp8", fp64_prefix_iters=1, max_iter=2)
    assert info.status == 1 and info.iterations == 2
    r1 = oracle_lib.sp2(inst.H, inst.n_occ, max_iter=1)
    X1 = r1.D
    grow = int(np.trace(X1) - inst.n_occ <= 0)
    rng = np.random.default_rng(3)
    I = np.concatenate([rng.integers(0, n, 3000), np.arange(n)])
    J = np.concatenate([rng.integers(0, n, 3000), np.arange(n)])
    want = oracle_lib.sp2_step_entries(X1, grow, I, J)
    absX = np.abs(X1)
    bound = 2.0 ** -6 * np.einsum("tk,tk->t", absX[I], absX[J]) + 1e-6
    assert np.all(np.abs(D2[I, J] - want) <= bound)
    assert np.array_equal(D2, D2.T)
