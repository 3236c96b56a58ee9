"""GPU parity of thresholded SP2 with tile skipping (sp2_density_sparse).

The oracle (oracle_sp2_thresh) runs the SP2 listing with its cutoff tau:
the product and the 2X - X^2 update drop every entry with |x| < tau.  The
GPU path must reproduce it: same status, iterations and branches, and D
within FP64 rounding, whenever no drop decision sits on the threshold (the
oracle reports the closest one; the cases below keep it well away).  With
tau = 0 the path is plain FP64 SP2.
"""
import numpy as np
import pytest

from tbgen import gapped_random_hamiltonian, make_local_hamiltonian, make_tb_hamiltonian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_13772_amd as m
    return m


@pytest.mark.parametrize("n", [300, 1100])
def test_tau_zero_is_plain_sp2(sp2, oracle_lib, n):
    if n % 4 == 0:
        inst = make_tb_hamiltonian(n, seed=n)
        H, n_occ = inst.H, inst.n_occ
    else:
        H, _ = gapped_random_hamiltonian(n, n // 2, gap=1.0, seed=n)
        n_occ = n // 2
    print(f"[gpu] sparse tau=0 n={n}", flush=True)
    Hg = torch.from_numpy(H).cuda()
    nbytes = sp2.sp2_sparse_workspace_size(n)
    raw = torch.empty(nbytes + sp2.WORKSPACE_ALIGN, dtype=torch.uint8, device="cuda")
    off = (-raw.data_ptr()) % sp2.WORKSPACE_ALIGN
    ws = raw[off:off + nbytes]
    D, info = sp2.sp2_density_sparse(Hg, n_occ, 0.0, workspace=ws)
    ref = oracle_lib.sp2(H, n_occ, nthreads=8)
    assert info.status == ref.status == 0 and info.iterations == ref.iterations
    # branches agree wherever the trace decides them (|tr - n_occ| > 1e-9 n);
    # a near-tie may go either way under a different summation order
    tr, e = sp2.sp2_history(ws, info.iterations)
    decided = np.abs(np.asarray(ref.tr_hist) - n_occ) > 1e-9 * n
    assert np.array_equal(np.asarray(info.branches())[decided], np.asarray(ref.branches())[decided])
    assert np.abs(tr - ref.tr_hist).max() <= 1e-9 * n
    assert np.abs(D.cpu().numpy() - ref.D).max() <= 1e-11


@pytest.mark.parametrize("n,tau", [(512, 1e-5), (512, 1e-3), (1000, 1e-6)])
def test_matches_thresholded_oracle(sp2, oracle_lib, n, tau):
    if n % 4 == 0:
        inst = make_local_hamiltonian(n, seed=n + 1)
        H, n_occ = inst.H, inst.n_occ
    else:
        inst = make_local_hamiltonian(1000, seed=9)
        H, n_occ = inst.H, inst.n_occ
    ref = oracle_lib.sp2_thresh(H, n_occ, tau, nthreads=8)
    assert ref.margin > 1e-9, "a drop decision sits on the threshold; pick another seed"
    print(f"[gpu] sparse n={n} tau={tau}: oracle {ref.iterations} steps, status {ref.status}", flush=True)
    D, info = sp2.sp2_density_sparse(torch.from_numpy(H).cuda(), n_occ, tau)
    Dg = D.cpu().numpy()
    assert info.status == ref.status and info.iterations == ref.iterations
    assert info.branch_mask == ref.branch_mask
    assert abs(info.idempotency - ref.idempotency) <= 1e-9 * max(1.0, ref.idempotency)
    assert np.abs(Dg - ref.D).max() <= 1e-10
    assert np.array_equal(Dg == 0, ref.D == 0)        # the same entries dropped
    assert np.array_equal(Dg, Dg.T)


def test_local_model_skips_tiles(sp2, oracle_lib):
    """n = 4096 local model, tau = 1e-5: entries of D are dropped (whole
    128-tiles where the local model allows), D is bitwise symmetric, its trace
    and idempotency are within the threshold's reach, and it is close to plain
    FP64 SP2."""
    n, tau = 4096, 1e-5
    inst = make_local_hamiltonian(n, seed=4, dtype=np.float32)
    H = torch.from_numpy(inst.H).cuda()
    print(f"[gpu] sparse local n={n} tau={tau}", flush=True)
    D, info = sp2.sp2_density_sparse(H, inst.n_occ, tau)
    Dd, idense = sp2.sp2_density(H, inst.n_occ)
    assert info.status in (0, sp2.STAGNATED) and idense.status == 0
    Dg = D.double()
    T = n // 128
    tiles = Dg.reshape(T, 128, T, 128).abs().amax(dim=(1, 3))
    zero_frac = float((tiles == 0).double().mean())
    err = float(torch.linalg.norm(Dg - Dd.double())) / np.sqrt(n)
    print(f"[gpu]   {info.iterations} steps, zero tiles {zero_frac:.2f}, rms vs dense {err:.2e}, "
          f"e {info.idempotency:.2e}", flush=True)
    assert int((Dg == 0).sum()) > n * n // 4
    assert torch.equal(D, D.T)
    assert abs(info.trace - inst.n_occ) < 1e-2 and info.idempotency < 1e-2
    assert err < 1e-3
