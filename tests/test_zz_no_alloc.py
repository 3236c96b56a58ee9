"""sp2_density_noalloc (the entry point with the library's fixed per-GPU
workspace) against sp2_density on the same inputs.  Both run the same kernels
with the same launch shapes, so D and the info must agree bit for bit; two
calls in a row, the second on a smaller problem, check that the state left in
the shared array by one call does not leak into the next."""
import numpy as np
import pytest

from tbgen import make_tb_hamiltonian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_13772_amd as m
    return m


def same_info(a, b):
    return (a.status, a.iterations, a.fp64_prefix_iters, a.refine_steps, a.branch_mask, a.trace,
            a.idempotency, a.emin, a.emax) == (b.status, b.iterations, b.fp64_prefix_iters,
                                               b.refine_steps, b.branch_mask, b.trace, b.idempotency,
                                               b.emin, b.emax)


@pytest.mark.parametrize("compute,sizes", [("f64", (512, 260)), ("f16x2", (384, 128))])
def test_noalloc_matches_sp2_density(sp2, compute, sizes):
    for k, n in enumerate(sizes):
        inst = make_tb_hamiltonian(n, seed=40 + k, gap=0.5)
        print(f"[gpu] noalloc {compute} n={n}", flush=True)
        H = torch.from_numpy(inst.H).cuda()
        Dref, iref = sp2.sp2_density(H, inst.n_occ, compute=compute)
        D = torch.full_like(H, float("nan"))
        D, info = sp2.sp2_density_noalloc(H, inst.n_occ, D, compute=compute)
        torch.cuda.synchronize()
        assert iref.status == 0 and info.status == 0, (iref, info)
        assert same_info(info, iref), (info, iref)
        assert torch.equal(D, Dref)


def test_noalloc_rejects_sizes_beyond_its_array(sp2):
    assert sp2.sp2_workspace_size(2048, "f64", "f64") > sp2.NOALLOC_MAX_BYTES
    inst = make_tb_hamiltonian(2048, seed=3, gap=0.5)
    H = torch.from_numpy(inst.H).cuda()
    D = torch.full_like(H, 7.0)
    _, info = sp2.sp2_density_noalloc(H, inst.n_occ, D)
    assert info.status == sp2.E_WORKSPACE
    assert bool((D == 7.0).all())
    # a small call afterwards still works
    small = make_tb_hamiltonian(64, seed=5, gap=0.5)
    Hs = torch.from_numpy(small.H).cuda()
    Ds = torch.empty_like(Hs)
    _, i2 = sp2.sp2_density_noalloc(Hs, small.n_occ, Ds)
    Dr, ir = sp2.sp2_density(Hs, small.n_occ)
    assert i2.status == 0 and torch.equal(Ds, Dr)
