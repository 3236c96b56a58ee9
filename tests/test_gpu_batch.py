"""GPU parity of the batched plan (sp2_plan_create / sp2_plan_run).

The plan solves many independent problems (the per-part dense solves of the
paper's graph-partitioned workflow, Section "Graph-based Divide electronic
structure") in one graph replay.  With the default tile shape it runs the
single-matrix kernels' tile code in the same summation orders, so each D and
each info must equal the matrix's own sp2_density result bit for bit; a
sample is also checked against the FP64 oracle (paper: Section "SP2
solver").  With an autotuned tile shape the rounding order may differ: D is
then checked against the oracle at the FP64 bar (rms <= 1e-11).
"""
import numpy as np
import pytest

from tbgen import batch_sizes, gapped_random_hamiltonian, make_tb_hamiltonian

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


def mixed_batch(sizes, seed0, dtype=np.float64):
    Hs, nocc = [], []
    for k, n in enumerate(sizes):
        if n % 4 == 0:
            inst = make_tb_hamiltonian(int(n), seed=seed0 + k, gap=0.5, dtype=dtype)
            Hs.append(inst.H)
            nocc.append(inst.n_occ)
        else:
            H, _ = gapped_random_hamiltonian(int(n), int(n) // 2, gap=0.8, seed=seed0 + k)
            Hs.append(H.astype(dtype))
            nocc.append(int(n) // 2)
    return Hs, nocc


def same_info(a, b):
    return (a.status, a.iterations, a.branch_mask, a.trace, a.idempotency, a.emin, a.emax) == (
        b.status, b.iterations, b.branch_mask, b.trace, b.idempotency, b.emin, b.emax)


def test_plan_bitwise_equals_single_solves(sp2, oracle_lib):
    sizes = [64, 512, 37, 128, 200, 100, 260, 64, 388, 4, 129, 300]
    Hs, nocc = mixed_batch(sizes, 500)
    print(f"[gpu] plan bitwise, sizes {sizes}", flush=True)
    Ht = [torch.from_numpy(H).cuda() for H in Hs]
    plan = sp2.Plan(sizes, nocc)
    assert plan.config == "bt64w4"
    Ds, infos = plan.run(Ht)
    torch.cuda.synchronize()
    for k, n in enumerate(sizes):
        D1, i1 = sp2.sp2_density(Ht[k], nocc[k])
        assert infos[k].status == 0 and same_info(infos[k], i1), (k, n, infos[k], i1)
        assert torch.equal(Ds[k], D1), (k, n)
    for k in (1, 2, 6):
        ref = oracle_lib.sp2(Hs[k], nocc[k])
        assert infos[k].iterations == ref.iterations
        assert rms(Ds[k].cpu().numpy() - ref.D) <= 1e-11
    # a second run of the same plan on the same inputs is bitwise identical
    Ds2, infos2 = plan.run(Ht)
    assert all(torch.equal(a, b) for a, b in zip(Ds, Ds2))
    plan.close()


def test_plan_special_and_degenerate_members(sp2):
    inst = make_tb_hamiltonian(64, seed=9)
    Hc = np.eye(32) * 3.0
    # non-finite members: a NaN in the only tile pair of an n = 64 matrix, an
    # Inf in tile pair (2, 0) of an n = 160 matrix (a later pair item)
    Hnan = inst.H.copy()
    Hnan[3, 9] = float("nan")
    Hinf = make_tb_hamiltonian(160, seed=10).H.copy()
    Hinf[150, 20] = float("inf")
    Hs = [inst.H, inst.H, Hc, inst.H, Hnan, Hinf]
    nocc = [0, 64, 10, 32, 32, 80]
    Ht = [torch.from_numpy(H).cuda() for H in Hs]
    Ds = [torch.full_like(h, 7.0) for h in Ht]
    plan = sp2.Plan([64, 64, 32, 64, 64, 160], nocc)
    Ds, infos = plan.run(Ht, Ds)
    assert infos[0].status == 0 and not Ds[0].any()
    assert infos[1].status == 0 and torch.equal(Ds[1], torch.eye(64, dtype=torch.float64, device="cuda"))
    assert infos[2].status == sp2.E_DEGENERATE and bool((Ds[2] == 7.0).all())
    assert infos[3].status == 0
    for k in (4, 5):
        assert infos[k].status == sp2.E_INVALID and bool((Ds[k] == 7.0).all()), k
    assert plan.last_status == sp2.E_DEGENERATE   # the most negative member status
    plan.close()


def test_plan_fp32_storage_against_oracle(sp2, oracle_lib):
    sizes = [256, 68, 412, 132]
    Hs, nocc = mixed_batch(sizes, 700, dtype=np.float32)
    print(f"[gpu] plan fp32 storage {sizes}", flush=True)
    Ht = [torch.from_numpy(H).cuda() for H in Hs]
    plan = sp2.Plan(sizes, nocc, dtype="f32")
    Ds, infos = plan.run(Ht)
    for k in range(len(sizes)):
        ref = oracle_lib.sp2(Hs[k].astype(np.float64), nocc[k])
        assert infos[k].status == 0 and infos[k].iterations == ref.iterations
        assert rms(Ds[k].cpu().numpy().astype(np.float64) - ref.D) <= 1e-7   # FP32 output
    plan.close()


def test_plan_autotune_cache(sp2, oracle_lib, tmp_path):
    sizes = [int(v) for v in batch_sizes(40, seed=3, lo=64, hi=256)]
    Hs, nocc = mixed_batch(sizes, 900)
    print(f"[gpu] plan autotune, {len(sizes)} matrices", flush=True)
    Ht = [torch.from_numpy(H).cuda() for H in Hs]
    cache = tmp_path / "autotune.txt"
    plan = sp2.Plan(sizes, nocc, autotune_cache=str(cache))
    chosen = plan.config
    assert chosen in ("bt64w4", "bt32w1")
    lines = cache.read_text().split()
    assert len(lines) == 2 and lines[1] == chosen
    Ds, infos = plan.run(Ht)
    for k in (0, 5, 17, 39):
        ref = oracle_lib.sp2(Hs[k], nocc[k])
        assert infos[k].status == 0 and infos[k].iterations == ref.iterations
        assert rms(Ds[k].cpu().numpy() - ref.D) <= 1e-11
    plan.close()
    # a second plan with the same size mix reads the choice from the cache
    plan2 = sp2.Plan(sizes, nocc, autotune_cache=str(cache))
    assert plan2.config == chosen and cache.read_text().split() == lines
    plan2.close()
    # each tile shape, forced through the cache entry, against the oracle
    for shape in ("bt64w4", "bt32w1"):
        cache.write_text(f"{lines[0]} {shape}\n")
        plan3 = sp2.Plan(sizes, nocc, autotune_cache=str(cache))
        assert plan3.config == shape
        Ds, infos = plan3.run(Ht)
        for k in (1, 6, 23, 38):
            ref = oracle_lib.sp2(Hs[k], nocc[k])
            assert infos[k].status == 0 and infos[k].iterations == ref.iterations, (shape, k)
            assert rms(Ds[k].cpu().numpy() - ref.D) <= 1e-11, (shape, k)
        plan3.close()


def test_plan_config3_batch(sp2, oracle_lib):
    """512 problems with sizes uniform on {64, 68, ..., 512}, FP32 storage: the
    batched workload at its full size, in the launch configuration the
    benchmark times.  Every problem must converge; a sample is checked against
    the oracle and the rest against the projector properties."""
    sizes = [int(v) for v in batch_sizes(512, seed=0)]
    print("[gpu] plan config-3 batch: generating 512 Hamiltonians", flush=True)
    Hs, nocc = [], []
    for k, n in enumerate(sizes):
        inst = make_tb_hamiltonian(n, seed=10_000 + k, gap=0.5, dtype=np.float32)
        Hs.append(inst.H)
        nocc.append(inst.n_occ)
    Ht = [torch.from_numpy(H).cuda() for H in Hs]
    plan = sp2.Plan(sizes, nocc, dtype="f32")
    print("[gpu] plan config-3 batch: run", flush=True)
    Ds, infos = plan.run(Ht)
    assert all(i.status == 0 for i in infos)
    assert all(i.idempotency <= 1e-10 for i in infos)
    assert max(abs(i.trace - no) for i, no in zip(infos, nocc)) < 1e-8
    rng = np.random.default_rng(0)
    for k in rng.choice(512, 4, replace=False):
        ref = oracle_lib.sp2(Hs[k].astype(np.float64), nocc[k])
        assert infos[k].iterations == ref.iterations
        assert rms(Ds[k].cpu().numpy().astype(np.float64) - ref.D) <= 1e-7
    plan.close()
