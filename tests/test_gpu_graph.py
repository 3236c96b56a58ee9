"""GPU parity of the graph-partitioned solver (sp2_graph_*).

The parts (thresholded adjacency of G, regular core segments, one-hop
halos) must equal the oracle's exactly; D must match the oracle's graph
density matrix, whose per-part solves are Jacobi projectors at the chemical
potential mu (Section "Graph-based Divide electronic structure" with the
zero-temperature Fermi-Dirac function of Section "Single-particle density
matrix"), at the FP64 SP2 bar.  Each part's SP2 steps are steered by mu:
the branches must follow the scalar recursion of mu's image.
"""
import numpy as np
import pytest

from tbgen import gapped_random_hamiltonian, make_local_hamiltonian

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp2():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_13772_amd as m
    return m


def expected_branches(info, mu):
    """Branch bits of a mu-steered solve from its bounds: 2X - X^2 while mu's
    image is at or below 1/2, X^2 above, the image following the map."""
    x = (info.emax - mu) / (info.emax - info.emin)
    bits = []
    for _ in range(info.iterations):
        g = 1 if x <= 0.5 else 0
        bits.append(g)
        x = x * (2.0 - x) if g else x * x
    return bits


@pytest.mark.parametrize("n,parts,tau,dtype", [(512, 4, 0.3, "f64"), (512, 4, 0.05, "f64"),
                                               (300, 7, 0.1, "f32")])
def test_parts_match_oracle(sp2, oracle_lib, n, parts, tau, dtype):
    inst = make_local_hamiltonian(n, seed=n + parts, dtype=np.float64 if dtype == "f64" else np.float32)
    G = torch.from_numpy(inst.H).cuda()
    print(f"[gpu] graph parts n={n} parts={parts} tau={tau} {dtype}", flush=True)
    g = sp2.Graph(G, tau, parts)
    member = oracle_lib.graph_parts(inst.H.astype(np.float64), tau, parts)
    sizes, cores = g.sizes()
    st = oracle_lib.segment_starts(n, parts)
    assert cores == [st[k + 1] - st[k] for k in range(parts)]
    assert sizes == list(member.sum(1))
    for k in range(parts):
        assert g.nodes(k) == list(np.nonzero(member[k])[0])
    g.close()


@pytest.mark.parametrize("n,parts,tau", [(512, 4, 0.1), (300, 7, 0.05)])
def test_density_matches_oracle(sp2, oracle_lib, n, parts, tau):
    inst = make_local_hamiltonian(n, seed=7 * n + parts)
    H = torch.from_numpy(inst.H).cuda()
    print(f"[gpu] graph density n={n} parts={parts} tau={tau}", flush=True)
    g = sp2.Graph(H, tau, parts)
    D, infos = g.density(H, inst.mu)
    want, sizes = oracle_lib.graph_density(inst.H, tau, parts, inst.mu)
    assert list(sizes) == g.sizes()[0]
    assert all(i.status == 0 for i in infos)
    for i in infos:
        assert i.branches() == expected_branches(i, inst.mu)
    err = np.abs(D.cpu().numpy() - want).max()
    print(f"[gpu]   max |D - D_oracle| = {err:.2e}; iterations {[i.iterations for i in infos]}", flush=True)
    assert err <= 1e-9
    g.close()


def test_one_part_is_the_projector_at_mu(sp2, oracle_lib):
    """parts = 1: one mu-steered SP2 solve of the whole H; mu anywhere in the
    gap gives the same D, mu outside the Gershgorin interval gives 0 or I
    with no step."""
    H, w = gapped_random_hamiltonian(96, 40, gap=1.0, seed=5)
    Hg = torch.from_numpy(H).cuda()
    g = sp2.Graph(Hg, 0.0, 1)
    want, _ = oracle_lib.mu_dm(H, 0.0)
    for mu in (-0.3, 0.0, 0.4):
        D, infos = g.density(Hg, mu)
        assert infos[0].status == 0 and abs(infos[0].trace - 40) < 1e-8
        assert infos[0].branches() == expected_branches(infos[0], mu)
        assert np.abs(D.cpu().numpy() - want).max() <= 1e-10
    D, infos = g.density(Hg, -1e3)
    assert infos[0].iterations == 0 and torch.count_nonzero(D) == 0
    D, infos = g.density(Hg, 1e3)
    assert infos[0].iterations == 0 and torch.equal(D, torch.eye(96, dtype=D.dtype, device=D.device))
    g.close()


def test_reuse_and_auxiliary_graph(sp2, oracle_lib):
    """The parts come from the auxiliary matrix given at creation (here the
    FP64 projector of H, the section's 'previously computed DM'); later
    solves reuse them for a perturbed H."""
    n, parts, tau = 256, 4, 1e-2
    inst = make_local_hamiltonian(n, seed=41)
    P, _ = oracle_lib.mu_dm(inst.H, inst.mu)
    g = sp2.Graph(torch.from_numpy(P).cuda(), tau, parts)
    assert g.sizes()[0] == list(oracle_lib.graph_parts(P, tau, parts).sum(1))
    rng = np.random.default_rng(1)
    for step in range(2):
        E = 0.01 * rng.standard_normal((n, n))
        H = inst.H + (E + E.T) * (inst.H != 0)
        D, infos = g.density(torch.from_numpy(H).cuda(), inst.mu)
        want, _ = oracle_lib.graph_density(H, tau, parts, inst.mu, G=P)
        assert np.abs(D.cpu().numpy() - want).max() <= 1e-9
    g.close()


def test_full_size_parts_and_sampled_rows(sp2, oracle_lib):
    """n = 8192 local model, 32 parts: every part's node list equals the
    oracle's; two sampled parts' rows of D equal the LAPACK projector of their
    sub-matrix; the assembled occupation is n/2."""
    n, parts, tau = 8192, 32, 0.03
    inst = make_local_hamiltonian(n, seed=3, dtype=np.float32)
    H64 = inst.H.astype(np.float64)
    H = torch.from_numpy(inst.H).cuda()
    print(f"[gpu] graph full size n={n} parts={parts} tau={tau}", flush=True)
    g = sp2.Graph(H, tau, parts)
    member = oracle_lib.graph_parts(H64, tau, parts)
    assert g.sizes()[0] == list(member.sum(1))
    D, infos = g.density(H, inst.mu)
    assert all(i.status == 0 for i in infos)
    Dn = D.cpu().numpy().astype(np.float64)
    st = oracle_lib.segment_starts(n, parts)
    for k in (0, parts // 2 + 1):
        nodes = np.nonzero(member[k])[0]
        w, V = np.linalg.eigh(H64[np.ix_(nodes, nodes)])
        Pk = V[:, w < inst.mu] @ V[:, w < inst.mu].T
        core = np.arange(st[k], st[k + 1])
        want = np.zeros((core.size, n))
        want[:, nodes] = Pk[np.searchsorted(nodes, core)]
        assert np.abs(Dn[core] - want).max() <= 1e-6     # FP32 storage of D
    assert abs(np.trace(Dn) - n / 2) < 0.01 * n
    g.close()
