"""GPU parity of the learned recursive expansion (sp2_learned_*).

Each layer maps X -> a X^2 + b X + c I, or its particle-hole form when the
trace is at or below n_occ (a deep-network form of the recursive polynomial
expansion of the paper's Section "GPU friendly algorithms", steered like SP2).
The oracle evaluates the same layers literally on the matrix
(oracle_learned_matrix, FP64, triple-loop products); the GPU output after the
layers and the SP2 check step must match it at the FP64 bar.  With SP2's
coefficients the network is SP2 itself, bit for bit.
"""
import numpy as np
import pytest

from tbgen import gapped_random_hamiltonian, make_tb_hamiltonian

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


def sp2_step(oracle_lib, X, n_occ):
    """One SP2 step of X through the oracle (the check step after the layers)."""
    n = X.shape[0]
    grow = int(np.trace(X) - n_occ <= 0)
    I, J = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return oracle_lib.sp2_step_entries(X, grow, I.ravel(), J.ravel()).reshape(n, n)


def test_sp2_coefficients_are_sp2(sp2):
    inst = make_tb_hamiltonian(128, seed=61)
    H = torch.from_numpy(inst.H).cuda()
    L = 12
    model = sp2.Learned.from_coefficients(np.tile([1.0, 0.0, 0.0], L))
    Ds, infos = model.density([H], [inst.n_occ], idem_fallback=1e9)
    D1, i1 = sp2.sp2_density(H, inst.n_occ, max_iter=L + 1)
    assert infos[0].status == 0 and infos[0].iterations == L + 1
    assert infos[0].branch_mask == i1.branch_mask
    assert torch.equal(Ds[0], D1)
    model.close()


@pytest.mark.parametrize("n,n_occ", [(100, 41), (130, 65)])
def test_layers_match_oracle(sp2, oracle_lib, n, n_occ):
    rng = np.random.default_rng(n)
    H, _ = gapped_random_hamiltonian(n, n_occ, gap=1.0, seed=n)
    # mild perturbations of SP2: large ones make the composed maps diverge
    # (then the check step rightly rejects the output and SP2 starts from H)
    coef = np.column_stack([1.0 + 0.05 * rng.standard_normal(8), 0.02 * rng.standard_normal(8),
                            0.005 * rng.standard_normal(8)]).astype(np.float32).astype(np.float64)
    model = sp2.Learned.from_coefficients(coef)
    Ds, infos = model.density([torch.from_numpy(H).cuda()], [n_occ], idem_fallback=1e9)
    XL, br = oracle_lib.learned_matrix(H, n_occ, coef)
    want = sp2_step(oracle_lib, XL, n_occ)
    assert np.isfinite(XL).all() and np.abs(XL).max() < 10
    assert infos[0].status == 0 and infos[0].iterations == 9
    assert infos[0].branches()[:8] == br
    assert np.abs(Ds[0].cpu().numpy() - want).max() <= 1e-10 * max(1.0, np.abs(want).max())
    model.close()


def test_fallback_to_sp2(sp2):
    """Four SP2 layers are far from idempotent: every matrix is rejected at
    the check step and restarts plain SP2 from its kept X_0 in the same run;
    D, the SP2 step count and its result equal sp2_density's."""
    Hs, nocc = [], []
    for k in range(3):
        inst = make_tb_hamiltonian(96, seed=70 + k)
        Hs.append(torch.from_numpy(inst.H).cuda())
        nocc.append(inst.n_occ)
    model = sp2.Learned.from_coefficients(np.tile([1.0, 0.0, 0.0], 4))
    Ds, infos = model.density(Hs, nocc, idem_fallback=1e-6)
    for H, D, i, no in zip(Hs, Ds, infos, nocc):
        D1, i1 = sp2.sp2_density(H, no)
        assert i.status == sp2.FALLBACK and i.fp64_prefix_iters == 4
        assert i.refine_steps == i1.iterations and i.iterations == 4 + 1 + i1.iterations
        assert torch.equal(D, D1)
    model.close()


def test_continuation_with_plain_sp2(sp2, oracle_lib):
    """Layers that leave X close to a projector but above the bar hand over to
    plain SP2 on the device: the check step, one step of the other branch
    (the pull-in into [0, 1]), then trace-steered steps.  With SP2's
    coefficients every map is an SP2 map: up to the check step the run is
    sp2_density's (same branches), the step after it takes the other branch,
    and D is the same projector to FP64 rounding."""
    inst = make_tb_hamiltonian(160, seed=77)
    ref = oracle_lib.sp2(inst.H, inst.n_occ)
    e = np.asarray(ref.e_hist)
    L = int(np.argmax((e < 0.2) & (e > 1e-4)))
    assert 0 < L < ref.iterations - 2
    model = sp2.Learned.from_coefficients(np.tile([1.0, 0.0, 0.0], L))
    H = torch.from_numpy(inst.H).cuda()
    Ds, infos = model.density([H], [inst.n_occ], idem_fallback=1e-6)
    D1, i1 = sp2.sp2_density(H, inst.n_occ)
    i = infos[0]
    assert i.status == 0 and i.fp64_prefix_iters == L
    assert i.refine_steps == i.iterations - L - 1 and i.refine_steps >= 1
    b, b1 = i.branches(), i1.branches()
    assert b[:L + 1] == b1[:L + 1] and b[L + 1] == 1 - b[L]
    assert torch.abs(Ds[0] - D1).max().item() <= 1e-12
    Dj, _, _ = oracle_lib.jacobi_dm(inst.H, inst.n_occ)
    assert np.abs(Ds[0].cpu().numpy() - Dj).max() <= 1e-10
    model.close()


def test_fit_beats_truncated_sp2_and_matches_oracle(sp2, oracle_lib, tmp_path):
    """A short training run from SP2 (12 layers, 96 spectra of n = 128, gaps
    0.3-2 eV) must lower the loss, beat 12 SP2 steps on held-out spectra
    (measured by the oracle's spectral form), and run on the GPU exactly as
    the oracle evaluates it; the model survives a save/load round trip."""
    n, L = 128, 12
    rng = np.random.default_rng(5)
    spec, gersh, nocc, Hs = [], [], [], []
    for s in range(112):
        inst = make_tb_hamiltonian(n, seed=3000 + s, gap=float(rng.uniform(0.3, 2.0)))
        lo, hi = oracle_lib.gershgorin(inst.H)
        spec.append(np.sort(inst.eigvals))
        gersh.append((lo, hi))
        nocc.append(inst.n_occ)
        Hs.append(inst.H)
    print("[gpu] learned fit: 96 training spectra", flush=True)
    model = sp2.Learned.fit(L, spec[:96], nocc[:96], gersh[:96], epochs=400, seed=1)
    coef, loss = model.coefficients()
    assert coef.shape == (L, 3) and np.all(coef == coef.astype(np.float32))

    def spectral_err(c, s):
        x, _, _ = oracle_lib.learned_spectral(spec[s], nocc[s], gersh[s][0], gersh[s][1], c)
        theta = (np.arange(n) < nocc[s]).astype(float)
        return float(np.sqrt(np.mean((x - theta) ** 2)))

    sp2c = np.tile([1.0, 0.0, 0.0], (L, 1))
    held = range(96, 112)
    e_net = np.array([spectral_err(coef, s) for s in held])
    e_sp2 = np.array([spectral_err(sp2c, s) for s in held])
    print(f"[gpu] learned: loss {loss:.2f}; held-out rms median net {np.median(e_net):.2e} "
          f"vs SP2x{L} {np.median(e_sp2):.2e}", flush=True)
    assert np.median(e_net) < 0.5 * np.median(e_sp2)
    path = tmp_path / "model.txt"
    model.save(path)
    model2 = sp2.Learned.load(path)
    coef2, loss2 = model2.coefficients()
    assert np.array_equal(coef, coef2) and loss2 == loss
    H = torch.from_numpy(Hs[100]).cuda()
    Ds, infos = model2.density([H], [nocc[100]], idem_fallback=1e9)
    XL, br = oracle_lib.learned_matrix(Hs[100], nocc[100], coef)
    want = sp2_step(oracle_lib, XL, nocc[100])
    assert np.abs(Ds[0].cpu().numpy() - want).max() <= 1e-9
    model.close()
    model2.close()
