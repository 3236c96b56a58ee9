"""The seeded input generator: determinism, symmetry, the opened gap, FP32 rounding."""
import numpy as np

from tbgen import batch_sizes, box_length, literal_hamiltonian, make_tb_hamiltonian


def test_deterministic_and_symmetric():
    a = make_tb_hamiltonian(64, 5).H
    b = make_tb_hamiltonian(64, 5).H
    assert np.array_equal(a, b)
    assert np.array_equal(a, a.T)
    assert not np.array_equal(a, make_tb_hamiltonian(64, 6).H)


def test_gap_opened_to_target():
    for n, gap in ((64, 0.5), (128, 1.7)):
        inst = make_tb_hamiltonian(n, 1, gap=gap)
        w = np.linalg.eigvalsh(inst.H)
        assert abs((w[inst.n_occ] - w[inst.n_occ - 1]) - gap) < 1e-9
        assert inst.gap_literal < gap


def test_float32_storage_symmetric():
    inst = make_tb_hamiltonian(128, 2, dtype=np.float32)
    assert inst.H.dtype == np.float32
    assert np.array_equal(inst.H, inst.H.T)


def test_literal_model_structure():
    H = literal_hamiltonian(64, 3)
    # orbitals on one atom do not couple
    for a in range(16):
        blk = H[4 * a:4 * a + 4, 4 * a:4 * a + 4]
        assert np.count_nonzero(blk - np.diag(np.diag(blk))) == 0
    assert abs(np.diag(H).mean() + 5.0) < 0.5
    off = H[~np.eye(64, dtype=bool)]
    assert off.max() <= 0.0 and off.min() > -2.0 * 1.5
    assert abs(box_length(64) - 8.6177) < 1e-3


def test_batch_sizes_range():
    s = batch_sizes(512, 0)
    assert s.min() >= 64 and s.max() <= 512 and np.all(s % 4 == 0)
    assert np.array_equal(s, batch_sizes(512, 0))
