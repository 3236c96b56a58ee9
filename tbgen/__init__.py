"""Seeded synthetic tight-binding Hamiltonians (input generator only).

This module produces the inputs that both the HIP path and the CPU oracle
consume.  It holds none of the purification arithmetic: no spectral bounds,
no initial matrix, no squaring, no steering.  It builds a Hamiltonian and,
because the literal model has almost no gap at half filling, opens a
HOMO-LUMO gap by shifting the virtual eigenvalues (a statement about the
*input*, not about how the density matrix is computed).

Model (stand-in for the paper's peptide-in-water DFTB benchmark, which is not
available; the paper describes the Hamiltonian only as a symmetric N x N
matrix in a localized basis, Section "Single-particle density matrix"):

* ``natom = n // 4`` atoms uniform in a periodic cube at density 0.1 / A^3,
  edge ``L = (natom / 0.1) ** (1/3)``;
* 4 orbitals per atom, orbital ``i`` on atom ``i // 4``;
* onsite energies ``H_ii ~ N(-5, 1)`` eV;
* hopping ``H_ij = -2 exp(-r/1.5) (1 + 0.1 N(0,1))`` eV for orbitals on
  distinct atoms with minimum-image distance ``r < 6`` A, zero otherwise
  (orbitals on the same atom do not couple);
* the upper triangle is drawn and mirrored, so ``H`` is bitwise symmetric;
* gap opening: ``H = V diag(eps) V^T``; the virtual levels ``eps[i]`` for
  ``i >= n_occ`` (0-based) are shifted up by ``max(0, gap - (eps[n_occ] -
  eps[n_occ-1]))``; the result is rebuilt as ``V diag(eps') V^T`` and
  symmetrised as ``(A + A^T)/2``;
* optional rounding to float32 last (the rounded matrix is symmetric too,
  because rounding is elementwise).

Draw order from ``numpy.random.default_rng(seed)`` (PCG64): positions
(natom x 3 uniforms), then one normal per upper-triangle pair in
``numpy.triu_indices(n, 1)`` order, then the n onsite normals.
"""
from __future__ import annotations

import numpy as np

ORBITALS_PER_ATOM = 4
DENSITY = 0.1          # atoms per cubic Angstrom
CUTOFF = 6.0           # Angstrom
DECAY = 1.5            # Angstrom
HOP_SCALE = -2.0       # eV
HOP_NOISE = 0.1
ONSITE_MEAN = -5.0     # eV
ONSITE_STD = 1.0       # eV


def box_length(natom: int) -> float:
    return (natom / DENSITY) ** (1.0 / 3.0)


def literal_hamiltonian(n: int, seed: int) -> np.ndarray:
    """The tight-binding model before gap opening, float64, bitwise symmetric."""
    if n <= 0 or n % ORBITALS_PER_ATOM:
        raise ValueError(f"n must be a positive multiple of {ORBITALS_PER_ATOM}, got {n}")
    natom = n // ORBITALS_PER_ATOM
    L = box_length(natom)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, size=(natom, 3))
    iu, ju = np.triu_indices(n, 1)
    noise = rng.standard_normal(iu.size)
    onsite = ONSITE_MEAN + ONSITE_STD * rng.standard_normal(n)

    ai = iu // ORBITALS_PER_ATOM
    aj = ju // ORBITALS_PER_ATOM
    d = pos[ai] - pos[aj]
    d -= L * np.round(d / L)                       # minimum image
    r = np.sqrt((d * d).sum(axis=1))
    hop = HOP_SCALE * np.exp(-r / DECAY) * (1.0 + HOP_NOISE * noise)
    hop[(ai == aj) | (r >= CUTOFF)] = 0.0

    H = np.zeros((n, n), dtype=np.float64)
    H[iu, ju] = hop
    H[ju, iu] = hop
    H[np.arange(n), np.arange(n)] = onsite
    return H


class TBInstance:
    """One generated Hamiltonian with the facts of its construction."""

    def __init__(self, H, n_occ, gap_target, gap_literal, shift, eigvals):
        self.H = H                      # float64 or float32, (n, n), symmetric
        self.n_occ = n_occ
        self.gap_target = gap_target
        self.gap_literal = gap_literal  # HOMO-LUMO gap of the literal model
        self.shift = shift              # amount added to the virtual levels
        self.eigvals = eigvals          # spectrum used to build H (float64)

    @property
    def n(self):
        return self.H.shape[0]


def make_tb_hamiltonian(n: int, seed: int, gap: float = 0.5, n_occ: int | None = None,
                        dtype=np.float64, eigh_device: str | None = None) -> TBInstance:
    """Generate a gapped tight-binding Hamiltonian of size ``n`` (float64 or float32).

    eigh_device: None = LAPACK on the host; a torch device name ("cuda") =
    the same FP64 eigendecomposition and rebuild on that device (for large n,
    where the host takes minutes; the input differs from the host-built one
    only by rounding)."""
    if n_occ is None:
        n_occ = n // 2
    if not (0 < n_occ < n):
        raise ValueError("0 < n_occ < n required for a gap to open")
    H0 = literal_hamiltonian(n, seed)
    if eigh_device is None:
        eps, V = np.linalg.eigh(H0)
    else:
        import torch
        Hd = torch.from_numpy(H0).to(eigh_device)
        del H0
        epsd, Vd = torch.linalg.eigh(Hd)
        del Hd
        eps = epsd.cpu().numpy()
    gap_lit = float(eps[n_occ] - eps[n_occ - 1])
    shift = max(0.0, gap - gap_lit)
    eps2 = eps.copy()
    eps2[n_occ:] += shift
    if eigh_device is None:
        A = (V * eps2) @ V.T
        H = 0.5 * (A + A.T)
    else:
        e2 = torch.from_numpy(eps2).to(eigh_device)
        A = (Vd * e2) @ Vd.T
        del Vd
        H = (0.5 * (A + A.T)).cpu().numpy()
        del A
    H = np.ascontiguousarray(H.astype(dtype))
    return TBInstance(H, n_occ, gap, gap_lit, shift, eps2)


def batch_sizes(count: int, seed: int, lo: int = 64, hi: int = 512, step: int = 4) -> np.ndarray:
    """Sizes drawn uniformly from {lo, lo+step, ..., hi} (the uneven-subsystem batch)."""
    rng = np.random.default_rng(seed)
    choices = np.arange(lo, hi + 1, step)
    return choices[rng.integers(0, choices.size, size=count)]


def diagonal_hamiltonian(n: int, seed: int) -> np.ndarray:
    """A diagonal H with distinct entries (float64), for elementwise special cases."""
    rng = np.random.default_rng(seed)
    d = rng.permutation(np.linspace(-10.0, 10.0, n)) + 1e-3 * rng.standard_normal(n)
    return np.diag(d)


def two_level_hamiltonian(n: int, k: int, alpha: float, beta: float, seed: int):
    """H = alpha P + beta (I - P) with P a random rank-k orthogonal projector.

    Returns (H, P).  With alpha < beta and n_occ = k the density matrix is P.
    """
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    P = Q[:, :k] @ Q[:, :k].T
    P = 0.5 * (P + P.T)
    H = alpha * P + beta * (np.eye(n) - P)
    H = 0.5 * (H + H.T)
    return H, P


def gapped_random_hamiltonian(n: int, n_occ: int, gap: float, seed: int, spread: float = 10.0):
    """Dense symmetric H = Q diag(eps) Q^T with a prescribed gap at n_occ.

    eps: n_occ levels uniform in [-spread, -gap/2] and n - n_occ levels
    uniform in [gap/2, spread], with the two innermost levels placed exactly at
    -gap/2 and +gap/2 (so the HOMO-LUMO gap equals `gap`).  Works for any n
    (the tight-binding model needs a multiple of 4).  Returns (H, eps sorted).
    """
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-spread, -gap / 2, size=n_occ)
    hi = rng.uniform(gap / 2, spread, size=n - n_occ)
    if n_occ > 0:
        lo[np.argmax(lo)] = -gap / 2
    if n - n_occ > 0:
        hi[np.argmin(hi)] = gap / 2
    eps = np.sort(np.concatenate([lo, hi]))
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * eps) @ Q.T
    return np.ascontiguousarray(0.5 * (A + A.T)), eps


# ---------------------------------------------------------------- local model
# A tight-binding model whose gap comes from its orbitals rather than from a
# spectral shift, so that H stays sparse and spatially local (the input of
# the graph-partitioned solver, which needs locality).
LOCAL_SPLIT = 8.0        # eV between the two low and the two high orbitals of an atom
LOCAL_ONSITE_STD = 0.3   # eV
LOCAL_HOP = 1.5          # eV
LOCAL_DECAY = 1.0        # Angstrom
LOCAL_CUTOFF = 5.0       # Angstrom
LOCAL_MORTON_BITS = 5    # 32^3 cells for the spatial ordering


def _morton(c: np.ndarray, bits: int) -> np.ndarray:
    code = np.zeros(c.shape[0], dtype=np.int64)
    for b in range(bits):
        for axis in range(3):
            code |= ((c[:, axis] >> b) & 1).astype(np.int64) << (3 * b + (2 - axis))
    return code


class LocalInstance:
    """One local gapped Hamiltonian with the facts of its construction."""

    def __init__(self, H, n_occ, mu, positions, box):
        self.H = H                  # (n, n) float64 or float32, bitwise symmetric
        self.n_occ = n_occ          # n / 2: the two low orbitals of every atom
        self.mu = mu                # 0 eV: the middle of the orbital splitting
        self.positions = positions  # atoms in index order (Angstrom)
        self.box = box

    @property
    def n(self):
        return self.H.shape[0]


def make_local_hamiltonian(n: int, seed: int, dtype=np.float64) -> LocalInstance:
    """Spatially local, gapped tight-binding Hamiltonian of size ``n``.

    * ``n // 4`` atoms uniform in a periodic cube at density 0.1 / A^3, then
      ordered along a Morton curve of a 32^3 cell grid (stable), so that
      regular segments of the index list are compact regions of space;
    * 4 orbitals per atom: orbitals 0, 1 at -4 eV and 2, 3 at +4 eV, each
      plus 0.3 N(0, 1) eV;
    * hopping between orbitals of distinct atoms closer than 5 A (minimum
      image): ``-1.5 exp(-r / 1 A) s (1 + 0.1 N(0, 1))`` eV with a random
      sign ``s = +-1`` per orbital pair;
    * n_occ = n / 2 fills the low orbitals; the gap lies around mu = 0 eV.

    Draw order from ``numpy.random.default_rng(seed)``: positions (natom x 3
    uniforms); then, over the orbital pairs (i < j) within the cutoff in
    lexicographic order, one uniform per pair for the sign (s = -1 below
    1/2), then one normal per pair; then the n onsite normals.
    """
    from scipy.spatial import cKDTree
    if n <= 0 or n % ORBITALS_PER_ATOM:
        raise ValueError(f"n must be a positive multiple of {ORBITALS_PER_ATOM}, got {n}")
    natom = n // ORBITALS_PER_ATOM
    L = box_length(natom)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, L, size=(natom, 3))
    g = 1 << LOCAL_MORTON_BITS
    cell = np.minimum((pos / L * g).astype(np.int64), g - 1)
    pos = pos[np.argsort(_morton(cell, LOCAL_MORTON_BITS), kind="stable")]
    pos = np.mod(pos, L)
    ap = cKDTree(pos, boxsize=L).query_pairs(LOCAL_CUTOFF, output_type="ndarray")
    ap = ap[np.lexsort((ap[:, 1], ap[:, 0]))] if ap.size else ap.reshape(0, 2)
    d = pos[ap[:, 0]] - pos[ap[:, 1]]
    d -= L * np.round(d / L)
    r = np.sqrt((d * d).sum(axis=1))
    # every atom pair (a < b) gives the 16 orbital pairs (4a + p, 4b + q)
    o = np.arange(ORBITALS_PER_ATOM)
    oi = (ORBITALS_PER_ATOM * ap[:, 0])[:, None, None] + o[None, :, None]
    oj = (ORBITALS_PER_ATOM * ap[:, 1])[:, None, None] + o[None, None, :]
    oi, oj = np.broadcast_arrays(oi, oj)
    oi, oj = oi.reshape(-1), oj.reshape(-1)
    rr = np.repeat(r, ORBITALS_PER_ATOM * ORBITALS_PER_ATOM)
    order = np.lexsort((oj, oi))
    oi, oj, rr = oi[order], oj[order], rr[order]
    sign = np.where(rng.random(oi.size) < 0.5, -1.0, 1.0)
    noise = rng.standard_normal(oi.size)
    onsite = rng.standard_normal(n)
    hop = -LOCAL_HOP * np.exp(-rr / LOCAL_DECAY) * sign * (1.0 + HOP_NOISE * noise)
    H = np.zeros((n, n), dtype=np.float64)
    H[oi, oj] = hop
    H[oj, oi] = hop
    orb = np.arange(n) % ORBITALS_PER_ATOM
    H[np.arange(n), np.arange(n)] = np.where(orb < 2, -LOCAL_SPLIT / 2, LOCAL_SPLIT / 2) + \
        LOCAL_ONSITE_STD * onsite
    H = np.ascontiguousarray(H.astype(dtype))
    return LocalInstance(H, n // 2, 0.0, pos, L)
