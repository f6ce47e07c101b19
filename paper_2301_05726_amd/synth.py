"""Seeded synthetic inputs for the sparse-wavefunction UCC solver.

This module only *generates inputs*: a random real molecular-like Hamiltonian
(one-electron matrix h1 and chemist-notation two-electron tensor h2), the
spin-conserving UCCSD excitation list in the applied order, the Hartree-Fock
reference determinant and the random parameter vectors.  It holds none of the
solver's arithmetic (no factor application, no energy, no gradient); both the
HIP library and the CPU oracle receive what it produces as plain arrays.

Conventions (the paper fixes none of them; they are the readings recorded in
the design notes):

* spatial orbital p = 0..n-1, spin sigma = 0 (alpha) / 1 (beta), spin-orbital
  q = 2p + sigma; determinant bit q set <=> spin-orbital q occupied;
* the reference |Psi_0> (Eq. 1) is the aufbau determinant with spatial
  orbitals 0..o-1 doubly occupied;
* excitations (Eq. 2): singles tau_i^a = a+_a a_i with i occupied, a virtual,
  same spin; doubles tau_ij^ab = a+_a a+_b a_j a_i with i<j occupied, a<b
  virtual, conserving N_alpha and N_beta.  Encoded as int8 rows (i, j, a, b);
  a single has j = b = -1;
* applied order (Methods section, factorized product Eq. 3): doubles first,
  sorted by descending |MP2-like amplitude| (stable, ties kept in canonical
  generation order), then all singles in canonical order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# benchmark workloads (sizes follow the paper's range: up to 32 spatial
# orbitals = 64 spin-orbitals, tens of thousands of factors)
# --------------------------------------------------------------------------


@dataclass(frozen=True)
class Workload:
    name: str
    n_orb: int          # spatial orbitals n (qubits = 2n)
    n_occ: int          # doubly occupied spatial orbitals o (N_alpha = N_beta = o)
    theta_sigma: float  # theta ~ N(0, sigma)
    threshold: float    # pruning threshold on |amplitude|
    capacity: int       # hash slots per state
    batch: int = 1
    cfg: int = 0        # seed offset

    @property
    def n_qubits(self) -> int:
        return 2 * self.n_orb


WORKLOADS = {
    "q8": Workload("q8", 4, 2, 0.05, 0.0, 1 << 8, 1, 1),
    "q20": Workload("q20", 10, 5, 0.02, 0.0, 1 << 17, 1, 2),
    "q32": Workload("q32", 16, 8, 0.01, 1e-6, 1 << 26, 1, 3),
    "q48": Workload("q48", 24, 12, 0.005, 1e-5, 1 << 26, 8, 4),
    "q64": Workload("q64", 32, 16, 0.003, 1e-4, 1 << 28, 1, 5),
}


# --------------------------------------------------------------------------
# Hamiltonian
# --------------------------------------------------------------------------


def canonical_eri_order(n: int):
    """Canonical (pq|rs) index quadruples p>=q, r>=s, pq>=rs (compound
    indices pq = p(p+1)/2+q), in lexicographic order of (p, q, r, s)."""
    out = []
    for p in range(n):
        for q in range(p + 1):
            pq = p * (p + 1) // 2 + q
            for r in range(n):
                for s in range(r + 1):
                    rs = r * (r + 1) // 2 + s
                    if pq >= rs:
                        out.append((p, q, r, s))
    return out


def make_hamiltonian(n: int, seed: int):
    """Random real Hamiltonian with the shapes of a molecular one.

    h1: symmetric, off-diagonal ~ N(0,1) * exp(-|p-q|/2), diagonal -(4 - p/2).
    h2: chemist notation (pq|rs), 8-fold symmetric, canonical elements
        ~ N(0, 0.1) * exp(-(|p-q| + |r-s|)/2).
    Draw order: h1 off-diagonals (p<q row-major), then canonical ERIs.
    """
    rng = np.random.default_rng(seed)
    h1 = np.zeros((n, n))
    for p in range(n):
        h1[p, p] = -(4.0 - p / 2.0)
    for p in range(n):
        for q in range(p + 1, n):
            v = rng.normal(0.0, 1.0) * math.exp(-abs(p - q) / 2.0)
            h1[p, q] = v
            h1[q, p] = v
    h2 = np.zeros((n, n, n, n))
    for (p, q, r, s) in canonical_eri_order(n):
        v = rng.normal(0.0, 0.1) * math.exp(-(abs(p - q) + abs(r - s)) / 2.0)
        for (a, b, c, d) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                             (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
            h2[a, b, c, d] = v
    return h1, h2


# --------------------------------------------------------------------------
# excitations
# --------------------------------------------------------------------------


def spin(q: int) -> int:
    return q & 1


def hf_det(n_occ: int) -> int:
    """Aufbau determinant: spin-orbitals 2p, 2p+1 for p < o."""
    return (1 << (2 * n_occ)) - 1


def canonical_excitations(n_orb: int, n_occ: int):
    """Spin-conserving singles and doubles relative to the aufbau reference,
    in canonical generation order.  Returns (singles, doubles) as lists of
    (i, j, a, b) tuples (singles with j = b = -1)."""
    nq = 2 * n_orb
    occ = list(range(2 * n_occ))
    vir = list(range(2 * n_occ, nq))
    singles = [(i, -1, a, -1) for i in occ for a in vir if spin(i) == spin(a)]
    doubles = []
    for ii, i in enumerate(occ):
        for j in occ[ii + 1:]:
            for aa, a in enumerate(vir):
                for b in vir[aa + 1:]:
                    if spin(i) + spin(j) == spin(a) + spin(b):
                        doubles.append((i, j, a, b))
    return singles, doubles


def open_shell_det(n_alpha: int, n_beta: int) -> int:
    """Aufbau determinant with n_alpha alpha (2p) and n_beta beta (2p+1)
    electrons in the lowest spatial orbitals."""
    return sum(1 << (2 * p) for p in range(n_alpha)) | sum(1 << (2 * p + 1) for p in range(n_beta))


def open_shell_excitations(n_orb: int, n_alpha: int, n_beta: int) -> np.ndarray:
    """Spin-conserving singles, then doubles, relative to
    open_shell_det(n_alpha, n_beta), as an int8 array of (i, j, a, b) rows."""
    ref = open_shell_det(n_alpha, n_beta)
    occ = [q for q in range(2 * n_orb) if ref >> q & 1]
    vir = [q for q in range(2 * n_orb) if not ref >> q & 1]
    rows = [(i, -1, a, -1) for i in occ for a in vir if spin(i) == spin(a)]
    for ii, i in enumerate(occ):
        for j in occ[ii + 1:]:
            for aa, a in enumerate(vir):
                for b in vir[aa + 1:]:
                    if spin(i) + spin(j) == spin(a) + spin(b):
                        rows.append((i, j, a, b))
    return np.array(rows, dtype=np.int8).reshape(-1, 4)


def uccsd_count(n_orb: int, n_occ: int) -> int:
    """Closed form 2ov + 2 C(o,2) C(v,2) + o^2 v^2 for o occupied and v
    virtual spatial orbitals per spin."""
    o, v = n_occ, n_orb - n_occ
    return 2 * o * v + 2 * math.comb(o, 2) * math.comb(v, 2) + o * o * v * v


def _antisym(h2, p, q, r, s):
    """<pq||rs> over spin-orbitals from spatial chemist integrals."""
    def phys(p, q, r, s):
        if spin(p) != spin(r) or spin(q) != spin(s):
            return 0.0
        return h2[p >> 1, r >> 1, q >> 1, s >> 1]
    return phys(p, q, r, s) - phys(p, q, s, r)


def orbital_energies(h1, h2, n_occ: int):
    """Diagonal Fock elements f_pp = h_pp + sum_{k<o} [2 (pp|kk) - (pk|kp)]
    (spatial), used only to order the doubles."""
    n = h1.shape[0]
    eps = np.empty(n)
    for p in range(n):
        eps[p] = h1[p, p] + sum(2.0 * h2[p, p, k, k] - h2[p, k, k, p] for k in range(n_occ))
    return eps


def ordered_excitations(h1, h2, n_occ: int) -> np.ndarray:
    """UCCSD excitation list in applied order (Methods section): doubles by
    descending |<ij||ab> / (e_i + e_j - e_a - e_b)| (stable), then singles."""
    n = h1.shape[0]
    singles, doubles = canonical_excitations(n, n_occ)
    eps = orbital_energies(h1, h2, n_occ)
    mags = []
    for (i, j, a, b) in doubles:
        gap = eps[i >> 1] + eps[j >> 1] - eps[a >> 1] - eps[b >> 1]
        num = _antisym(h2, i, j, a, b)
        mags.append(abs(num / gap) if gap != 0.0 else math.inf)
    order = sorted(range(len(doubles)), key=lambda k: -mags[k])  # sorted() is stable
    rows = [doubles[k] for k in order] + singles
    return np.asarray(rows, dtype=np.int8).reshape(-1, 4)


def make_theta(n_params: int, sigma: float, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, sigma, n_params)


@dataclass
class Problem:
    wl: Workload
    h1: np.ndarray
    h2: np.ndarray
    exc: np.ndarray                     # int8 [M, 4]
    theta: np.ndarray                   # float64 [B, M]
    hf: int
    extras: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.exc.shape[0])


def make_problem(wl: Workload | str, batch: int | None = None, n_factors: int | None = None) -> Problem:
    """Build the seeded problem for a workload: H from seed 1000+cfg, theta
    for batch member b from seed 2000+cfg+b.  ``n_factors`` keeps only the
    first factors of the applied order (a prefix of the circuit)."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    B = wl.batch if batch is None else batch
    h1, h2 = make_hamiltonian(wl.n_orb, 1000 + wl.cfg)
    exc = ordered_excitations(h1, h2, wl.n_occ)
    if n_factors is not None:
        exc = exc[:n_factors].copy()
    M = exc.shape[0]
    theta = np.stack([make_theta(M, wl.theta_sigma, 2000 + wl.cfg + b) for b in range(B)])
    return Problem(wl, h1, h2, exc, theta, hf_det(wl.n_occ))


def fd_subset(M: int, count: int, seed: int) -> np.ndarray:
    """Parameter indices for finite-difference checks, drawn without
    replacement from seed (3000+cfg by convention)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(M, size=min(count, M), replace=False))
