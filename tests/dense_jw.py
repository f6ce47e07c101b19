"""Dense Jordan-Wigner statevector checker (test infrastructure).

Builds fermionic operators as sparse matrices from Kronecker products of
2x2 Pauli-type matrices, applies each UCC factor exp(theta (tau - tau^dag))
(Eqs. 3-5) with scipy's ``expm_multiply``, and evaluates <psi|H|psi> from the
second-quantized Hamiltonian.  Nothing here uses the closed-form pair
rotation or the popcount sign rule, so it pins the oracle independently.

Basis index D = sum_q b_q 2^q with b_q = 1 when spin-orbital q is occupied.
a_q = I x ... x I x sigma^- x Z x ... x Z with the Z string on the qubits
below q (Kronecker factors ordered from qubit nq-1 down to qubit 0).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh, expm_multiply

_SM = sp.csr_matrix(np.array([[0.0, 1.0], [0.0, 0.0]]))  # |1> -> |0>
_Z = sp.csr_matrix(np.diag([1.0, -1.0]))
_I = sp.identity(2, format="csr")


def annihilators(nq: int):
    ops = []
    for q in range(nq):
        factors = [_I] * (nq - 1 - q) + [_SM] + [_Z] * q
        m = factors[0]
        for f in factors[1:]:
            m = sp.kron(m, f, format="csr")
        ops.append(m.tocsr())
    return ops


class DenseJW:
    def __init__(self, nq: int):
        self.nq = nq
        self.dim = 1 << nq
        self.a = annihilators(nq)
        self.ad = [m.T.tocsr() for m in self.a]

    def tau(self, row):
        i, j, a, b = (int(x) for x in row)
        if j < 0:
            return (self.ad[a] @ self.a[i]).tocsr()
        return (self.ad[a] @ self.ad[b] @ self.a[j] @ self.a[i]).tocsr()

    def basis(self, dets, amps=None):
        v = np.zeros(self.dim)
        amps = np.ones(len(dets)) if amps is None else amps
        for d, c in zip(dets, amps):
            v[int(d)] += c
        return v / np.linalg.norm(v)

    def apply_factors(self, psi, exc, theta):
        for row, th in zip(exc, theta):
            t = self.tau(row)
            A = (t - t.T).tocsc()
            psi = expm_multiply(th * A, psi)
        return psi

    # -- Hamiltonian ------------------------------------------------------
    def h_literal(self, h1, h2):
        """Sparse H assembled term by term (small nq only)."""
        n = h1.shape[0]
        H = sp.csr_matrix((self.dim, self.dim))
        for s in range(2):
            for p in range(n):
                for q in range(n):
                    if h1[p, q] != 0.0:
                        H = H + h1[p, q] * (self.ad[2 * p + s] @ self.a[2 * q + s])
        for s, t in itertools.product(range(2), repeat=2):
            for p, q, r, u in itertools.product(range(n), repeat=4):
                v = h2[p, q, r, u]
                if v == 0.0:
                    continue
                H = H + 0.5 * v * (self.ad[2 * p + s] @ self.ad[2 * r + t] @ self.a[2 * u + t] @ self.a[2 * q + s])
        return H.tocsr()

    def excitation_ops(self, n):
        return [[(self.ad[2 * p] @ self.a[2 * q] + self.ad[2 * p + 1] @ self.a[2 * q + 1]).tocsr()
                 for q in range(n)] for p in range(n)]

    def energy_epq(self, h1, h2, psi):
        """<psi|H|psi> via spin-summed E_pq:  sum_{sigma tau} a+_p a+_r a_s a_q
        = E_pq E_rs - delta_qr E_ps."""
        n = h1.shape[0]
        E = self.excitation_ops(n)
        V = np.stack([E[p][q] @ psi for p in range(n) for q in range(n)])  # row pq
        one = sum(h1[p, q] * psi @ V[p * n + q] for p in range(n) for q in range(n))
        G = V @ V.T  # G[(pq),(rs)] = <E_pq psi | E_rs psi>
        two = 0.0
        for p, q, r, s in itertools.product(range(n), repeat=4):
            v = h2[p, q, r, s]
            if v != 0.0:
                two += v * G[q * n + p, r * n + s]
        corr = sum(h2[p, q, q, s] * psi @ V[p * n + s] for p in range(n) for q in range(n) for s in range(n))
        return (one + 0.5 * two - 0.5 * corr) / (psi @ psi)

    def sector(self, n_alpha, n_beta):
        idx = []
        for D in range(self.dim):
            na = bin(D & int("01" * (self.nq // 2), 2)).count("1")
            nb = bin(D & int("10" * (self.nq // 2), 2)).count("1")
            if na == n_alpha and nb == n_beta:
                idx.append(D)
        return np.asarray(idx)

    def fci(self, H, n_alpha, n_beta):
        idx = self.sector(n_alpha, n_beta)
        Hs = H[idx][:, idx]
        if Hs.shape[0] <= 400:
            return float(np.linalg.eigvalsh(Hs.toarray())[0])
        return float(eigsh(Hs, k=1, which="SA")[0][0])
