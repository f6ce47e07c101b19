"""Host-side parts of the outer loop: FCIDUMP reading and writing, and the
scipy minimisation driven by energies and adjoint gradients (here served by
the CPU oracle, so the loop itself is checked without a GPU)."""
import os

import numpy as np
import pytest

from paper_2301_05726_amd import synth, vqe
from dense_jw import DenseJW

HERE = os.path.dirname(os.path.abspath(__file__))


def test_fcidump_fixture_symmetry_and_core():
    """A hand-written file (arbitrary values, not a molecule): every listed
    integral lands on all its symmetry partners; D exponents parse."""
    n, nelec, ms2, h1, h2, e_core = vqe.read_fcidump(os.path.join(HERE, "golden", "tiny.fcidump"))
    assert (n, nelec, ms2) == (2, 2, 0)
    assert e_core == 0.75
    assert h1[0, 0] == -1.25 and h1[0, 1] == h1[1, 0] == 0.05 and h1[1, 1] == -0.5
    assert h2[0, 0, 0, 0] == 0.5
    for idx in [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1)]:
        assert h2[idx] == 0.25
    for idx in [(1, 0, 1, 0), (0, 1, 1, 0), (1, 0, 0, 1), (0, 1, 0, 1)]:
        assert h2[idx] == 0.125
    assert h2[1, 1, 0, 0] == h2[0, 0, 1, 1] == -0.3
    assert h2[1, 1, 1, 1] == 0.7


def test_fcidump_round_trip(tmp_path):
    h1, h2 = synth.make_hamiltonian(5, 1234)
    p = tmp_path / "h.fcidump"
    vqe.write_fcidump(str(p), h1, h2, n_elec=4, e_core=-1.5)
    n, nelec, ms2, g1, g2, e_core = vqe.read_fcidump(str(p))
    assert (n, nelec, ms2, e_core) == (5, 4, 0, -1.5)
    assert np.array_equal(g1, h1) and np.array_equal(g2, h2)


class OracleSolver:
    """Stands in for the GPU solver: energy_and_grad from the CPU oracle."""

    def __init__(self, orc, nq, hf):
        import torch
        self.orc, self.nq, self.hf, self.device = orc, nq, hf, torch.device("cpu")

    def energy_and_grad(self, theta, exc, thr, h1, h2):
        import torch
        E, g, _ = self.orc.energy_and_grad(self.nq, [self.hf], [1.0], exc, theta[0].numpy(), thr, h1.numpy(),
                                           h2.numpy())
        return torch.tensor([E], dtype=torch.float64), torch.tensor(g, dtype=torch.float64)[None, :]


@pytest.mark.parametrize("method", ["L-BFGS-B", "SLSQP"])
def test_minimize_reaches_near_fci(orc, method):
    """8 qubits, 4 electrons: the optimised factorised UCCSD energy is above
    FCI (variational) and within 1 mHa of it; the gradient vanishes there."""
    h1, h2 = synth.make_hamiltonian(4, 1001)
    exc = synth.ordered_excitations(h1, h2, 2)
    hf = synth.hf_det(2)
    jw = DenseJW(8)
    efci = jw.fci(jw.h_literal(h1, h2), 2, 2)
    res, hist = vqe.minimize(OracleSolver(orc, 8, hf), exc, h1, h2, np.zeros(exc.shape[0]), method=method,
                             maxiter=300)
    ehf = hist[0][1]
    assert res.fun >= efci - 1e-10
    assert res.fun - efci < 1e-3 < ehf - efci
    _, g, _ = orc.energy_and_grad(8, [hf], [1.0], exc, res.x, 0.0, h1, h2)
    assert np.max(np.abs(g)) < 1e-4
