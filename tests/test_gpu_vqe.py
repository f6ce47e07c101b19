"""The outer loop on the GPU: scipy minimisation driven by the library's
energy and adjoint gradient, from an FCIDUMP file to a converged energy."""
import numpy as np
import pytest
import torch

from gpu_common import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_minimize_on_gpu_matches_oracle(orc, prec, tmp_path):
    from paper_2301_05726_amd import swc, synth, vqe
    from dense_jw import DenseJW
    h1, h2 = synth.make_hamiltonian(4, 1001)
    p = tmp_path / "q8.fcidump"
    vqe.write_fcidump(str(p), h1, h2, n_elec=4)
    n, nelec, ms2, h1, h2, e_core = vqe.read_fcidump(str(p))
    exc = synth.ordered_excitations(h1, h2, 2)
    hf = synth.hf_det(2)
    s = swc.Solver(8, 2, 2, 256, prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state()
    res, hist = vqe.minimize(s, exc, h1, h2, np.zeros(exc.shape[0]), method="L-BFGS-B", maxiter=300)
    jw = DenseJW(8)
    efci = jw.fci(jw.h_literal(h1, h2), 2, 2)
    e_or = orc.energy_theta(8, [hf], [1.0], exc, res.x, 0.0, h1, h2)
    say(f"[case] vqe prec={prec}: E={res.fun:.10f} FCI={efci:.10f} evals={len(hist)} oracle(E(x*))={e_or:.10f}")
    tol = 1e-10 if prec == 0 else 1e-6
    assert abs(res.fun - e_or) <= tol
    assert e_or >= efci - 1e-10
    assert res.fun - efci < 1e-5
    s.close()


def test_vqe_cli(tmp_path, capsys):
    from paper_2301_05726_amd import synth, vqe
    h1, h2 = synth.make_hamiltonian(4, 1001)
    p = tmp_path / "q8.fcidump"
    vqe.write_fcidump(str(p), h1, h2, n_elec=4, e_core=1.0)
    assert vqe.main(["--fcidump", str(p), "--capacity-log2", "10", "--maxiter", "100"]) == 0
    out = capsys.readouterr().out
    assert "L-BFGS-B: E = " in out and "success=True" in out
