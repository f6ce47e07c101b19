"""GPU parity for open-shell states (alpha and beta electron counts differ,
one of them possibly zero): the excitation classes that sigma enumerates per
determinant then differ in size per spin, and some are empty."""
import math

import numpy as np
import pytest
import torch

from gpu_common import TOL, compare_states, say
from paper_2301_05726_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swc():
    from paper_2301_05726_amd import swc as s
    s.lib()
    assert torch.cuda.is_available()
    return s


CASES = [
    # (name, n_orb, n_alpha, n_beta, sigma, seed, threshold)
    ("q12_3a2b", 6, 3, 2, 0.2, 121, 0.0),
    ("q12_3a2b_thr", 6, 3, 2, 0.25, 122, 2e-3),
    ("q14_4a2b", 7, 4, 2, 0.15, 123, 0.0),
    ("q14_5a2b_thr", 7, 5, 2, 0.1, 124, 1e-4),
    ("q10_3a0b", 5, 3, 0, 0.3, 125, 0.0),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_open_shell_vs_oracle(swc, orc, case, prec):
    name, n_orb, na, nb, sigma, seed, thr = case
    say(f"[case] open shell {name} prec={prec} thr={thr}")
    h1, h2 = synth.make_hamiltonian(n_orb, seed)
    exc = synth.open_shell_excitations(n_orb, na, nb)
    theta = synth.make_theta(exc.shape[0], sigma, seed + 1)[None, :]
    ref = synth.open_shell_det(na, nb)
    nq = 2 * n_orb
    tol = TOL[prec]
    orc.set_nearcut_window(1e-5)
    d_ref, a_ref, nc, du_ref = orc.apply_ucc(nq, [ref], [1.0], exc, theta[0], thr)
    E_ref, g_ref, nc2 = orc.energy_and_grad(nq, [ref], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0 and nc2 == 0, "test instance must have no amplitude near the cut"
    cap = 64
    while cap < 2 * math.comb(n_orb, na) * math.comb(n_orb, nb):
        cap *= 2
    s = swc.Solver(nq, na, nb, cap, prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state()
    d0, _ = s.get_state(0)
    assert list(d0) == [ref]
    s.apply_ucc(theta, exc, thr)
    assert s.stats()["det_updates"] == du_ref
    d, a = s.get_state(0)
    compare_states(d, a, d_ref, a_ref, tol["amp"])
    E = s.energy(h1, h2).cpu().numpy()[0]
    assert abs(E - E_ref) <= tol["E"]
    # the same state's energy with the doubles of sigma by pairing
    s.set_sigma_scratch(64 << 20, mode=1)
    E_pair = s.energy(h1, h2).cpu().numpy()[0]
    assert s.stats()["sigma_partitions"] >= 1
    say(f"  N={len(d)} dE={abs(E - E_ref):.3e} pair-probe={E_pair - E:.3e}")
    assert abs(E_pair - E) <= 1e-12 * abs(E_ref)
    s.set_sigma_scratch(0)
    E2, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    E2 = E2.cpu().numpy()[0]
    g = g.cpu().numpy()[0]
    say(f"  grad: dE={abs(E2 - E_ref):.3e} max|dg|={np.max(np.abs(g - g_ref)):.3e}")
    assert abs(E2 - E_ref) <= tol["E"]
    assert np.max(np.abs(g - g_ref)) <= tol["g"]
    s.close()
