"""Captured sweeps on one context across calls that change what a capture
bakes in: the excitation list (which neighbouring factors share a launch)
and the live-count tracking.  Checked against the oracle."""
import numpy as np
import pytest
import torch

from gpu_common import capacity_for, compare_states, say, small_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swc():
    from paper_2301_05726_amd import swc as s
    s.lib()
    assert torch.cuda.is_available()
    return s


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_new_excitation_list_with_equal_neighbour_masks(swc, orc, prec):
    """List A fuses its first two factors into one launch at threshold 0;
    list B (same length, so the same step ranges) repeats its first factor,
    which must not be fused.  B's gradient after A's on the same context
    equals the oracle's."""
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 141)
    excB = exc.copy()
    excB[1] = excB[0]
    say(f"[case] excitation list change prec={prec}")
    s = swc.Solver(12, 3, 3, capacity_for(6, 3), prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state()
    tol_E, tol_g = (1e-10, 1e-8) if prec == 0 else (1e-6, 1e-5)
    for ex in (exc, excB, exc):
        E_ref, g_ref, _ = orc.energy_and_grad(12, [hf], [1.0], ex, theta[0], 0.0, h1, h2)
        E, g = s.energy_and_grad(theta, ex, 0.0, h1, h2)
        assert abs(E.cpu().numpy()[0] - E_ref) <= tol_E
        assert np.max(np.abs(g.cpu().numpy()[0] - g_ref)) <= tol_g
        s.apply_ucc(theta, ex, 0.0)
        d, a = s.get_state(0)
        d_ref, a_ref, _, _ = orc.apply_ucc(12, [hf], [1.0], ex, theta[0], 0.0)
        compare_states(d, a, d_ref, a_ref, 1e-12 if prec == 0 else 2e-5)
        s.build_state()
    s.close()


@pytest.mark.parametrize("thr", [0.0, 1e-3])
def test_live_tracking_switched_on_after_captures(swc, orc, thr):
    """Sweeps captured before swc_track_live(1) must not be replayed without
    the live-count array once it is on."""
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 142)
    say(f"[case] live tracking after capture thr={thr}")
    s = swc.Solver(12, 3, 3, capacity_for(6, 3), prec=0, batch=1, max_factors=exc.shape[0])
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    s.energy_and_grad(theta, exc, thr, h1, h2)
    n_ref = orc.live_trajectory(12, [hf], [1.0], exc, theta[0], thr)
    s.track_live(True)
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    assert np.array_equal(s.live_counts(0), n_ref)
    s.energy_and_grad(theta, exc, thr, h1, h2)
    assert np.array_equal(s.live_counts(0), n_ref)
    s.track_live(False)
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    d, a = s.get_state(0)
    d_ref, a_ref, _, _ = orc.apply_ucc(12, [hf], [1.0], exc, theta[0], thr)
    compare_states(d, a, d_ref, a_ref, 1e-12)
    s.close()
