"""Degenerate inputs through the C ABI against the oracle: the empty circuit,
a single factor at a quarter turn (the pair swaps), all angles zero (the
gradient is 2<HF|[H, tau_k]|HF>), and an initial state with an exact zero
amplitude kept by threshold 0."""
import numpy as np
import pytest
import torch

from gpu_common import TOL, capacity_for, compare_states, say, small_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swc():
    from paper_2301_05726_amd import swc as s
    s.lib()
    assert torch.cuda.is_available()
    return s


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_empty_circuit(swc, orc, prec):
    say(f"[case] empty circuit prec={prec}")
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 151)
    e0 = exc[:0].copy()
    t0 = np.zeros((2, 0))
    s = swc.Solver(12, 3, 3, 1024, prec=prec, batch=2, max_factors=exc.shape[0])
    s.build_state()
    s.apply_ucc(t0, e0, 0.0)
    d, a = s.get_state(1)
    assert list(d) == [hf] and a.tolist() == [1.0]
    E_ref = orc.energy(6, h1, h2, [hf], [1.0])
    E = s.energy(h1, h2).cpu().numpy()
    E2, g = s.energy_and_grad(t0, e0, 0.0, h1, h2)
    assert g.shape == (2, 0)
    for e in (E, E2.cpu().numpy()):
        assert np.all(np.abs(e - E_ref) <= 1e-12 * abs(E_ref))
    s.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_quarter_turn_swaps_the_pair(swc, orc, prec):
    say(f"[case] single factor at pi/2 prec={prec}")
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 152)
    e1 = exc[:1].copy()
    t1 = np.array([[np.pi / 2]])
    s = swc.Solver(12, 3, 3, 1024, prec=prec, batch=1, max_factors=1)
    s.build_state()
    s.apply_ucc(t1, e1, 1e-6)  # HF keeps cos(pi/2) ~ 6e-17: removed by any threshold
    d, a = s.get_state(0)
    d_ref, a_ref, nc, _ = orc.apply_ucc(12, [hf], [1.0], e1, t1[0], 1e-6)
    assert len(d_ref) == 1 and hf not in list(d_ref)
    compare_states(d, a, d_ref, a_ref, TOL[prec]["amp"])
    assert abs(abs(a[0]) - 1.0) < 1e-7
    E_ref, g_ref, _ = orc.energy_and_grad(12, [hf], [1.0], e1, t1[0], 1e-6, h1, h2)
    E, g = s.energy_and_grad(t1, e1, 1e-6, h1, h2)
    assert abs(E.item() - E_ref) <= TOL[prec]["E"]
    assert np.max(np.abs(g.cpu().numpy()[0] - g_ref)) <= TOL[prec]["g"]
    s.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_zero_angles(swc, orc, prec):
    say(f"[case] all angles zero prec={prec}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 153)
    t = np.zeros((1, exc.shape[0]))
    s = swc.Solver(16, 4, 4, capacity_for(8, 4), prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state()
    E, g = s.energy_and_grad(t, exc, 0.0, h1, h2)
    E_ref, g_ref, _ = orc.energy_and_grad(16, [hf], [1.0], exc, t[0], 0.0, h1, h2)
    assert abs(E.item() - E_ref) <= TOL[prec]["E"]
    assert np.max(np.abs(g.cpu().numpy()[0] - g_ref)) <= TOL[prec]["g"]
    # at theta = 0 every created partner has amplitude 0: threshold 0 keeps them
    s.apply_ucc(t, exc, 0.0)
    d, a = s.get_state(0)
    d_ref, a_ref, _, _ = orc.apply_ucc(16, [hf], [1.0], exc, t[0], 0.0)
    compare_states(d, a, d_ref, a_ref, TOL[prec]["amp"])
    s.close()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_initial_zero_amplitude_kept(swc, orc, prec):
    say(f"[case] initial state with a zero amplitude prec={prec}")
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 154, 40)
    d0 = [hf, hf ^ 0b11110000, hf ^ 0b100000100]  # HF, a double, a single (3 alpha + 3 beta each)
    a0 = [0.8, 0.0, 0.6]
    s = swc.Solver(12, 3, 3, 1024, prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state(d0, a0)
    s.apply_ucc(theta, exc, 0.0)
    d, a = s.get_state(0)
    d_ref, a_ref, _, _ = orc.apply_ucc(12, d0, a0, exc, theta[0], 0.0)
    compare_states(d, a, d_ref, a_ref, TOL[prec]["amp"])
    s.build_state(d0, a0)
    E, g = s.energy_and_grad(theta, exc, 0.0, h1, h2)
    E_ref, g_ref, _ = orc.energy_and_grad(12, d0, a0, exc, theta[0], 0.0, h1, h2)
    assert abs(E.item() - E_ref) <= TOL[prec]["E"]
    assert np.max(np.abs(g.cpu().numpy()[0] - g_ref)) <= TOL[prec]["g"]
    s.close()


@pytest.mark.parametrize("thr", [0.0, 1e-4], ids=["thr0", "thr"])
def test_gradient_calls_around_other_calls(swc, orc, thr):
    """A gradient call that follows another starts from the table the first
    one left; every call that changes the state or the settings in between
    makes the next one rebuild |Psi_0>. All results are bit-identical."""
    say(f"[case] gradient calls around other calls thr={thr}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 162)  # no amplitude within 1e-5 of the cut
    s = swc.Solver(16, 4, 4, capacity_for(8, 4), prec=1, batch=1, max_factors=exc.shape[0])
    s.build_state()
    E0, g0 = (x.cpu().numpy() for x in s.energy_and_grad(theta, exc, thr, h1, h2))
    orc.set_nearcut_window(1e-5)
    E_ref, g_ref, nc = orc.energy_and_grad(16, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0
    assert abs(E0[0] - E_ref) <= TOL[1]["E"] and np.max(np.abs(g0[0] - g_ref)) <= TOL[1]["g"]

    def again():
        E, g = (x.cpu().numpy() for x in s.energy_and_grad(theta, exc, thr, h1, h2))
        assert np.array_equal(E, E0) and np.array_equal(g, g0)

    again()                           # right after a gradient call
    s.apply_ucc(theta, exc, thr)      # the table now holds the circuit's output
    again()
    s.energy(h1, h2)
    again()
    s.get_state(0)
    again()
    s.set_topk(0, 0)
    again()
    s.track_live(True)
    again()
    s.build_state()
    again()
    d, a = s.get_state(0)
    assert list(d) == [hf] and a.tolist() == [1.0]
    s.close()
