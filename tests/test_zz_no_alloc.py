"""swc_energy_noalloc (no device allocation: its scratch is a static device
array) against swc_build_state + swc_energy on the same states, through the
C ABI: several calls in a row on the one scratch array, the second with a
smaller state, then its size limit and its device-side input checks."""
import numpy as np
import pytest
import torch

from gpu_common import TOL, capacity_for, say, small_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def swc():
    from paper_2301_05726_amd import swc as s
    s.lib()
    assert torch.cuda.is_available()
    return s


def ucc_state(swc, nq, n_occ, cap, exc, theta, thr):
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=swc.FP64, batch=1, max_factors=exc.shape[0])
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    d, a = s.get_state(0)
    s.close()
    return d, a


def energy_with_context(swc, nq, n_occ, cap, d, a, h1, h2):
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=swc.FP64, batch=1, max_factors=1)
    s.build_state(d, a)
    E = float(s.energy(h1, h2).cpu().item())
    s.close()
    return E


def energy_noalloc(swc, nq, d, a, h1, h2):
    dev = torch.device("cuda:0")
    dt = torch.from_numpy(d.view(np.int64).copy()).to(dev)
    at = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    h1t = torch.from_numpy(np.ascontiguousarray(h1, dtype=np.float64)).to(dev)
    h2t = torch.from_numpy(np.ascontiguousarray(h2, dtype=np.float64)).to(dev)
    E = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    swc.energy_noalloc(nq, dt, at, h1t, h2t, E)
    return float(E.cpu().item())


def test_noalloc_matches_context_energy(swc):
    from paper_2301_05726_amd import synth
    tol = TOL[0]["E"]
    # 1: the 20-qubit workload's full state (63,504 determinants, near the
    # 65,536 maximum)
    wl = synth.WORKLOADS["q20"]
    p = synth.make_problem(wl, batch=1)
    d1, a1 = ucc_state(swc, wl.n_qubits, wl.n_occ, wl.capacity, p.exc, p.theta, wl.threshold)
    say(f"[case] noalloc q20 state n={d1.size}")
    assert 60000 < d1.size <= swc.NOALLOC_MAX_DETS
    E1_ref = energy_with_context(swc, wl.n_qubits, wl.n_occ, wl.capacity, d1, a1, p.h1, p.h2)
    E1 = energy_noalloc(swc, wl.n_qubits, d1, a1, p.h1, p.h2)
    say(f"  E={E1:.15f} ref={E1_ref:.15f} |dE|={abs(E1 - E1_ref):.2e}")
    assert abs(E1 - E1_ref) <= tol
    # 2: a smaller state on other qubits, in the same scratch array (the
    # first call's contents still there)
    h1, h2, exc, theta, _ = small_problem(6, 3, 0.3, 511)
    d2, a2 = ucc_state(swc, 12, 3, capacity_for(6, 3), exc, theta, 1e-3)
    say(f"[case] noalloc 12-qubit state n={d2.size}")
    assert d2.size < d1.size
    E2_ref = energy_with_context(swc, 12, 3, capacity_for(6, 3), d2, a2, h1, h2)
    E2 = energy_noalloc(swc, 12, d2, a2, h1, h2)
    say(f"  E={E2:.15f} ref={E2_ref:.15f} |dE|={abs(E2 - E2_ref):.2e}")
    assert abs(E2 - E2_ref) <= tol
    # 3: an unnormalised subset (the energy is the Rayleigh quotient)
    d3, a3 = d2[::3].copy(), 2.5 * a2[::3]
    E3_ref = energy_with_context(swc, 12, 3, capacity_for(6, 3), d3, a3, h1, h2)
    E3 = energy_noalloc(swc, 12, d3, a3, h1, h2)
    say(f"[case] noalloc subset n={d3.size}: |dE|={abs(E3 - E3_ref):.2e}")
    assert abs(E3 - E3_ref) <= tol
    # 4: the first state again gives the first result, bit for bit
    assert energy_noalloc(swc, wl.n_qubits, d1, a1, p.h1, p.h2) == E1


def test_noalloc_rejects_bad_input(swc):
    h1, h2, exc, theta, _ = small_problem(6, 3, 0.3, 512)
    d, a = ucc_state(swc, 12, 3, capacity_for(6, 3), exc, theta, 0.0)
    say(f"[case] noalloc input checks n={d.size}")
    # above the maximum: refused before any device work
    big = np.arange(swc.NOALLOC_MAX_DETS + 1, dtype=np.uint64)
    with pytest.raises(swc.SwcError) as e:
        energy_noalloc(swc, 12, big, np.ones(big.size), h1, h2)
    assert e.value.code == swc.EINVAL and "65,536" in str(e.value)
    # found by the device checks
    dup = np.concatenate([d, d[:1]])
    with pytest.raises(swc.SwcError) as e:
        energy_noalloc(swc, 12, dup, np.concatenate([a, a[:1]]), h1, h2)
    assert e.value.code == swc.EINVAL
    high = d.copy()
    high[0] |= np.uint64(1 << 12)
    with pytest.raises(swc.SwcError) as e:
        energy_noalloc(swc, 12, high, a, h1, h2)
    assert e.value.code == swc.EINVAL
    bad = a.copy()
    bad[-1] = np.inf
    with pytest.raises(swc.SwcError) as e:
        energy_noalloc(swc, 12, d, bad, h1, h2)
    assert e.value.code == swc.EINVAL
    with pytest.raises(swc.SwcError) as e:
        energy_noalloc(swc, 12, d, np.zeros(d.size), h1, h2)
    assert e.value.code == swc.EINVAL
    # and a good call afterwards still agrees
    E_ref = energy_with_context(swc, 12, 3, capacity_for(6, 3), d, a, h1, h2)
    assert abs(energy_noalloc(swc, 12, d, a, h1, h2) - E_ref) <= TOL[0]["E"]
