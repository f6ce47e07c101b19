"""sigma by pairing determinants on two-electron-removed keys (device radix
sort) against the hash-probe path and the oracle, through the C ABI."""
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


CASES = [
    ("q8", 4, 2, 0.3, 101, None, 0.0),
    ("q12", 6, 3, 0.2, 102, None, 0.0),
    ("q16_thr", 8, 4, 0.1, 105, None, 1e-4),
    ("q20_pre", 10, 5, 0.05, 106, 160, 0.0),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_pairing_sigma_matches_probes_and_oracle(swc, orc, case, prec):
    name, n_orb, n_occ, sigma, seed, nf, thr = case
    say(f"[case] pairs {name} prec={prec}")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    nq = 2 * n_orb
    cap = capacity_for(n_orb, n_occ)
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    E_probe = s.energy(h1, h2).cpu().numpy()[0]
    assert s.stats()["sigma_partitions"] == 0
    s.set_sigma_scratch(64 << 20, mode=1)
    E_pair = s.energy(h1, h2).cpu().numpy()[0]
    assert s.stats()["sigma_partitions"] >= 1
    E_pair2 = s.energy(h1, h2).cpu().numpy()[0]
    assert E_pair == E_pair2
    d, a = s.get_state(0)
    E_ref = orc.energy(n_orb, h1, h2, d, a)
    say(f"  E pair-probe {E_pair - E_probe:.3e}, pair-oracle(same state) {E_pair - E_ref:.3e}")
    assert abs(E_pair - E_probe) <= 1e-12 * abs(E_ref)
    assert abs(E_pair - E_ref) <= 1e-11
    orc.set_nearcut_window(1e-5)
    E_g, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    E_or, g_or, nc = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0
    assert abs(E_g.cpu().numpy()[0] - E_or) <= TOL[prec]["E"]
    assert np.max(np.abs(g.cpu().numpy()[0] - g_or)) <= TOL[prec]["g"]
    s.close()


def test_pairing_sigma_many_partitions(swc):
    """A scratch far smaller than the record count: the records are split
    into hash partitions of K; the energy does not change."""
    h1, h2, exc, theta, hf = small_problem(10, 5, 0.05, 106, 160)
    s = swc.Solver(20, 5, 5, 1 << 17, prec=0, batch=1, max_factors=exc.shape[0])
    s.build_state()
    s.apply_ucc(theta, exc, 0.0)
    n = s.stats()["n_live"]
    s.set_sigma_scratch(64 << 20, mode=1)
    E1 = s.energy(h1, h2).cpu().numpy()[0]
    records = n * 45
    s.set_sigma_scratch(24 * (1 << 17) + 41 * (records // 7) + (1 << 20), mode=1)
    E2 = s.energy(h1, h2).cpu().numpy()[0]
    parts = s.stats()["sigma_partitions"]
    say(f"[case] pairs partitions={parts} dE={E2 - E1:.3e}")
    assert parts >= 7
    assert abs(E2 - E1) <= 1e-13 * abs(E1)
    s.close()


@pytest.mark.parametrize("name,K,B", [("q32", 200, 1), ("q48", 150, 2), ("q64", 300, 1)])
def test_pairing_sigma_workload_prefixes(swc, orc, name, K, B):
    from paper_2301_05726_amd import synth
    wl = synth.WORKLOADS[name]
    p = synth.make_problem(wl, batch=B, n_factors=K)
    s = swc.Solver(wl.n_qubits, wl.n_occ, wl.n_occ, wl.capacity, prec=1, batch=B, max_factors=p.M)
    s.set_sigma_scratch(256 << 20, mode=1)
    s.build_state()
    E, g = s.energy_and_grad(p.theta, p.exc, wl.threshold, p.h1, p.h2)
    E, g = E.cpu().numpy(), g.cpu().numpy()
    orc.set_nearcut_window(1e-5)
    for b in range(B):
        E_ref, g_ref, nc = orc.energy_and_grad(wl.n_qubits, [p.hf], [1.0], p.exc, p.theta[b], wl.threshold, p.h1,
                                               p.h2)
        assert nc == 0
        say(f"[case] pairs {name} b={b} dE={abs(E[b] - E_ref):.3e} max|dg|={np.max(np.abs(g[b] - g_ref)):.3e}")
        assert abs(E[b] - E_ref) <= TOL[1]["E"]
        assert np.max(np.abs(g[b] - g_ref)) <= TOL[1]["g"]
    s.close()
