"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on
the same seeded inputs, element by element."""
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


CASES = [
    # (name, n_orb, n_occ, sigma, seed, n_factors, threshold)
    ("q8", 4, 2, 0.3, 101, None, 0.0),
    ("q12", 6, 3, 0.2, 102, None, 0.0),
    ("q12_thr", 6, 3, 0.25, 103, None, 2e-3),
    ("q16", 8, 4, 0.1, 104, None, 0.0),
    ("q16_thr", 8, 4, 0.1, 105, None, 1e-4),
    ("q20_pre", 10, 5, 0.05, 106, 160, 0.0),
    ("q20_pre_thr", 10, 5, 0.05, 107, 300, 1e-5),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forward_energy_grad_vs_oracle(swc, orc, case, prec):
    name, n_orb, n_occ, sigma, seed, nf, thr = case
    say(f"[case] {name} prec={prec} thr={thr}")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    nq = 2 * n_orb
    tol = TOL[prec]
    orc.set_nearcut_window(1e-5)
    d_ref, a_ref, nc, du_ref = orc.apply_ucc(nq, [hf], [1.0], exc, theta[0], thr)
    E_ref, g_ref, nc2 = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
    say(f"  oracle N={len(d_ref)} nearcut={nc} E={E_ref:.12f}")
    assert nc == 0, "test instance must have no amplitude near the cut"
    cap = capacity_for(n_orb, n_occ)
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=prec, batch=1, max_factors=exc.shape[0])
    s.track_live(True)
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    # det-updates: live determinants when each step begins, summed (exact count)
    assert s.stats()["det_updates"] == du_ref
    # and the live count before every step and after the last (exact)
    n_ref = orc.live_trajectory(nq, [hf], [1.0], exc, theta[0], thr)
    assert np.array_equal(s.live_counts(0), n_ref)
    d, a = s.get_state(0)
    err = compare_states(d, a, d_ref, a_ref, tol["amp"])
    E = s.energy(h1, h2).cpu().numpy()[0]
    say(f"  gpu N={len(d)} amp_err={err:.3e} dE={abs(E - E_ref):.3e}")
    assert abs(E - E_ref) <= tol["E"]
    E2, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    E2 = E2.cpu().numpy()[0]
    g = g.cpu().numpy()[0]
    say(f"  grad: dE={abs(E2 - E_ref):.3e} max|dg|={np.max(np.abs(g - g_ref)):.3e}")
    assert abs(E2 - E_ref) <= tol["E"]
    assert np.max(np.abs(g - g_ref)) <= tol["g"]
    assert np.array_equal(s.live_counts(0), n_ref)  # the gradient's forward sweep
    # energy_and_grad leaves |Psi_0>
    d0, a0 = s.get_state(0)
    assert list(d0) == [hf] and abs(a0[0] - 1.0) < 1e-15
    s.close()


def test_batch_members_independent(swc, orc):
    say("[case] batch3 q12")
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 111, batch=3)
    s = swc.Solver(12, 3, 3, 1024, prec=0, batch=3, max_factors=exc.shape[0])
    s.build_state()
    E, g = s.energy_and_grad(theta, exc, 0.0, h1, h2)
    E = E.cpu().numpy()
    g = g.cpu().numpy()
    for b in range(3):
        E_ref, g_ref, _ = orc.energy_and_grad(12, [hf], [1.0], exc, theta[b], 0.0, h1, h2)
        assert abs(E[b] - E_ref) < 1e-10
        assert np.max(np.abs(g[b] - g_ref)) < 1e-8
    s.apply_ucc(theta, exc, 0.0)
    for b in range(3):
        d, a = s.get_state(b)
        d_ref, a_ref, _, _ = orc.apply_ucc(12, [hf], [1.0], exc, theta[b], 0.0)
        compare_states(d, a, d_ref, a_ref, 1e-12)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_batch_members_launched_apart(swc, orc, monkeypatch, prec):
    """One-factor step launches of one batch member each (what large batched
    states use: SWC_SPLIT=1 forces them at any size) give the bits of one
    launch for all members, and the oracle's values for every member; the
    index grows during the forward sweep."""
    say(f"[case] batch3 q16 members launched apart prec={prec}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 181, batch=3)
    M, thr = exc.shape[0], 1e-4
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    res = {}
    for split in ("0", "1"):
        monkeypatch.setenv("SWC_SPLIT", split)
        s = swc.Solver(16, 4, 4, capacity_for(8, 4), prec=prec, batch=3, max_factors=M)
        s.build_state()
        E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
        st = s.stats()
        res[split] = (E.cpu().numpy(), g.cpu().numpy(), st["rotate_launches"], st["reverse_launches"],
                      st["rehashes"])
        s.close()
    (E0, g0, f0, r0, h0), (E1, g1, f1, r1, h1_) = res["0"], res["1"]
    say(f"  launches forward {f0} -> {f1}, reverse {r0} -> {r1}, growths {h0}")
    assert h0 == h1_ > 0
    assert f1 == 3 * f0 and r1 == 3 * r0
    assert E1.tobytes() == E0.tobytes() and g1.tobytes() == g0.tobytes()
    tol = TOL[prec]
    for b in range(3):
        E_ref, g_ref, _ = orc.energy_and_grad(16, [hf], [1.0], exc, theta[b], thr, h1, h2)
        assert abs(E1[b] - E_ref) <= tol["E"]
        assert np.max(np.abs(g1[b] - g_ref)) <= tol["g"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("batch", [1, 2], ids=["b1", "b2_apart"])
def test_forward_high_occupancy_build(swc, orc, monkeypatch, prec, batch):
    """The forward build for more resident waves per SIMD (what indexes of
    2^22 slots and more use: SWC_HIOCC=1 forces it at any size; with two
    members, launched one member each) gives the bits of the lighter build
    and the oracle's values; the index grows during the forward sweep."""
    say(f"[case] forward high-occupancy build q16 batch{batch} prec={prec}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 187, batch=batch)
    M, thr = exc.shape[0], 1e-4
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    monkeypatch.setenv("SWC_SPLIT", "1" if batch > 1 else "0")
    res = {}
    for ho in ("0", "1"):
        monkeypatch.setenv("SWC_HIOCC", ho)
        s = swc.Solver(16, 4, 4, capacity_for(8, 4), prec=prec, batch=batch, max_factors=M)
        s.build_state()
        E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
        st = s.stats()
        res[ho] = (E.cpu().numpy(), g.cpu().numpy(), st["kernel_builds"], st["rehashes"])
        s.close()
    (E0, g0, b0, h0), (E1, g1, b1, h1_) = res["0"], res["1"]
    say(f"  builds {b0:#x} -> {b1:#x}, growths {h0}")
    assert h0 == h1_ > 0
    assert b0 & swc.BUILD_FWD and not b0 & swc.BUILD_FWD_HO
    assert b1 & swc.BUILD_FWD_HO and not b1 & swc.BUILD_FWD
    assert E1.tobytes() == E0.tobytes() and g1.tobytes() == g0.tobytes()
    tol = TOL[prec]
    for b in range(batch):
        E_ref, g_ref, _ = orc.energy_and_grad(16, [hf], [1.0], exc, theta[b], thr, h1, h2)
        assert abs(E1[b] - E_ref) <= tol["E"]
        assert np.max(np.abs(g1[b] - g_ref)) <= tol["g"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("shape", ["b1", "b2_apart", "b1_hiocc"])
def test_presence_filter_probes(swc, orc, monkeypatch, prec, shape):
    """Steps whose probes consult the index's presence filter first
    (SWC_PFILTER=2: forward and reverse at every index size; by themselves
    the library's forward steps use it from 2^22 index slots on, its reverse
    steps at every size) give the bits of the plain probes and the oracle's
    values: the forward sweep creates entries, grows the index (the filter is
    rebuilt with it) and is undone by the adjoint sweep; a second call reuses
    the state's filter after the reset."""
    say(f"[case] presence filter q16 {shape} prec={prec}")
    batch = 2 if shape == "b2_apart" else 1
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 191, batch=batch)
    M, thr = exc.shape[0], 1e-4
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    monkeypatch.setenv("SWC_SPLIT", "1" if batch > 1 else "0")
    monkeypatch.setenv("SWC_HIOCC", "1" if shape == "b1_hiocc" else "0")
    res = {}
    for pf in ("0", "1", "2"):
        monkeypatch.setenv("SWC_PFILTER", pf)
        s = swc.Solver(16, 4, 4, capacity_for(8, 4), prec=prec, batch=batch, max_factors=M)
        s.build_state()
        out = []
        for rep in range(2):
            E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
            st = s.stats()
            out.append((E.cpu().numpy(), g.cpu().numpy(), st["kernel_builds"], st["rehashes"]))
        s.apply_ucc(theta, exc, thr)
        states = [s.get_state(b) for b in range(batch)]
        res[pf] = (out, states)
        s.close()
    o0, st0 = res["0"]
    for pf, fwd_pf in (("1", False), ("2", True)):  # "1": an index this small keeps forward steps plain
        o1, st1 = res[pf]
        for (E0, g0, b0, h0), (E1, g1, b1, h1_) in zip(o0, o1):
            say(f"  SWC_PFILTER={pf}: builds {b0:#x} -> {b1:#x}, growths {h0}")
            assert h0 == h1_
            assert not b0 & (swc.BUILD_FWD_PF | swc.BUILD_REV_PF)
            assert bool(b1 & swc.BUILD_FWD_PF) == fwd_pf and b1 & swc.BUILD_REV_PF
            assert E1.tobytes() == E0.tobytes() and g1.tobytes() == g0.tobytes()
        for (d0, a0), (d1, a1) in zip(st0, st1):
            assert np.array_equal(d0, d1) and a0.tobytes() == a1.tobytes()
    assert o0[0][3] > 0  # the first call grew the index
    o1 = res["2"][0]
    tol = TOL[prec]
    E1, g1 = o1[0][0], o1[0][1]
    for b in range(batch):
        E_ref, g_ref, _ = orc.energy_and_grad(16, [hf], [1.0], exc, theta[b], thr, h1, h2)
        assert abs(E1[b] - E_ref) <= tol["E"]
        assert np.max(np.abs(g1[b] - g_ref)) <= tol["g"]


@pytest.mark.parametrize("seed,thr", [(191, 1e-4), (192, 0.0)], ids=["thr1e-4", "thr0"])
def test_presence_filter_chosen_from_last_sweep(swc, orc, monkeypatch, seed, thr):
    """With SWC_PFILTER unset a call's reverse steps probe through the
    filter (rebuilt from the entries, since forward steps on an index this
    small do without it) unless the last completed forward sweep found the
    partner of more than 1 rotated pair in 4 (threshold 0, one factor per
    launch: most partners exist); the results match the oracle."""
    say(f"[case] presence filter policy q16 seed={seed} thr={thr}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, seed)
    monkeypatch.delenv("SWC_PFILTER", raising=False)
    monkeypatch.setenv("SWC_FUSE", "0")
    s = swc.Solver(16, 4, 4, capacity_for(8, 4), prec=0, batch=1, max_factors=exc.shape[0])
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    st = s.stats()
    # (an index this small: forward steps without the filter)
    assert not st["kernel_builds"] & swc.BUILD_FWD_PF
    expect = st["partner_hits"] <= st["pair_updates"] // 4
    say(f"  pairs {st['pair_updates']} hits {st['partner_hits']} -> filter {expect}")
    E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    got = s.stats()["kernel_builds"]
    assert not got & swc.BUILD_FWD_PF and bool(got & swc.BUILD_REV_PF) == expect
    E_ref, g_ref, _ = orc.energy_and_grad(16, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert abs(E.cpu().numpy()[0] - E_ref) <= TOL[0]["E"]
    assert np.max(np.abs(g.cpu().numpy()[0] - g_ref)) <= TOL[0]["g"]
    s.close()


def test_bitwise_reproducible(swc):
    say("[case] determinism q16 thr")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 121)
    out = []
    for prec in (0, 1):
        for rep in range(2):
            s = swc.Solver(16, 4, 4, 16384, prec=prec, batch=1, max_factors=exc.shape[0])
            s.build_state()
            E, g = s.energy_and_grad(theta, exc, 1e-4, h1, h2)
            out.append((prec, E.cpu().numpy().tobytes(), g.cpu().numpy().tobytes()))
            s.close()
    assert out[0] == out[1] and out[2] == out[3]


def test_custom_initial_state_and_sequential_calls(swc, orc):
    say("[case] initial state + two apply calls")
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.3, 131)
    rng = np.random.default_rng(7)
    _, d0, a0 = None, None, None
    d_ref0, a_ref0, _, _ = orc.apply_ucc(12, [hf], [1.0], exc[:40], theta[0, :40], 0.0)
    dets = d_ref0[:25]
    amps = rng.normal(size=25)
    s = swc.Solver(12, 3, 3, 2048, prec=0, batch=1, max_factors=exc.shape[0])
    s.build_state(dets, amps)
    s.apply_ucc(theta[:, :50], exc[:50], 1e-3)
    s.apply_ucc(theta[:, 50:], exc[50:], 1e-3)
    d, a = s.get_state(0)
    d1, a1, nc1, _ = orc.apply_ucc(12, dets, amps, exc[:50], theta[0, :50], 1e-3)
    d2, a2, nc2, _ = orc.apply_ucc(12, d1, a1, exc[50:], theta[0, 50:], 1e-3)
    assert nc1 == 0 and nc2 == 0
    compare_states(d, a, d2, a2, 1e-12)
    E = s.energy(h1, h2).cpu().numpy()[0]
    assert abs(E - orc.energy(6, h1, h2, d2, a2)) < 1e-10


def test_error_paths(swc):
    say("[case] error paths")
    h1, h2, exc, theta, hf = small_problem(4, 2, 0.3, 141)
    s = swc.Solver(8, 2, 2, 256, prec=0, batch=1, max_factors=exc.shape[0])
    with pytest.raises(swc.SwcError) as e:
        s.apply_ucc(theta, exc, 0.0)
    assert e.value.code == swc.ESTATE
    with pytest.raises(swc.SwcError) as e:  # live counts are kept only while tracked
        s.live_counts(0)
    assert e.value.code == swc.ESTATE
    s.build_state()
    bad = exc.copy()
    bad[0] = (0, 2, 0, 6)
    with pytest.raises(swc.SwcError) as e:
        s.apply_ucc(theta, bad, 0.0)
    assert e.value.code == swc.EINVAL
    t = theta.copy()
    t[0, 3] = np.nan
    with pytest.raises(swc.SwcError) as e:
        s.apply_ucc(t, exc, 0.0)
    assert e.value.code == swc.EINVAL
    # the gradient call checks the angles together with the forward sweep's
    # status; the context stays usable and the next call is exact
    E_ok, g_ok = s.energy_and_grad(theta, exc, 0.0, h1, h2)
    with pytest.raises(swc.SwcError) as e:
        s.energy_and_grad(t, exc, 0.0, h1, h2)
    assert e.value.code == swc.EINVAL
    E_2, g_2 = s.energy_and_grad(theta, exc, 0.0, h1, h2)
    assert E_2.cpu().numpy().tobytes() == E_ok.cpu().numpy().tobytes()
    assert g_2.cpu().numpy().tobytes() == g_ok.cpu().numpy().tobytes()
    d0, a0 = s.get_state(0)
    assert list(d0) == [hf]
    with pytest.raises(swc.SwcError) as e:
        s.apply_ucc(theta, exc, -1.0)
    assert e.value.code == swc.EINVAL
    with pytest.raises(swc.SwcError) as e:
        s.apply_ucc(theta, exc, 2.0)
    assert e.value.code == swc.EEMPTY
    s.build_state()
    with pytest.raises(swc.SwcError) as e:
        s.build_state([1 << 8], [1.0])
    assert e.value.code == swc.EINVAL
    # a table too small for the state
    s2 = swc.Solver(12, 3, 3, 64, prec=0, batch=1, max_factors=200)
    s2.build_state()
    h1b, h2b, excb, thetab, _ = small_problem(6, 3, 0.3, 142)
    with pytest.raises(swc.SwcError) as e:
        s2.apply_ucc(thetab, excb, 0.0)
    assert e.value.code == swc.ECAPACITY


def test_autograd_function(swc, orc):
    say("[case] autograd")
    h1, h2, exc, theta, hf = small_problem(6, 3, 0.2, 151)
    s = swc.Solver(12, 3, 3, 1024, prec=1, batch=1, max_factors=exc.shape[0])
    s.build_state()
    th = torch.tensor(theta[0], dtype=torch.float64, device="cuda", requires_grad=True)
    E = swc.ucc_energy(th, s, exc, 0.0, h1, h2)
    (2.0 * E.sum()).backward()
    E_ref, g_ref, _ = orc.energy_and_grad(12, [hf], [1.0], exc, theta[0], 0.0, h1, h2)
    assert abs(E.item() - E_ref) < 1e-6
    assert np.max(np.abs(th.grad.cpu().numpy() - 2.0 * g_ref)) < 2e-5


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_sweep_modes_bitwise_identical(swc, monkeypatch, prec):
    """Captured-graph replay, direct per-step launches and the persistent
    cooperative sweep run the same step arithmetic: results agree to the
    bit, and repeated graph replays (with eager work in between) agree too."""
    say(f"[case] sweep modes prec={prec}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 161)
    results = {}
    for mode, env in (("graph", {}), ("direct", {"SWC_GRAPH": "0"}), ("persistent", {"SWC_SWEEP": "persistent"})):
        for k in ("SWC_GRAPH", "SWC_SWEEP"):
            monkeypatch.delenv(k, raising=False)
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        s = swc.Solver(16, 4, 4, 16384, prec=prec, batch=1, max_factors=exc.shape[0])
        s.build_state()
        reps = []
        for rep in range(3):
            E, g = s.energy_and_grad(theta, exc, 1e-4, h1, h2)
            s.apply_ucc(theta, exc, 0.0)          # eager work between replays
            d, a = s.get_state(0)
            s.build_state()
            reps.append((E.cpu().numpy().tobytes(), g.cpu().numpy().tobytes(), d.tobytes(), a.tobytes()))
        assert reps[0] == reps[1] == reps[2], mode
        results[mode] = reps[0]
        s.close()
    assert results["graph"] == results["direct"] == results["persistent"]


GROW_CASES = [
    ("q16", 8, 4, 0.1, 104, None, 0.0),
    ("q12_thr", 6, 3, 0.25, 103, None, 2e-3),
    ("q16_thr", 8, 4, 0.1, 105, None, 1e-4),
    ("q20_pre_thr", 10, 5, 0.05, 107, 300, 1e-5),
]


def _run_with_table_min(swc, monkeypatch, tmin, nq, n_occ, cap, prec, batch, exc, theta, thr, h1, h2):
    monkeypatch.setenv("SWC_TABLE_MIN", str(tmin))
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=prec, batch=batch, max_factors=exc.shape[0])
    s.track_live(True)
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    st = s.stats()
    states = [s.get_state(b) for b in range(batch)]
    E = s.energy(h1, h2).cpu().numpy()
    E2, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    st2 = s.stats()
    st2["live_counts"] = s.live_counts(0).tolist()
    s.close()
    return st, st2, states, E, E2.cpu().numpy(), g.cpu().numpy()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", GROW_CASES, ids=[c[0] for c in GROW_CASES])
def test_table_growth_exact(swc, orc, monkeypatch, case, prec):
    """A table that starts at 64 slots and is rehashed into larger ones during
    the sweep gives the same bits as a table of full capacity from the start
    (every reduction is an exact fixed-point sum and each pair rotation is
    independent of slot placement), and matches the oracle."""
    name, n_orb, n_occ, sigma, seed, nf, thr = case
    say(f"[case] growth {name} prec={prec} thr={thr}")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    nq = 2 * n_orb
    cap = capacity_for(n_orb, n_occ)
    grown = _run_with_table_min(swc, monkeypatch, 64, nq, n_occ, cap, prec, 1, exc, theta, thr, h1, h2)
    fixed = _run_with_table_min(swc, monkeypatch, cap, nq, n_occ, cap, prec, 1, exc, theta, thr, h1, h2)
    say(f"  grown: rehashes={grown[0]['rehashes']}/{grown[1]['rehashes']} table={grown[0]['table_slots']} "
        f"fixed: rehashes={fixed[0]['rehashes']} table={fixed[0]['table_slots']}")
    assert grown[0]["rehashes"] >= 2 and grown[1]["rehashes"] >= 2
    assert fixed[0]["rehashes"] == 0 and fixed[0]["table_slots"] == cap
    # the entries never move: with one factor per launch (a threshold, or an
    # index that may still grow) the sweeps scan the same entries whatever
    # the index size; at threshold 0 the full-size index fuses factor pairs
    if thr > 0.0:
        for i in (0, 1):
            assert grown[i]["fwd_slots_scanned"] == fixed[i]["fwd_slots_scanned"] > 0
            assert grown[i]["rev_slots_scanned"] == fixed[i]["rev_slots_scanned"]
    assert grown[0]["n_live"] == fixed[0]["n_live"]
    assert grown[1]["live_counts"] == fixed[1]["live_counts"]
    for x, y in zip(grown[2][0], fixed[2][0]):
        assert x.tobytes() == y.tobytes()
    for i in (3, 4, 5):
        assert grown[i].tobytes() == fixed[i].tobytes()
    tol = TOL[prec]
    orc.set_nearcut_window(1e-5)
    d_ref, a_ref, nc, _ = orc.apply_ucc(nq, [hf], [1.0], exc, theta[0], thr)
    E_ref, g_ref, _ = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0
    compare_states(grown[2][0][0], grown[2][0][1], d_ref, a_ref, tol["amp"])
    assert abs(grown[3][0] - E_ref) <= tol["E"] and abs(grown[4][0] - E_ref) <= tol["E"]
    assert np.max(np.abs(grown[5][0] - g_ref)) <= tol["g"]


def test_table_growth_batch(swc, orc, monkeypatch):
    """Batch members share one table size: a growth triggered by any member
    rehashes all of them; each still matches its own oracle run."""
    say("[case] growth batch3 q16_thr fp32")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 171, batch=3)
    thr = 1e-4
    cap = capacity_for(8, 4)
    grown = _run_with_table_min(swc, monkeypatch, 64, 16, 4, cap, 1, 3, exc, theta, thr, h1, h2)
    fixed = _run_with_table_min(swc, monkeypatch, cap, 16, 4, cap, 1, 3, exc, theta, thr, h1, h2)
    assert grown[0]["rehashes"] >= 2
    for i in (3, 4, 5):
        assert grown[i].tobytes() == fixed[i].tobytes()
    orc.set_nearcut_window(1e-5)
    for b in range(3):
        E_ref, g_ref, nc = orc.energy_and_grad(16, [hf], [1.0], exc, theta[b], thr, h1, h2)
        assert nc == 0
        assert abs(grown[4][b] - E_ref) <= TOL[1]["E"]
        assert np.max(np.abs(grown[5][b] - g_ref)) <= TOL[1]["g"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_launch_grid_bitwise(swc, monkeypatch, prec):
    """The number of blocks of the sweep launches (resident-sized by default;
    SWC_GRID caps them at one block per arena of entries here, so every lane
    takes many passes) changes no bit
    of the state, energy or gradient: every sum is an exact fixed-point sum
    and every pair has one owner, wherever it sits in the launch."""
    say(f"[case] grid caps q16_thr prec={prec}")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 105)
    thr = 1e-4
    cap = capacity_for(8, 4)
    out = []
    for g in (None, "16", "3"):
        monkeypatch.delenv("SWC_GRID", raising=False)
        monkeypatch.setenv("SWC_TABLE_MIN", "64")
        if g:
            monkeypatch.setenv("SWC_GRID", g)
        s = swc.Solver(16, 4, 4, cap, prec=prec, batch=1, max_factors=exc.shape[0])
        s.build_state()
        s.apply_ucc(theta, exc, thr)
        d, a = s.get_state(0)
        st = s.stats()
        E, gr = s.energy_and_grad(theta, exc, thr, h1, h2)
        out.append((d.tobytes(), a.tobytes(), st["det_updates"], E.cpu().numpy().tobytes(),
                    gr.cpu().numpy().tobytes()))
        s.close()
    assert out[0] == out[1] == out[2]


SCAN_CASES = [
    ("q16", 8, 4, 0.1, 104, None, 0.0, 0),
    ("q16_thr_ckpt", 8, 4, 0.1, 105, None, 1e-4, 16),
    ("q20_pre_thr", 10, 5, 0.05, 107, 300, 1e-5, 0),
    ("q20_pre_thr_ckpt", 10, 5, 0.05, 107, 300, 1e-5, 64),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", SCAN_CASES, ids=[c[0] for c in SCAN_CASES])
def test_reverse_sweep_scans_shrink(swc, orc, monkeypatch, case, prec):
    """Undoing factor k scans only the entries that existed after forward
    step k (those created later lie past the arena counts of the next forward
    launch): the reverse sweep scans fewer entries than M times the largest
    state, gradient calls repeat bit for bit (the log records and checkpoints
    are found by determinant), the state after the call is |Psi_0>, and the
    results match the oracle."""
    name, n_orb, n_occ, sigma, seed, nf, thr, ck = case
    say(f"[case] reverse scans {name} prec={prec} thr={thr} ckpt={ck}")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    nq = 2 * n_orb
    cap = capacity_for(n_orb, n_occ)
    M = exc.shape[0]
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=prec, batch=1, max_factors=M)
    if ck:
        s.set_checkpoints(ck, cap)
    s.track_live(True)
    s.build_state()
    reps = []
    for _ in range(2):
        E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
        reps.append((E.cpu().numpy().tobytes(), g.cpu().numpy().tobytes()))
    st = s.stats()
    assert reps[0] == reps[1]
    d, a = s.get_state(0)
    assert d.tolist() == [hf] and a.tolist() == [1.0]
    s.apply_ucc(theta, exc, thr)  # the entries a forward sweep ends with, and its visits
    st_f = s.stats()
    n_end = st_f["slots_used"]
    s.close()
    say(f"  forward entries scanned {st['fwd_slots_scanned']}, reverse {st['rev_slots_scanned']}, "
        f"entries at the end {n_end}, log records {st['log_records']}")
    # a two-factor launch scans each entry once for two steps of visits
    assert st_f["fwd_slots_scanned"] == st["fwd_slots_scanned"]
    assert 2 * st["fwd_slots_scanned"] >= st_f["det_updates"] > 0
    assert st["fwd_slots_scanned"] <= st["rev_slots_scanned"] < M * n_end
    assert st["shrinks"] == 0
    orc.set_nearcut_window(1e-5)
    E_ref, g_ref, nc = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0
    E = np.frombuffer(reps[0][0], dtype=np.float64)[0]
    g = np.frombuffer(reps[0][1], dtype=np.float64)
    assert abs(E - E_ref) <= TOL[prec]["E"]
    assert np.max(np.abs(g - g_ref)) <= TOL[prec]["g"]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_tombstone_compaction_sequential_calls(swc, orc, monkeypatch, prec):
    """Three apply calls on one state with no reset in between: U(theta), its
    inverse (factors reversed, angles negated: nearly every determinant is
    truncated away and left as a tombstone), then U(theta) again.  The third
    sweep starts with a compacting rehash that drops the tombstones; the state
    matches the oracle applied three times in a row."""
    say(f"[case] compaction q20 prefix prec={prec}")
    h1, h2, exc, theta, hf = small_problem(10, 5, 0.1, 197, 200)
    thr = 3e-4
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    s = swc.Solver(20, 5, 5, 1 << 17, prec=prec, batch=1, max_factors=exc.shape[0])
    s.build_state()
    orc.set_nearcut_window(1e-5)
    inv_exc = exc[::-1].copy()
    inv_theta = -theta[:, ::-1].copy()
    d_ref, a_ref = [hf], [1.0]
    comp = []
    for call, (e, t) in enumerate([(exc, theta), (inv_exc, inv_theta), (exc, theta)]):
        s.apply_ucc(t, e, thr)
        st = s.stats()
        comp.append(st["compactions"])
        d_ref, a_ref, nc, _ = orc.apply_ucc(20, d_ref, a_ref, e, t[0], thr)
        assert nc == 0
        d, a = s.get_state(0)
        err = compare_states(d, a, d_ref, a_ref, TOL[prec]["amp"] * 2)
        say(f"  call {call}: N={len(d)} used={st['slots_used']} pruned={st['pruned']} rehashes={st['rehashes']} "
            f"compactions={st['compactions']} table={st['table_slots']} err={err:.3e}")
    assert comp == [0, 0, 1]
    E = s.energy(h1, h2).cpu().numpy()[0]
    assert abs(E - orc.energy(10, h1, h2, d_ref, a_ref)) <= TOL[prec]["E"] * 2
    s.close()


FUSE_CASES = [
    ("q16", 8, 4, 0.1, 104, None),
    ("q20_pre", 10, 5, 0.05, 106, 161),
    ("q12_dup", 6, 3, 0.2, 102, None),
]


@pytest.mark.parametrize("mode", ["graph", "direct"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", FUSE_CASES, ids=[c[0] for c in FUSE_CASES])
def test_two_factor_launches_bitwise(swc, orc, monkeypatch, case, prec, mode):
    """At threshold 0 two neighbouring factors share a launch (forward and
    adjoint); the results, state and counters are bit-identical to one
    factor per launch.  q12_dup repeats factors so that some neighbours have
    equal masks (never fused), q20_pre has an odd factor count."""
    name, n_orb, n_occ, sigma, seed, nf = case
    say(f"[case] fused {name} prec={prec} mode={mode}")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    if name.endswith("_dup"):
        idx = np.repeat(np.arange(exc.shape[0]), 2)[: exc.shape[0] + 7]
        exc = exc[idx].copy()
        theta = theta[:, idx].copy() * 0.5
    nq = 2 * n_orb
    out = {}
    for fuse in ("0", "1"):
        for k in ("SWC_GRAPH", "SWC_FUSE"):
            monkeypatch.delenv(k, raising=False)
        monkeypatch.setenv("SWC_FUSE", fuse)
        if mode == "direct":
            monkeypatch.setenv("SWC_GRAPH", "0")
        s = swc.Solver(nq, n_occ, n_occ, capacity_for(n_orb, n_occ), prec=prec, batch=1, max_factors=exc.shape[0])
        s.build_state()
        reps = []
        for rep in range(2):
            E, g = s.energy_and_grad(theta, exc, 0.0, h1, h2)
            st_g = s.stats()
            s.apply_ucc(theta, exc, 0.0)
            st = s.stats()
            d, a = s.get_state(0)
            s.build_state()
            reps.append((E.cpu().numpy().tobytes(), g.cpu().numpy().tobytes(), d.tobytes(), a.tobytes(),
                         st["det_updates"], st["pair_updates"], st["inserts"], st["partner_hits"], st["n_live"]))
        assert reps[0] == reps[1]
        out[fuse] = (reps[0], st["rotate_launches"], st_g["reverse_launches"])
        s.close()
    say(f"  launches fwd {out['0'][1]} -> {out['1'][1]}, rev {out['0'][2]} -> {out['1'][2]}")
    assert out["0"][0] == out["1"][0]
    M = exc.shape[0]
    assert out["0"][1] == M and out["0"][2] == M
    assert out["1"][1] < M and out["1"][2] < M
    E_ref, g_ref, _ = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], 0.0, h1, h2)
    E = np.frombuffer(out["1"][0][0], dtype=np.float64)[0]
    g = np.frombuffer(out["1"][0][1], dtype=np.float64)
    assert abs(E - E_ref) <= TOL[prec]["E"]
    assert np.max(np.abs(g - g_ref)) <= TOL[prec]["g"]


ENT_CASES = [
    ("q16", 8, 4, 0.1, 104, None, 0.0),
    ("q12_thr", 6, 3, 0.25, 103, None, 2e-3),
    ("q20_pre_thr", 10, 5, 0.05, 107, 300, 1e-5),
]


@pytest.mark.parametrize("mode", ["graph", "persistent"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", ENT_CASES, ids=[c[0] for c in ENT_CASES])
def test_entropy_trajectory_vs_oracle(swc, orc, monkeypatch, case, prec, mode):
    """Entropy (Eq. 6) of the state before and after every factor, tracked by
    the forward sweep (table growth on, batch of 2), against the oracle;
    tracking leaves every result unchanged."""
    name, n_orb, n_occ, sigma, seed, nf, thr = case
    say(f"[case] entropy {name} prec={prec} mode={mode}")
    for k in ("SWC_SWEEP", "SWC_TABLE_MIN"):
        monkeypatch.delenv(k, raising=False)
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    if mode == "persistent":
        monkeypatch.setenv("SWC_SWEEP", "persistent")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf, batch=2)
    nq, M = 2 * n_orb, exc.shape[0]
    s = swc.Solver(nq, n_occ, n_occ, capacity_for(n_orb, n_occ), prec=prec, batch=2, max_factors=M)
    s.build_state()
    E0, g0 = s.energy_and_grad(theta, exc, thr, h1, h2)
    with pytest.raises(swc.SwcError) as e:
        s.entropy(0)
    assert e.value.code == swc.ESTATE
    s.track_entropy(True)
    E1, g1 = s.energy_and_grad(theta, exc, thr, h1, h2)
    assert E1.cpu().numpy().tobytes() == E0.cpu().numpy().tobytes()
    assert g1.cpu().numpy().tobytes() == g0.cpu().numpy().tobytes()
    S_grad = [s.entropy(b) for b in range(2)]
    s.apply_ucc(theta, exc, thr)
    tol = 1e-11 if prec == 0 else 2e-5
    orc.set_nearcut_window(1e-5)
    for b in range(2):
        S = s.entropy(b)
        assert S.shape == (M + 1,)
        assert S.tobytes() == S_grad[b].tobytes()
        S_ref = orc.entropy_trajectory(nq, [hf], [1.0], exc, theta[b], thr)
        err = np.max(np.abs(S - S_ref))
        say(f"  b={b} S_M={S[-1]:.6f} max|dS|={err:.3e}")
        assert err <= tol
    s.close()


TOPK_CASES = [
    # (name, n_orb, n_occ, sigma, seed, n_factors, threshold, n_max, n_cut)
    ("q12_t0", 6, 3, 0.3, 201, None, 0.0, 150, 100),
    ("q16_thr", 8, 4, 0.1, 201, None, 1e-4, 1200, 800),
    ("q16_t0", 8, 4, 0.15, 201, None, 0.0, 2000, 1500),
    ("q20_pre_thr", 10, 5, 0.05, 201, 300, 1e-5, 3000, 2000),
    ("q20_pre_t0", 10, 5, 0.08, 201, 200, 0.0, 2500, 1200),
]


@pytest.mark.parametrize("mode", ["graph", "grow_batch", "persistent"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", TOPK_CASES, ids=[c[0] for c in TOPK_CASES])
def test_topk_truncation_vs_oracle(swc, orc, monkeypatch, case, prec, mode):
    """N_MAX / N_CUT truncation after every factor (radix selection on the
    device) against the oracle: surviving set bit-exact, amplitudes, E, the
    frozen-decision gradient and det-updates."""
    name, n_orb, n_occ, sigma, seed, nf, thr, n_max, n_cut = case
    say(f"[case] topk {name} prec={prec} mode={mode}")
    for k in ("SWC_SWEEP", "SWC_TABLE_MIN"):
        monkeypatch.delenv(k, raising=False)
    B = 2 if mode == "grow_batch" else 1
    if mode == "grow_batch":
        monkeypatch.setenv("SWC_TABLE_MIN", "64")
    elif mode == "persistent":
        monkeypatch.setenv("SWC_SWEEP", "persistent")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf, batch=B)
    if B == 2:
        theta[1] = theta[0]  # member 1 repeats member 0 under a second table layout of the batch
    nq = 2 * n_orb
    tol = TOL[prec]
    orc.set_nearcut_window(1e-5)
    orc.set_topk(n_max, n_cut)
    try:
        d_ref, a_ref, nc, du_ref = orc.apply_ucc(nq, [hf], [1.0], exc, theta[0], thr)
        E_ref, g_ref, _ = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
        n_ref = orc.live_trajectory(nq, [hf], [1.0], exc, theta[0], thr)
    finally:
        orc.set_topk(0, 0)
    assert nc == 0
    cap = capacity_for(n_orb, n_occ)
    # determinants flicker across the N_CUT boundary: many tombstones are
    # revived, each saved in the truncation log
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=prec, batch=B, max_factors=exc.shape[0], log_capacity=64 * cap)
    s.set_topk(n_max, n_cut)
    s.track_live(True)
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    st = s.stats()
    assert st["det_updates"] == B * du_ref
    for b in range(B):
        assert np.array_equal(s.live_counts(b), n_ref)
        d, a = s.get_state(b)
        err = compare_states(d, a, d_ref, a_ref, tol["amp"])
    E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    E, g = E.cpu().numpy(), g.cpu().numpy()
    for b in range(B):
        dg = np.max(np.abs(g[b] - g_ref))
        say(f"  b={b} N={len(d_ref)} amp_err={err:.3e} dE={abs(E[b] - E_ref):.3e} max|dg|={dg:.3e}")
        assert abs(E[b] - E_ref) <= tol["E"]
        assert dg <= tol["g"]
    s.set_topk(0, 0)
    s.build_state()
    s.apply_ucc(theta, exc, thr)
    assert s.stats()["n_live"] > len(d_ref)  # the truncation was active
    with pytest.raises(swc.SwcError):
        s.set_topk(10, 11)
    s.close()


# ---------------------------------------------------------------- kernel builds used at full size
BUILD_CASES = [
    # (name, n_orb, n_occ, sigma, seed, n_factors, threshold, capacity, table_min, grid cap, builds expected)
    # one block per arena: the one-factor builds take many passes per lane
    ("fwd_passes_q16_thr", 8, 4, 0.1, 105, None, 1e-4, 1 << 16, 1 << 16, "64", ("BUILD_FWD", "BUILD_REV")),
    # threshold 0, one block per arena over an index of 2^16 slots: the
    # two-factor kernels that preload one index slot per probe
    ("fused_ph1_q16", 8, 4, 0.1, 104, None, 0.0, 1 << 16, 1 << 16, "64", ("BUILD_FWD2", "BUILD_REV2")),
    ("fused_ph1_q20_pre", 10, 5, 0.05, 106, 160, 0.0, 1 << 17, 1 << 17, "64", ("BUILD_FWD2", "BUILD_REV2")),
]


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", BUILD_CASES, ids=[c[0] for c in BUILD_CASES])
def test_full_size_builds_vs_oracle(swc, orc, monkeypatch, case, prec):
    """The kernel builds and launch shapes the large workloads run (one-factor
    steps whose lanes take many passes; the two-factor kernels that preload
    one index slot per probe) forced on small instances and checked against
    the oracle: the state, the live count of every step, E and the gradient.
    The builds that ran are read back from the statistics."""
    name, n_orb, n_occ, sigma, seed, nf, thr, cap, tmin, grid, builds = case
    say(f"[case] builds {name} prec={prec}")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    nq = 2 * n_orb
    monkeypatch.setenv("SWC_TABLE_MIN", str(tmin))
    if grid:
        monkeypatch.setenv("SWC_GRID", grid)
    else:
        monkeypatch.delenv("SWC_GRID", raising=False)
    s = swc.Solver(nq, n_occ, n_occ, cap, prec=prec, batch=1, max_factors=exc.shape[0])
    s.track_live(True)
    s.build_state()
    tol = TOL[prec]
    orc.set_nearcut_window(1e-5)
    d_ref, a_ref, nc, du_ref = orc.apply_ucc(nq, [hf], [1.0], exc, theta[0], thr)
    E_ref, g_ref, _ = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0
    n_ref = orc.live_trajectory(nq, [hf], [1.0], exc, theta[0], thr)
    E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    st = s.stats()
    got = st["kernel_builds"]
    say(f"  builds {got:#x}")
    for bname in builds:
        assert got & getattr(swc, bname), (bname, hex(got))
    assert abs(E.cpu().numpy()[0] - E_ref) <= tol["E"]
    assert np.max(np.abs(g.cpu().numpy()[0] - g_ref)) <= tol["g"]
    assert np.array_equal(s.live_counts(0), n_ref)
    s.apply_ucc(theta, exc, thr)
    assert s.stats()["det_updates"] == du_ref
    d, a = s.get_state(0)
    compare_states(d, a, d_ref, a_ref, tol["amp"])
    s.close()
