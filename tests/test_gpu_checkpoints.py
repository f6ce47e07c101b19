"""Checkpoints of the gradient sweep, through the C ABI: snapshots of the
forward state written back during the adjoint sweep must leave E unchanged,
keep the gradient within the oracle tolerances, work in every sweep mode and
with table growth, and report a too-small snapshot buffer."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import TOL, say, small_problem

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def swc():
    from paper_2301_05726_amd import swc as s
    s.lib()
    assert torch.cuda.is_available()
    return s


CASES = [
    # (name, n_orb, n_occ, sigma, seed, n_factors, threshold)
    ("q16_thr", 8, 4, 0.1, 105, None, 1e-4),
    ("q20_pre", 10, 5, 0.05, 106, 160, 0.0),
    ("q20_pre_thr", 10, 5, 0.05, 107, 300, 1e-5),
]


@pytest.mark.parametrize("mode", ["graph", "direct", "persistent"])
@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_checkpointed_gradient(swc, orc, monkeypatch, case, prec, mode):
    name, n_orb, n_occ, sigma, seed, nf, thr = case
    say(f"[case] ckpt {name} prec={prec} mode={mode}")
    for k in ("SWC_GRAPH", "SWC_SWEEP", "SWC_TABLE_MIN"):
        monkeypatch.delenv(k, raising=False)
    if mode == "direct":
        monkeypatch.setenv("SWC_GRAPH", "0")
    elif mode == "persistent":
        monkeypatch.setenv("SWC_SWEEP", "persistent")
    monkeypatch.setenv("SWC_TABLE_MIN", "64")
    h1, h2, exc, theta, hf = small_problem(n_orb, n_occ, sigma, seed, nf)
    nq, M = 2 * n_orb, exc.shape[0]
    orc.set_nearcut_window(1e-5)
    E_ref, g_ref, nc = orc.energy_and_grad(nq, [hf], [1.0], exc, theta[0], thr, h1, h2)
    assert nc == 0
    s = swc.Solver(nq, n_occ, n_occ, 1 << 17, prec=prec, batch=1, max_factors=M)
    s.build_state()
    E0, g0 = s.energy_and_grad(theta, exc, thr, h1, h2)
    tol = TOL[prec]
    for interval in (1, 7, 64):
        s.set_checkpoints(interval)
        E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
        st = s.stats()
        assert st["checkpoints"] == (M - 1) // interval
        E, g = E.cpu().numpy()[0], g.cpu().numpy()[0]
        dg = np.max(np.abs(g - g_ref))
        say(f"  interval={interval} snapshots={st['checkpoints']} dE={abs(E - E_ref):.3e} max|dg|={dg:.3e} "
            f"(no ckpt {np.max(np.abs(g0.cpu().numpy()[0] - g_ref)):.3e})")
        assert E == E0.cpu().numpy()[0]  # the forward sweep is unchanged
        assert dg <= tol["g"]
    s.set_checkpoints(0)
    E, g = s.energy_and_grad(theta, exc, thr, h1, h2)
    assert s.stats()["checkpoints"] == 0
    assert g.cpu().numpy().tobytes() == g0.cpu().numpy().tobytes()
    s.close()


def test_checkpoints_long_fp32_circuit(swc):
    """Full 20-qubit workload (875 factors) in FP32: with a snapshot every 64
    steps the gradient stays within the FP32 tolerance of the stored oracle
    values, as without."""
    from paper_2301_05726_amd import synth
    ref = json.load(open(os.path.join(HERE, "golden", "q20_oracle.json")))
    wl = synth.WORKLOADS["q20"]
    p = synth.make_problem(wl, batch=1)
    s = swc.Solver(wl.n_qubits, wl.n_occ, wl.n_occ, wl.capacity, prec=1, batch=1, max_factors=p.M)
    s.build_state()
    g_ref = np.array(ref["grad"])
    _, g0 = s.energy_and_grad(p.theta, p.exc, wl.threshold, p.h1, p.h2)
    s.set_checkpoints(64)
    _, g1 = s.energy_and_grad(p.theta, p.exc, wl.threshold, p.h1, p.h2)
    e0 = np.max(np.abs(g0.cpu().numpy()[0] - g_ref))
    e1 = np.max(np.abs(g1.cpu().numpy()[0] - g_ref))
    say(f"[case] q20 fp32 ckpt64: max|dg| without {e0:.3e}, with {e1:.3e}, snapshots {s.stats()['checkpoints']}")
    assert e1 <= TOL[1]["g"] and e0 <= TOL[1]["g"]
    s.close()


def test_checkpoint_buffer_too_small(swc):
    say("[case] ckpt too small")
    h1, h2, exc, theta, hf = small_problem(8, 4, 0.1, 105)
    s = swc.Solver(16, 4, 4, 16384, prec=1, batch=1, max_factors=exc.shape[0])
    s.build_state()
    s.set_checkpoints(8, max_entries=4)
    with pytest.raises(swc.SwcError) as e:
        s.energy_and_grad(theta, exc, 1e-4, h1, h2)
    assert e.value.code == swc.ECAPACITY
    # the context stays usable: a large enough buffer works again
    s.build_state()
    s.set_checkpoints(8, max_entries=8192)
    E, g = s.energy_and_grad(theta, exc, 1e-4, h1, h2)
    assert np.isfinite(E.cpu().numpy()).all()
    s.close()
