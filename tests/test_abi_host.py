"""Host-side checks of the C ABI library (no GPU needed): exported symbols,
argument validation, and the per-factor bit masks / sign rule used by the
kernels, checked against the oracle's operator-by-operator signs."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_05726_amd import swc, synth

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "swc.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swc_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = swc.lib()
    names = header_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert sorted(names) == sorted(swc.EXPORTS)


def test_stats_binding_matches_header():
    """The ctypes mirror of swc_stats has the header's fields, in order and
    with the same C types (a mismatch would shift every later field)."""
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} swc_stats;", text, flags=re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    decl = re.findall(r"\b(int64_t|double)\s+(\w+)\s*;", body)
    ctype = {"int64_t": ctypes.c_int64, "double": ctypes.c_double}
    assert [(n, ctype[t]) for t, n in decl] == list(swc.Stats._fields_)
    assert ctypes.sizeof(swc.Stats) == 8 * len(decl)


def test_workspace_bytes_validation():
    assert swc.workspace_bytes(20, 1 << 17, swc.FP32, 1, 875) > 0
    assert swc.workspace_bytes(20, 1 << 17, swc.FP64, 1, 875) > swc.workspace_bytes(20, 1 << 17, swc.FP32, 1, 875)
    assert swc.workspace_bytes(1, 1 << 17, swc.FP32, 1, 875) == 0      # n_qubits too small
    assert swc.workspace_bytes(65, 1 << 17, swc.FP32, 1, 875) == 0     # > 64 spin-orbitals
    assert swc.workspace_bytes(20, 1000, swc.FP32, 1, 875) == 0        # not a power of two
    assert swc.workspace_bytes(20, 1 << 17, 7, 1, 875) == 0            # bad precision
    assert swc.workspace_bytes(20, 1 << 17, swc.FP32, 0, 875) == 0     # batch 0


def test_create_rejects_bad_arguments_without_device():
    L = swc.lib()
    ctx = ctypes.c_void_p()
    # workspace missing -> EINVAL before any device work
    r = L.swc_create(ctypes.byref(ctx), 20, 5, 5, 1 << 17, swc.FP32, 1, 875, 0, None, 0, None)
    assert r == swc.EINVAL
    r = L.swc_create(ctypes.byref(ctx), 20, 11, 5, 1 << 17, swc.FP32, 1, 875, 0, None, 0, None)
    assert r == swc.EINVAL
    assert L.swc_strerror(swc.ECAPACITY).decode() == "capacity exceeded"


@pytest.mark.parametrize("bad", [[[0, 2, 2, 6]], [[0, 2, 4, 8]], [[2, 0, 4, 6]], [[0, 2, 6, 4]], [[0, 0, 4, 6]],
                                 [[0, -1, 4, 6]], [[0, -1, 0, -1]], [[9, -1, 2, -1]]])
def test_excitation_validation_matches_oracle(orc, bad):
    assert swc.validate_excitations(8, bad) == swc.EINVAL
    with pytest.raises(orc.OracleError) as e:
        orc.apply_ucc(8, [synth.hf_det(2)], [1.0], np.array(bad, np.int8), [0.1])
    assert e.value.code == orc.EINVAL


def test_excitation_validation_accepts_uccsd():
    h1, h2 = synth.make_hamiltonian(10, 1002)
    ex = synth.ordered_excitations(h1, h2, 5)
    assert swc.validate_excitations(20, ex) == 0


def mask_sign(masks, D):
    occ, vir, sgn = (int(x) for x in masks)
    lower = (D & occ) == occ and (D & vir) == 0
    upper = (D & vir) == vir and (D & occ) == 0
    s = -1 if bin(D & sgn).count("1") & 1 else 1
    return lower, upper, s


def test_mask_sign_rule_exhaustive_10_qubits(orc):
    """Every excitation on 10 spin-orbitals and every determinant: the mask
    applicability test and popcount sign equal the oracle's sequential
    application of the four (two) fermionic operators."""
    nq = 10
    rows = []
    for i in range(nq):
        for a in range(nq):
            if i != a:
                rows.append((i, -1, a, -1))
    for i in range(nq):
        for j in range(i + 1, nq):
            for a in range(nq):
                for b in range(a + 1, nq):
                    if len({i, j, a, b}) == 4:
                        rows.append((i, j, a, b))
    masks = swc.factor_masks(nq, rows)
    rng = np.random.default_rng(0)
    dets = rng.choice(1 << nq, size=96, replace=False)
    for r, m in zip(rows, masks):
        for D in dets.tolist():
            lower, upper, s = mask_sign(m, D)
            so, P = orc.tau(r, D)
            assert (so != 0) == lower, (r, D)
            if lower:
                assert so == s and P == D ^ (int(m[0]) | int(m[1])), (r, D)
            if upper:  # the sign of tau|L> with L the partner of D
                L = D ^ (int(m[0]) | int(m[1]))
                sl, U = orc.tau(r, L)
                assert sl == s and U == D, (r, D)


def test_mask_sign_rule_random_64_qubits(orc):
    rng = np.random.default_rng(1)
    nq = 64
    for _ in range(300):
        idx = rng.choice(nq, size=4, replace=False)
        if rng.random() < 0.3:
            row = (int(idx[0]), -1, int(idx[1]), -1)
        else:
            i, j = sorted(idx[:2].tolist())
            a, b = sorted(idx[2:].tolist())
            row = (i, j, a, b)
        m = swc.factor_masks(nq, [row])[0]
        for _ in range(40):
            D = int(rng.integers(0, 1 << 63, dtype=np.uint64)) | (int(rng.integers(0, 2)) << 63)
            D &= ~(1 << 63) if D == (1 << 64) - 1 else D
            # force applicability half of the time
            if rng.random() < 0.5:
                D = (D | int(m[0])) & ~int(m[1])
            lower, upper, s = mask_sign(m, D)
            so, P = orc.tau(row, D)
            assert (so != 0) == lower
            if lower:
                assert so == s


def test_solver_collected_at_interpreter_exit_is_quiet(tmp_path):
    """A solver still referenced by a script's globals is collected while the
    interpreter finalises, when module globals may already be cleared: its
    destructor makes no device call then and raises nothing."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = tmp_path / "hold.py"
    script.write_text(
        "import sys\n"
        f"sys.path.insert(0, {root!r})\n"
        "from paper_2301_05726_amd import swc\n"
        "class Held(swc.Solver):\n"
        "    def __init__(self):\n"
        "        pass\n"
        "    def close(self):\n"
        "        print('device call at exit', flush=True)\n"
        "held = Held()\n")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "Exception ignored" not in r.stderr, r.stderr
    assert "device call at exit" not in r.stdout
