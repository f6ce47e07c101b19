"""Outer variational loop and molecular-integral input.

The paper optimises the UCC parameters with SciPy's SLSQP (Methods section),
starting from MP2 amplitudes, on integrals from PySCF.  This module supplies
the same loop around the library: the energy and the adjoint gradient of one
`energy_and_grad` call feed `scipy.optimize.minimize` (SLSQP, L-BFGS-B, BFGS,
...), and integrals can be read from (or written to) an FCIDUMP text file,
the plain exchange format quantum chemistry codes write.

    python -m paper_2301_05726_amd.vqe --fcidump FILE [--threshold T]
           [--method L-BFGS-B] [--maxiter N] [--prec fp32|fp64] [--capacity-log2 C]

FCIDUMP layout: a namelist header (&FCI NORB=.., NELEC=.., MS2=.., ... /)
then one integral per line, `value i j k l` with 1-based orbital indices:
(ij|kl) for i, j, k, l > 0 (chemist notation, 8-fold symmetric), h_ij for
k = l = 0, and the constant (core) energy for i = j = k = l = 0.
"""
from __future__ import annotations

import argparse
import re
import sys
import time

import numpy as np


def read_fcidump(path: str):
    """Returns (n_orb, n_elec, ms2, h1[n,n], h2[n,n,n,n], e_core); every
    symmetry partner of each listed integral is filled in."""
    text = open(path).read()
    end = re.search(r"(&END|/)", text)
    if not text.lstrip().upper().startswith("&FCI") or end is None:
        raise ValueError("not an FCIDUMP file: missing the &FCI ... / header")
    header, body = text[: end.start()], text[end.end():]

    def field(name, default=None):
        m = re.search(name + r"\s*=\s*(-?\d+)", header, re.IGNORECASE)
        if m is None:
            if default is None:
                raise ValueError(f"FCIDUMP header lacks {name}")
            return default
        return int(m.group(1))

    n = field("NORB")
    nelec = field("NELEC")
    ms2 = field("MS2", 0)
    h1 = np.zeros((n, n))
    h2 = np.zeros((n, n, n, n))
    e_core = 0.0
    for line in body.splitlines():
        parts = line.replace(",", " ").split()
        if len(parts) != 5:
            continue
        v = float(parts[0].replace("D", "E").replace("d", "e"))
        i, j, k, l = (int(x) for x in parts[1:])
        if i == j == k == l == 0:
            e_core += v
        elif k == 0 and l == 0:
            h1[i - 1, j - 1] = h1[j - 1, i - 1] = v
        else:
            p, q, r, s = i - 1, j - 1, k - 1, l - 1
            for a, b, c, d in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                               (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
                h2[a, b, c, d] = v
    return n, nelec, ms2, h1, h2, e_core


def write_fcidump(path: str, h1, h2, n_elec: int, ms2: int = 0, e_core: float = 0.0, tol: float = 0.0):
    """Write the unique integrals (i>=j, k>=l, ij>=kl) with |value| > tol."""
    n = h1.shape[0]
    with open(path, "w") as f:
        f.write(f"&FCI NORB={n},NELEC={n_elec},MS2={ms2},\n ORBSYM={','.join(['1'] * n)},\n ISYM=1,\n&END\n")
        for i in range(n):
            for j in range(i + 1):
                for k in range(n):
                    for l in range(k + 1):
                        if i * (i + 1) // 2 + j < k * (k + 1) // 2 + l:
                            continue
                        v = h2[i, j, k, l]
                        if abs(v) > tol:
                            f.write(f"{float(v)!r} {i + 1} {j + 1} {k + 1} {l + 1}\n")
        for i in range(n):
            for j in range(i + 1):
                if abs(h1[i, j]) > tol:
                    f.write(f"{float(h1[i, j])!r} {i + 1} {j + 1} 0 0\n")
        f.write(f"{float(e_core)!r} 0 0 0 0\n")


def minimize(solver, exc, h1, h2, theta0, threshold=0.0, method="L-BFGS-B", maxiter=200, tol=1e-10,
             callback=None):
    """Minimise E(theta) of batch member 0 with scipy.optimize.minimize,
    energy and adjoint gradient from one library call per evaluation.
    Returns (scipy result, history of (evaluation, E))."""
    import scipy.optimize
    import torch

    h1d = torch.as_tensor(np.asarray(h1, np.float64), device=solver.device)
    h2d = torch.as_tensor(np.asarray(h2, np.float64), device=solver.device)
    history = []

    def fun(x):
        E, g = solver.energy_and_grad(torch.as_tensor(x, dtype=torch.float64, device=solver.device)[None, :],
                                      exc, threshold, h1d, h2d)
        e = float(E[0].item())
        history.append((len(history), e))
        if callback:
            callback(len(history), e)
        return e, g[0].cpu().numpy()

    res = scipy.optimize.minimize(fun, np.asarray(theta0, np.float64), jac=True, method=method, tol=tol,
                                  options={"maxiter": maxiter})
    return res, history


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description="UCC energy minimisation on a sparse wavefunction (one GPU)")
    ap.add_argument("--fcidump", required=True)
    ap.add_argument("--threshold", type=float, default=0.0)
    ap.add_argument("--method", default="L-BFGS-B")
    ap.add_argument("--maxiter", type=int, default=200)
    ap.add_argument("--prec", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--capacity-log2", type=int, default=20)
    args = ap.parse_args(argv)

    from paper_2301_05726_amd import swc, synth
    n, nelec, ms2, h1, h2, e_core = read_fcidump(args.fcidump)
    na, nb = (nelec + ms2) // 2, (nelec - ms2) // 2
    if na != nb:
        raise SystemExit("open-shell references are not generated here (closed-shell UCCSD only)")
    exc = synth.ordered_excitations(h1, h2, na)
    s = swc.Solver(2 * n, na, nb, 1 << args.capacity_log2, prec=swc.FP32 if args.prec == "fp32" else swc.FP64,
                   batch=1, max_factors=exc.shape[0])
    s.build_state()
    t0 = time.perf_counter()
    res, hist = minimize(s, exc, h1, h2, np.zeros(exc.shape[0]), args.threshold, args.method, args.maxiter,
                         callback=lambda i, e: print(f"eval {i:4d}  E = {e + e_core:.12f}", flush=True))
    print(f"{args.method}: E = {res.fun + e_core:.12f} Ha after {len(hist)} evaluations "
          f"({time.perf_counter() - t0:.2f} s), {exc.shape[0]} parameters, success={res.success}", flush=True)
    s.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
