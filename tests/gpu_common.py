"""Shared helpers of the GPU tests (test infrastructure)."""
import sys

import numpy as np

from paper_2301_05726_amd import synth

TOL = {
    # FP64 amplitudes: everything in double
    0: dict(amp=1e-12, E=1e-10, g=1e-8),
    # FP32 amplitudes, FP64 reductions
    1: dict(amp=2e-5, E=1e-6, g=1e-5),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_problem(n_orb, n_occ, sigma, seed, n_factors=None, batch=1):
    h1, h2 = synth.make_hamiltonian(n_orb, seed)
    exc = synth.ordered_excitations(h1, h2, n_occ)
    if n_factors is not None:
        exc = exc[:n_factors].copy()
    theta = np.stack([synth.make_theta(exc.shape[0], sigma, seed + 1 + b) for b in range(batch)])
    return h1, h2, exc, theta, synth.hf_det(n_occ)


def capacity_for(n_orb, n_occ):
    import math
    sector = math.comb(n_orb, n_occ) ** 2
    cap = 64
    while cap < 2 * sector:
        cap *= 2
    return cap


def compare_states(d_gpu, a_gpu, d_ref, a_ref, amp_tol, allow_support_diff=False):
    if not allow_support_diff:
        assert len(d_gpu) == len(d_ref), (len(d_gpu), len(d_ref))
        assert np.array_equal(d_gpu, d_ref)
        err = np.max(np.abs(a_gpu - a_ref)) if len(a_ref) else 0.0
        assert err <= amp_tol, err
        return err
    common, ig, ir = np.intersect1d(d_gpu, d_ref, return_indices=True)
    return np.max(np.abs(a_gpu[ig] - a_ref[ir]))
