"""Shared helpers of the GPU parity tests (the oracle decides, the GPU follows)."""
from __future__ import annotations

import sys

import numpy as np

EPS64 = np.finfo(np.float64).eps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(a, b, axis=None):
    a = np.asarray(a)
    b = np.asarray(b)
    if axis is None:
        return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
    return np.linalg.norm(a - b, axis=axis) / np.maximum(np.linalg.norm(b, axis=axis), 1e-300)


def fp64_tol(cond, steps):
    """1e-10 relative, widened to cond * steps * eps for ill-conditioned steps (cond > 1e6)."""
    return np.maximum(1e-10, 64.0 * np.asarray(cond) * max(steps, 1) * EPS64)


def run_chain(walkers, chain, draws, u01s, check_every=1, check_inverse=True, tol_ratio=None, tol_inv=None,
              stats=None, check_walkers=None):
    """Drive GPU walkers and the oracle chain through the same proposals.

    The oracle's Metropolis decision (from its own ratios) is fed to the GPU as
    the accept mask so both follow one trajectory.  Returns max errors.
    """
    import oracle as orc
    worst_r, worst_m = 0.0, 0.0
    cw = np.arange(walkers.W) if check_walkers is None else np.asarray(check_walkers)
    for t, ((k, elec, slot), u01) in enumerate(zip(draws, u01s)):
        walkers.set_draws(k, elec, slot)
        r_gpu = walkers.propose().cpu().numpy()
        r_orc = chain.propose(k, elec, slot)
        mask = orc.metropolis(r_orc, u01)
        er = rel_err(r_gpu[cw], r_orc[cw])
        worst_r = max(worst_r, float(er.max()))
        if tol_ratio is not None:
            tol = tol_ratio(t) if callable(tol_ratio) else tol_ratio
            assert np.all(er <= tol), f"step {t}: ratio error {er.max():.3e} > {np.min(tol):.1e}"
        walkers.decide(mask=mask)
        walkers.apply()
        chain.accept(k, elec, slot, mask)
        if check_inverse and (t + 1) % check_every == 0:
            inv = walkers.inverse().cpu().numpy()
            em = rel_err(inv[cw], chain.inv[cw], axis=(1, 2))
            worst_m = max(worst_m, float(em.max()))
            if tol_inv is not None:
                tol = tol_inv(t) if callable(tol_inv) else tol_inv
                assert np.all(em <= tol), f"step {t}: inverse error {em.max():.3e}"
        if stats is not None:
            stats.append((t, float(er.max()), int(mask.sum())))
    # occupancy bookkeeping agrees exactly
    np.testing.assert_array_equal(walkers.occ.cpu().numpy(), chain.book.occ)
    np.testing.assert_array_equal(walkers.empty.cpu().numpy(), chain.book.empty)
    # log|det| / phase tracked through the ratios agree with the recomputation
    la = walkers.st.logabs.cpu().numpy()
    ph = walkers.st.phase.cpu().numpy()
    return worst_r, worst_m, la, ph
