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


def ratio_err(r, r_ref):
    r = np.asarray(r)
    r_ref = np.asarray(r_ref)
    return np.abs(r - r_ref) / np.maximum(np.abs(r_ref), 1.0)


def det_ratio_bound(phi, occ_before, occ_after, inv_before, k, elec):
    """First-order relative error bound of r = det(I + u^T C) per unit relative error
    of the stored inverse columns: kappa_R * cond_1(A), where
    kappa_R = sum |R^-T| o (I + |u^T| |C|) is the condition number of det R with
    respect to the products u^T C (C = A^-1[:, I] from the oracle)."""
    out = np.empty(len(k))
    for w in range(len(k)):
        kw = int(k[w])
        rows = np.asarray(elec[w, :kw])
        a = phi[occ_before[w]]
        u = (phi[occ_after[w]] - a)[rows]
        c = inv_before[w][:, rows]
        r = np.eye(kw) + u @ c
        absr = np.eye(kw) + np.abs(u) @ np.abs(c)
        try:
            kap = float(np.sum(np.abs(np.linalg.inv(r).T) * absr))
        except np.linalg.LinAlgError:
            kap = np.inf
        cond = np.linalg.norm(a, 1) * np.linalg.norm(inv_before[w], 1)
        out[w] = kap * cond
    return out


def pf_ratio_bound(x, col, r):
    """Same for the Pfaffian hop r = 1 + x . col: (1 + sum |x||col|) / |r| * cond."""
    return (1.0 + np.sum(np.abs(x) * np.abs(col), axis=-1)) / np.maximum(np.abs(r), 1e-300)


def fp64_tol(cond, steps):
    """1e-10 relative, widened to cond * steps * eps for ill-conditioned steps (cond > 1e6)."""
    return np.maximum(1e-10, 64.0 * np.asarray(cond) * max(steps, 1) * EPS64)


def run_chain(walkers, chain, draws, u01s, check_every=1, check_inverse=True, tol_ratio=None, tol_inv=None,
              stats=None, check_walkers=None, bound_fn=None):
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
        if bound_fn is not None:
            chain.inv_before, chain.occ_before = chain.inv.copy(), chain.book.occ.copy()
        r_orc = chain.propose(k, elec, slot)
        mask = orc.metropolis(r_orc, u01)
        # The ratio is det(I + u^T C): its rounding error is relative to the identity
        # term, so the error is measured on the scale max(1, |r|) (pure relative
        # error for |r| >= 1, absolute for the strongly suppressed moves |r| < 1).
        er = ratio_err(r_gpu[cw], r_orc[cw])
        worst_r = max(worst_r, float(er.max()))
        if tol_ratio is not None:
            tol = tol_ratio(t) if callable(tol_ratio) else tol_ratio
            if np.any(er > tol) and bound_fn is not None:
                # widen to the computed first-order bound for ill-conditioned steps (counted)
                tol = np.maximum(tol, 8 * EPS64 * bound_fn(t, chain, k, elec, slot, cw))
                if stats is not None:
                    stats.append(("widened", t, int(np.sum(er > tol_ratio))))
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


def det_bound_fn(phi):
    """bound_fn for run_chain on determinant chains."""
    def fn(t, chain, k, elec, slot, cw):
        after = chain.book.proposed(k, elec, slot)
        return det_ratio_bound(phi, chain.occ_before[cw], after[cw], chain.inv_before[cw], k[cw], elec[cw])
    return fn
