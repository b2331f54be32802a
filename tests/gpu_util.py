"""Shared helpers of the GPU parity tests (the oracle decides, the GPU follows)."""
from __future__ import annotations

import sys

import numpy as np

EPS64 = float(np.finfo(np.float64).eps)
EPS32 = float(np.finfo(np.float32).eps)


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
    """Relative error |r - r_o| / |r_o| of ratios (a zero oracle ratio compares absolutely)."""
    r = np.asarray(r)
    r_ref = np.asarray(r_ref)
    return np.abs(r - r_ref) / np.where(r_ref == 0, 1.0, np.abs(r_ref))


class RatioTally:
    """Ratio checks of a test: relative error |r - r_o| / |r_o| against a flat tolerance;
    a walker-step above it is held instead to 8 eps growth times its first-order error
    bound (an ill-conditioned or strongly suppressed move), and counted."""

    def __init__(self, name=""):
        self.name, self.checked, self.widened, self.worst = name, 0, 0, 0.0

    def check(self, r, r_o, flat, bound=None, eps=EPS64, growth=1.0, where=""):
        er = np.atleast_1d(ratio_err(r, r_o))
        self.checked += er.size
        self.worst = max(self.worst, float(er.max()) if er.size else 0.0)
        over = er > flat
        if over.any():
            assert bound is not None, f"{where}: ratio error {er.max():.3e} > {flat:.1e}"
            b = np.atleast_1d(bound() if callable(bound) else np.asarray(bound))
            tol = np.where(over, np.maximum(flat, 8.0 * eps * np.asarray(growth) * b), flat)
            bad = er > tol
            assert not bad.any(), (f"{where}: ratio error {er[bad].max():.3e} above its widened bound "
                                   f"{tol[bad].min():.1e}")
            self.widened += int(over.sum())
        return er

    def report(self):
        say(f"  {self.name} ratio checks: {self.checked} walker-steps, {self.widened} above the flat "
            f"tolerance (held to their first-order bound), max rel err {self.worst:.2e}")


def assert_entries_close(got, ref, tol, what=""):
    """Element-by-element comparison: |got - ref| <= tol * max(|ref|, rms(ref)) for every
    entry (relative per entry, with the array's RMS as the floor for entries near zero)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2))) if ref.size else 0.0
    scale = np.maximum(np.abs(ref), rms)
    err = np.abs(got - ref)
    bad = err > tol * scale
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {ref.size} entries off, worst "
                           f"{float(np.max(err / np.where(scale > 0, scale, 1.0))):.3e} > {tol:.1e}")
    return float(np.max(err / np.where(scale > 0, scale, 1.0))) if ref.size else 0.0


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
              stats=None, check_walkers=None, bound_fn=None, eps=EPS64, growth=None):
    """Drive GPU walkers and the oracle chain through the same proposals.

    The oracle's Metropolis decision (from its own ratios) is fed to the GPU as
    the accept mask so both follow one trajectory.  Ratios are checked with a
    RatioTally: relative error against ``tol_ratio``, a walker-step above it held
    to 8 eps growth(t) times the first-order bound from ``bound_fn`` (growth(t) is
    the number of updates the stored inverse has taken since it was last
    recomputed) and counted.  Returns max errors; ``stats`` (a list) receives
    per-step records and the final ("widened_total", n_widened, n_checked).
    """
    import oracle as orc
    tally = RatioTally(type(chain).__name__)
    worst_m = 0.0
    cw = np.arange(walkers.W) if check_walkers is None else np.asarray(check_walkers)
    for t, ((k, elec, slot), u01) in enumerate(zip(draws, u01s)):
        walkers.set_draws(k, elec, slot)
        r_gpu = walkers.propose().cpu().numpy()
        if bound_fn is not None:
            chain.inv_before, chain.occ_before = chain.inv.copy(), chain.book.occ.copy()
        r_orc = chain.propose(k, elec, slot)
        mask = orc.metropolis(r_orc, u01)
        if tol_ratio is not None:
            flat = tol_ratio(t) if callable(tol_ratio) else tol_ratio
            before = tally.widened
            er = tally.check(r_gpu[cw], r_orc[cw], flat,
                             (lambda: bound_fn(t, chain, k, elec, slot, cw)) if bound_fn is not None else None,
                             eps, growth(t) if growth is not None else 1.0, where=f"step {t}")
            if stats is not None and tally.widened > before:
                stats.append(("widened", t, tally.widened - before))
        else:
            er = ratio_err(r_gpu[cw], r_orc[cw])
            tally.worst = max(tally.worst, float(er.max()))
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
    tally.report()
    if stats is not None:
        stats.append(("widened_total", tally.widened, tally.checked))
    # occupancy bookkeeping agrees exactly
    np.testing.assert_array_equal(walkers.occ.cpu().numpy(), chain.book.occ)
    np.testing.assert_array_equal(walkers.empty.cpu().numpy(), chain.book.empty)
    # log|det| / phase tracked through the ratios agree with the recomputation
    la = walkers.st.logabs.cpu().numpy()
    ph = walkers.st.phase.cpu().numpy()
    return tally.worst, worst_m, la, ph


def det_bound_fn(phi):
    """bound_fn for run_chain on determinant chains."""
    def fn(t, chain, k, elec, slot, cw):
        after = chain.book.proposed(k, elec, slot)
        return det_ratio_bound(phi, chain.occ_before[cw], after[cw], chain.inv_before[cw], k[cw], elec[cw])
    return fn


def pf_hop_bound(f, occ_before, occ_after, inv_before, elec):
    """First-order relative error bound of the Pfaffian hop ratio r = 1 + x . col per unit
    relative error of the stored column col = A^-1[:, i]: (1 + sum |x| |col|) / |r|
    times cond_1(A), per walker (x_j = F[s', occ_j] - F[s, occ_j], x_i = 0)."""
    out = np.empty(len(elec))
    for w in range(len(elec)):
        i = int(elec[w, 0])
        o = occ_before[w]
        x = f[occ_after[w][i], o] - f[o[i], o]
        x[i] = 0.0
        col = inv_before[w][:, i]
        a = f[np.ix_(o, o)]
        cond = np.linalg.norm(a, 1) * np.linalg.norm(inv_before[w], 1)
        out[w] = pf_ratio_bound(x, col, 1.0 + x @ col) * cond
    return out


def pf_bound_fn(f):
    """bound_fn for run_chain on Pfaffian chains."""
    def fn(t, chain, k, elec, slot, cw):
        after = chain.book.proposed(k, elec, slot)
        return pf_hop_bound(f, chain.occ_before[cw], after[cw], chain.inv_before[cw], elec[cw])
    return fn
