"""Pfaffian path on the GPU vs the full-recompute oracle (Sec. III, Appendix A)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import EPS32, EPS64, RatioTally, pf_ratio_bound, ratio_err, rel_err, run_chain, pf_bound_fn, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as orc  # noqa: E402
from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.walkers import Walkers  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "c64": torch.complex64, "c128": torch.complex128}


def pf_inputs(seed, L, n, W, cplx):
    g = gen.generator(seed)
    f = gen.skew_from(gen.normal(g, (L, L), cplx))
    occ, emp = gen.occupancy(g, W, L, n)
    return g, f, occ, emp


@pytest.mark.parametrize("dt,n", [(dt, n) for dt in ("c128", "f64", "c64") for n in (2, 8, 34, 100, 256)] +
                         [("c128", 520), ("f64", 616), ("c128", 1024)])
def test_pf_init_matches_oracle(dt, n):
    """Pfaffian init: blocked Parlett-Reid (panels of 16 real / 8-9 complex pairs, set by the
    LDS, so several panels with a ragged last one from n = 34 on; 9 complex pairs at n = 520,
    15 real at 616, 4 complex at the largest order 1024) and the inverse from the same
    factorisation (64 x 64 tiles of U, V = U^-1 and V D^-1 V^T; ragged last tiles at 34, 100,
    520, 616)."""
    say(f"pf init dt={dt} n={n}")
    cplx = dt.startswith("c")
    g, f, occ, emp = pf_inputs(300 + n, 2 * n, n, 4, cplx)
    wk = Walkers(lrx.LRX_PF, DT[dt], f, occ, emp)
    torch.cuda.synchronize()
    a = orc.pairing_matrices(f, occ)
    la, ph = orc.slogpf(a)
    inv = orc.skew_inverse(a)
    np.testing.assert_allclose(wk.st.logabs.cpu().numpy(), la, rtol=0, atol=1e-9 * n)
    np.testing.assert_allclose(wk.st.phase.cpu().numpy(), ph, rtol=0, atol=1e-9 * n)
    m = wk.st.inv.cpu().numpy()
    assert np.array_equal(m, -np.swapaxes(m, 1, 2)), "state must be exactly skew"
    tol = 1e-10 if dt in ("f64", "c128") else 1e-5
    cond = np.linalg.cond(a)
    em = rel_err(m.astype(inv.dtype), inv, axis=(1, 2))
    assert np.all(em <= np.maximum(tol, 64 * cond * (1e-16 if tol < 1e-8 else 6e-8))), em
    assert (wk.st.flags.cpu().numpy() == 0).all()


@pytest.mark.parametrize("dt", ["c128", "f64"])
def test_pf_zero_pivot_walker_is_flagged(dt):
    """A site with no pairing amplitude (zero row and column of F) makes the pairing matrix of
    the walker that holds it singular: its Parlett-Reid row reaches a zero pivot (in the
    second panel here: the site sits at position 50 of n = 64, and the zero row is never
    picked as a pivot partner), pf = 0.  That walker is flagged SINGULAR_A with log|pf| = -inf
    and a zero inverse; the other walkers, which do not hold the site, match the oracle."""
    say(f"pf zero pivot dt={dt}")
    cplx = dt.startswith("c")
    g, f, occ, emp = pf_inputs(910, 128, 64, 3, cplx)
    site = int(occ[1, 50])
    for w in (0, 2):                       # keep the site out of the other walkers
        if site in occ[w]:
            i = int(np.where(occ[w] == site)[0][0])
            occ[w, i] = int(emp[w, 0])
            emp[w, 0] = site
    f = f.copy()
    f[site, :] = 0.0
    f[:, site] = 0.0
    wk = Walkers(lrx.LRX_PF, DT[dt], f, occ, emp)
    torch.cuda.synchronize()
    flags = wk.st.flags.cpu().numpy()
    la = wk.st.logabs.cpu().numpy()
    m = wk.st.inv.cpu().numpy()
    assert flags[1] & lrx.LRX_FLAG_SINGULAR_A and np.isneginf(la[1])
    assert not np.any(m[1]), "a singular walker's inverse is left zero"
    ok = np.array([0, 2])
    assert (flags[ok] == 0).all()
    a = orc.pairing_matrices(f, occ[ok])
    la0, ph0 = orc.slogpf(a)
    np.testing.assert_allclose(la[ok], la0, rtol=0, atol=1e-9 * 64)
    np.testing.assert_allclose(wk.st.phase.cpu().numpy()[ok], ph0, rtol=0, atol=1e-9 * 64)
    em = rel_err(m[ok], orc.skew_inverse(a), axis=(1, 2))
    assert np.all(em <= np.maximum(1e-10, 64 * np.linalg.cond(a) * 1e-16)), em


@pytest.mark.parametrize("dt,n,K,W,steps", [
    ("c128", 64, 0, 6, 25),
    ("c128", 64, 5, 6, 23),
    ("f64", 50, 4, 5, 15),       # ragged n
    ("c128", 128, 32, 3, 36),    # the Pfaffian workload's delay length
])
def test_pf_chain(dt, n, K, W, steps):
    say(f"pf chain dt={dt} n={n} K={K}")
    cplx = dt.startswith("c")
    g, f, occ, emp = pf_inputs(400 + n + K, 2 * n, n, W, cplx)
    draws = [gen.hop_draws(g, W, n, n, (1,), 1) for _ in range(steps)]
    u01 = [gen.uniforms(g, W) for _ in range(steps)]
    wk = Walkers(lrx.LRX_PF, DT[dt], f, occ, emp, 1, K)
    chain = orc.PfChain(f, occ, emp)
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=4, tol_ratio=1e-10, tol_inv=1e-10,
                                         bound_fn=pf_bound_fn(f), growth=lambda t: 1.0 + t)
    say(f"  max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
    np.testing.assert_allclose(la, chain.logabs, atol=1e-8)
    np.testing.assert_allclose(ph, chain.phase, atol=1e-8)
    m = wk.st.inv.cpu().numpy()
    assert np.array_equal(m, -np.swapaxes(m, 1, 2)), "updates and flushes keep M exactly skew"


@pytest.mark.parametrize("K", [0, 5])
def test_pf_fused_hop_step_matches_oracle(K):
    """propose_hop (hop vector built in the ratio kernel), then accept_hop (device
    Metropolis with the given uniforms, fused occupancy commit) follow the oracle's
    chain; the x written by propose_hop equals the separately built one."""
    say(f"pf fused hop step K={K}")
    g, f, occ, emp = pf_inputs(700 + K, 96, 48, 5, True)
    steps = 17
    wk = Walkers(lrx.LRX_PF, torch.complex128, f, occ, emp, 1, K)
    chain = orc.PfChain(f, occ, emp)
    u01 = torch.zeros(5, dtype=torch.float64, device="cuda")
    tally = RatioTally("pf fused hop")
    bound = pf_bound_fn(f)
    for t in range(steps):
        k, elec, slot = gen.hop_draws(g, 5, 48, 48, (1,), 1)
        u = gen.uniforms(g, 5)
        wk.set_draws(k, elec, slot)
        u01.copy_(torch.as_tensor(u))
        x_sep = torch.zeros_like(wk.u)
        lrx.lrx_pf_build_hop(wk.st, wk.table, wk.sites, wk.occ, wk.empty, wk.n_empty, wk._k, wk._elec,
                             wk._slot, x_sep)
        wk.step_device(mode=lrx.LRX_MH_UNIFORMS, u01=u01)
        assert torch.equal(wk.u, x_sep), t
        chain.inv_before, chain.occ_before = chain.inv.copy(), chain.book.occ.copy()
        r_orc = chain.propose(k, elec, slot)
        tally.check(wk.ratio.cpu().numpy(), r_orc, 1e-10, lambda: bound(t, chain, k, elec, slot, np.arange(5)),
                    EPS64, 1.0 + t, where=f"step {t}")
        mask = orc.metropolis(r_orc, u)
        np.testing.assert_array_equal(wk.accept.cpu().numpy().astype(bool), mask)
        chain.accept(k, elec, slot, mask)
    tally.report()
    np.testing.assert_array_equal(wk.occ.cpu().numpy(), chain.book.occ)
    np.testing.assert_array_equal(wk.empty.cpu().numpy(), chain.book.empty)
    assert rel_err(wk.inverse().cpu().numpy(), chain.inv, axis=(1, 2)).max() <= 1e-10
    np.testing.assert_allclose(wk.st.logabs.cpu().numpy(), chain.logabs, atol=1e-9)


def test_pf_c64_bulk_error_is_bounded():
    say("pf c64 chain")
    g, f, occ, emp = pf_inputs(500, 256, 128, 4, True)
    steps = 40
    draws = [gen.hop_draws(g, 4, 128, 128, (1,), 1) for _ in range(steps)]
    u01 = [gen.uniforms(g, 4) for _ in range(steps)]
    wk = Walkers(lrx.LRX_PF, torch.complex64, f, occ, emp, 1, 8, refresh_period=20)
    chain = orc.PfChain(f, occ, emp)
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=10, tol_ratio=1e-4, tol_inv=5e-3,
                                         bound_fn=pf_bound_fn(f), eps=EPS32, growth=lambda t: 1.0 + t % 20)
    say(f"  c64: max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")


def test_pf_refresh_report():
    say("pf refresh")
    g, f, occ, emp = pf_inputs(600, 64, 32, 3, True)
    wk = Walkers(lrx.LRX_PF, torch.complex128, f, occ, emp)
    rep = wk.refresh().cpu().numpy()
    assert rep[:, 0].max() < 1e-13 and rep[:, 1].max() < 1e-12
    wk.st.logabs.add_(0.25)
    rep = wk.refresh().cpu().numpy()
    np.testing.assert_allclose(rep[:, 1], 0.25, atol=1e-10)


def test_pfaffian_workload_full_size_sampled():
    """F = (G - G^T)/2 with G 1024x1024 CN(0,1), n = 512, 256 walkers, complex64 bulk,
    K = 32, over one whole refresh period (64 steps: two delay windows, then the
    complex128 Parlett-Reid refresh) and a few steps past it.  Sampled walkers are
    recomputed by the complex128 oracle: every ratio within 1e-4 relative or, where
    above, within 8 eps32 (1 + steps since refresh) times its first-order bound
    (counted); the inverses before the refresh within 8 eps32 (1 + 64) sqrt(n) cond."""
    wl = gen.WORKLOADS["pfaffian_n512_c64"]
    say(f"full-size {wl.name}")
    f, occ, emp, g = gen.pairing_inputs(wl)
    wk = Walkers(lrx.LRX_PF, torch.complex64, f, occ, emp, 1, wl.delay)
    book = orc.Occupancy(occ, emp)
    sample = np.array([0, 77, 255])
    steps = wl.refresh + 4
    check = set(range(0, wl.refresh, 8)) | {wl.delay - 1, wl.refresh - 1, wl.refresh, steps - 1}
    tally = RatioTally("pfaffian full-size c64")
    errs = []
    for t in range(steps):
        k, elec, slot = gen.hop_draws(g, wl.walkers, wl.n, wl.sites - wl.n, (1,), 1)
        wk.set_draws(k, elec, slot)
        r = wk.propose().cpu().numpy()
        if t in check:
            prop = book.proposed(k, elec, slot)
            a0 = orc.pairing_matrices(f, book.occ[sample])
            la0, ph0 = orc.slogpf(a0)
            la1, ph1 = orc.slogpf(orc.pairing_matrices(f, prop[sample]))
            ref = orc.ratio(la1, ph1, la0, ph0)
            inv0 = orc.skew_inverse(a0)

            def bound():
                out = []
                for j, w in enumerate(sample):
                    i = int(elec[w, 0])
                    o = book.occ[w]
                    x = f[prop[w, i], o] - f[o[i], o]
                    x[i] = 0.0
                    col = inv0[j][:, i]
                    cond = np.linalg.norm(a0[j], 1) * np.linalg.norm(inv0[j], 1)
                    out.append(pf_ratio_bound(x, col, 1.0 + x @ col) * cond)
                return np.array(out)
            since = t % wl.refresh
            er = tally.check(r[sample], ref, 1e-4, bound, EPS32, 1.0 + since, where=f"step {t}")
            errs.append((since, float(er.max()), float(np.median(er))))
        mask = np.ones(wl.walkers, bool)
        wk.decide(mask=mask)
        wk.apply()
        book.commit(k, elec, slot, mask)
        if t == wl.refresh - 1:
            # the state just before the refresh, with every update of the period applied
            inv = wk.inverse().cpu().numpy()[sample]
            a_end = orc.pairing_matrices(f, book.occ[sample])
            oinv = orc.skew_inverse(a_end)
            cond = np.linalg.norm(a_end, 1, axis=(1, 2)) * np.linalg.norm(oinv, 1, axis=(1, 2))
            e_inv = rel_err(inv, oinv, axis=(1, 2))
            say(f"  inverse after {wl.refresh} steps (before the refresh): max {e_inv.max():.2e} "
                f"median {np.median(e_inv):.2e}")
            assert np.all(e_inv <= 8 * EPS32 * (1.0 + wl.refresh) * np.sqrt(wl.n) * cond), (e_inv, cond)
            wk.refresh(report=False)
    tally.report()
    for since, emax, emed in errs:
        say(f"  steps since refresh {since:3d}: ratio rel err max {emax:.2e} median {emed:.2e}")
    np.testing.assert_array_equal(wk.occ.cpu().numpy(), book.occ)
    m = wk.st.inv.cpu().numpy()
    assert np.array_equal(m, -np.swapaxes(m, 1, 2))
