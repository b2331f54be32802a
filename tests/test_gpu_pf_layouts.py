"""Fused (delay-one) and packed-skew Pfaffian layouts on the GPU vs the full-recompute
oracle (Eq. pf_inv with k = 1; skewness of A^-1, Sec. III.A), and the read-out of A^-1
from every layout (Eq. pf_delayed_Ainv)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import EPS32, rel_err, run_chain, pf_bound_fn, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as orc  # noqa: E402
from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.walkers import Walkers  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "c64": torch.complex64, "c128": torch.complex128}
FUSED, PACKED = lrx.LRX_LAYOUT_FUSED, lrx.LRX_LAYOUT_PACKED
NAME = {FUSED: "fused", PACKED: "packed"}


def pf_inputs(seed, L, n, W, cplx):
    g = gen.generator(seed)
    f = gen.skew_from(gen.normal(g, (L, L), cplx))
    occ, emp = gen.occupancy(g, W, L, n)
    return g, f, occ, emp


def read_inverse(wk):
    out = torch.empty(wk.W, wk.n, wk.n, dtype=wk.st.dtype, device="cuda")
    lrx.lrx_pf_read_inverse(wk.st, out)
    return out.cpu().numpy()


@pytest.mark.parametrize("dt,n,layout,W,steps,refresh", [
    ("c128", 64, FUSED, 6, 30, 0),
    ("c128", 64, PACKED, 6, 30, 0),
    ("f64", 50, FUSED, 5, 21, 0),          # ragged rows of the full-storage pass
    ("f64", 130, PACKED, 5, 21, 0),        # three tile rows, the last one ragged
    ("c128", 200, PACKED, 3, 26, 9),       # packed refresh inside the chain
    ("c128", 192, FUSED, 3, 26, 9),
])
def test_pf_layout_chain(dt, n, layout, W, steps, refresh):
    """The chain of single hops with Metropolis decisions (accepted and rejected walkers
    mixed): ratios every step against the oracle, the inverse every 7 steps (the check
    flushes the pending updates, so the pass runs both with and without one)."""
    say(f"pf layout chain dt={dt} n={n} layout={NAME[layout]} refresh={refresh}")
    cplx = dt.startswith("c")
    g, f, occ, emp = pf_inputs(800 + n + layout, 2 * n, n, W, cplx)
    draws = [gen.hop_draws(g, W, n, n, (1,), 1) for _ in range(steps)]
    u01 = [gen.uniforms(g, W) for _ in range(steps)]
    wk = Walkers(lrx.LRX_PF, DT[dt], f, occ, emp, 1, 0, refresh_period=refresh, layout=layout)
    chain = orc.PfChain(f, occ, emp)
    stats = []
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=7, tol_ratio=1e-10, tol_inv=1e-10,
                                         bound_fn=pf_bound_fn(f), growth=lambda t: 1.0 + t, stats=stats)
    acc = sum(s[2] for s in stats if isinstance(s[0], int))
    say(f"  max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}; accepted {acc} of {W * steps}")
    assert 0 < acc < W * steps, "the chain must mix accepted and rejected walkers"
    np.testing.assert_allclose(la, chain.logabs, atol=1e-8)
    np.testing.assert_allclose(ph, chain.phase, atol=1e-8)


@pytest.mark.parametrize("layout", [FUSED, PACKED])
def test_pf_layout_read_inverse_with_pending(layout):
    """read_inverse with a pending update per walker (no flush) equals the oracle's A^-1, is
    exactly skew, and equals the read-out after the flush; every walker accepts at the
    first step and about half at the second, so pending updates of both ages are present."""
    say(f"pf read-out with pending layout={NAME[layout]}")
    n, W = 96, 6
    g, f, occ, emp = pf_inputs(900 + layout, 2 * n, n, W, True)
    wk = Walkers(lrx.LRX_PF, torch.complex128, f, occ, emp, 1, 0, layout=layout)
    chain = orc.PfChain(f, occ, emp)
    for t, mask in enumerate([np.ones(W, bool), np.array([1, 0, 1, 0, 1, 0], bool),
                              np.array([0, 1, 1, 0, 0, 1], bool)]):
        k, elec, slot = gen.hop_draws(g, W, n, n, (1,), 1)
        wk.set_draws(k, elec, slot)
        r = wk.propose().cpu().numpy()
        r_o = chain.propose(k, elec, slot)
        assert rel_err(r, r_o).max() < 1e-10, t
        wk.decide(mask=mask)
        wk.apply()
        chain.accept(k, elec, slot, mask)
        assert wk.st.slot == 1
        m = read_inverse(wk)
        assert np.array_equal(m, -np.swapaxes(m, 1, 2)), "read-out must be exactly skew"
        assert rel_err(m, chain.inv, axis=(1, 2)).max() <= 1e-11, t
    before = read_inverse(wk)
    wk.flush()
    assert wk.st.slot == 0
    after = read_inverse(wk)
    assert rel_err(after, before, axis=(1, 2)).max() <= 1e-13
    if layout == FUSED:
        m0 = wk.st.inv.cpu().numpy()
        assert np.array_equal(m0, -np.swapaxes(m0, 1, 2)), "the pass keeps M0 exactly skew"


@pytest.mark.parametrize("dt,n,K,W,steps", [
    ("c128", 130, 5, 5, 23),       # ragged last tile row, flushes inside the chain
    ("f64", 200, 8, 4, 26),
    ("c128", 64, 32, 3, 36),       # one tile, the Pfaffian workload's delay length
])
def test_pf_packed_delayed_chain(dt, n, K, W, steps):
    """Delayed updates on packed skew storage (A_0^-1 x from the upper tiles, the flush writing
    the stored tiles only) against the oracle chain; read-outs mid-window equal the oracle's A^-1
    and are exactly skew."""
    say(f"pf packed delayed dt={dt} n={n} K={K}")
    cplx = dt.startswith("c")
    g, f, occ, emp = pf_inputs(990 + n + K, 2 * n, n, W, cplx)
    draws = [gen.hop_draws(g, W, n, n, (1,), 1) for _ in range(steps)]
    u01 = [gen.uniforms(g, W) for _ in range(steps)]
    wk = Walkers(lrx.LRX_PF, DT[dt], f, occ, emp, 1, K, layout=PACKED)
    chain = orc.PfChain(f, occ, emp)
    stats = []
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=7, tol_ratio=1e-10, tol_inv=1e-10,
                                         bound_fn=pf_bound_fn(f), growth=lambda t: 1.0 + t, stats=stats)
    say(f"  max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
    np.testing.assert_allclose(la, chain.logabs, atol=1e-8)
    np.testing.assert_allclose(ph, chain.phase, atol=1e-8)
    # a few more steps without a flush: the read-out carries the live slots
    for t in range(min(3, K - 1)):
        k, elec, slot = gen.hop_draws(g, W, n, n, (1,), 1)
        wk.set_draws(k, elec, slot)
        wk.propose()
        r_o = chain.propose(k, elec, slot)
        mask = np.abs(r_o) > 0.3
        wk.decide(mask=mask)
        wk.apply()
        chain.accept(k, elec, slot, mask)
    m = read_inverse(wk)
    assert np.array_equal(m, -np.swapaxes(m, 1, 2))
    assert rel_err(m, chain.inv, axis=(1, 2)).max() <= 1e-10


def test_pf_read_inverse_delayed_full_layout():
    """read_inverse of a delayed full-storage state mid-window (M0 plus live slots)."""
    say("pf read-out delayed")
    n, W, K = 80, 4, 6
    g, f, occ, emp = pf_inputs(950, 2 * n, n, W, False)
    wk = Walkers(lrx.LRX_PF, torch.float64, f, occ, emp, 1, K)
    chain = orc.PfChain(f, occ, emp)
    for t in range(4):
        k, elec, slot = gen.hop_draws(g, W, n, n, (1,), 1)
        wk.set_draws(k, elec, slot)
        wk.propose()
        r_o = chain.propose(k, elec, slot)
        mask = np.abs(r_o) > 0.3
        wk.decide(mask=mask)
        wk.apply()
        chain.accept(k, elec, slot, mask)
    assert wk.st.slot == 4
    m = read_inverse(wk)
    assert np.array_equal(m, -np.swapaxes(m, 1, 2))
    assert rel_err(m, chain.inv, axis=(1, 2)).max() <= 1e-11
    assert wk.st.slot == 4, "read-out leaves the state as it was"


def test_pf_packed_refresh_report_and_init():
    """Packed init/refresh: the unpacked state equals the full-storage init exactly (same
    factorisation, same rounding), and a refresh right after init reports no drift."""
    say("pf packed init")
    n, W = 150, 3
    g, f, occ, emp = pf_inputs(960, 2 * n, n, W, True)
    full = Walkers(lrx.LRX_PF, torch.complex64, f, occ, emp)
    packed = Walkers(lrx.LRX_PF, torch.complex64, f, occ, emp, layout=PACKED)
    assert np.array_equal(read_inverse(packed), full.st.inv.cpu().numpy())
    rep = packed.refresh().cpu().numpy()
    assert rep[:, 0].max() < 1e-7 and rep[:, 1].max() < 1e-6
    np.testing.assert_array_equal(packed.st.logabs.cpu().numpy(), full.st.logabs.cpu().numpy())


def test_pf_layouts_agree_at_workload_shape():
    """The Pfaffian workload's shape (n = 512, L = 1024), complex128 bulk: 32 walkers, 16
    steps on the plain, fused and packed layouts from the same draws and the same decisions
    (accept iff |r| > 0.3 from the plain layout's ratio).  The read-outs agree across layouts
    on every walker, and with the oracle chain on two sampled walkers."""
    say("pf layouts at n=512")
    n, L, W, steps = 512, 1024, 32, 16
    g, f, occ, emp = pf_inputs(970, L, n, W, True)
    lays = (lrx.LRX_LAYOUT_FULL, FUSED, PACKED, "packed_delayed")
    wks = {lay: Walkers(lrx.LRX_PF, torch.complex128, f, occ, emp, 1, 0, layout=lay) for lay in lays[:3]}
    wks["packed_delayed"] = Walkers(lrx.LRX_PF, torch.complex128, f, occ, emp, 1, 6, layout=PACKED)
    NAME["packed_delayed"] = "packed delayed (K = 6)"
    sample = np.array([3, 21])
    chain = orc.PfChain(f, occ[sample], emp[sample])
    taken = 0
    for t in range(steps):
        k, elec, slot = gen.hop_draws(g, W, n, L - n, (1,), 1)
        rs = {}
        for lay, wk in wks.items():
            wk.set_draws(k, elec, slot)
            rs[lay] = wk.propose().cpu().numpy()
        for lay in lays[1:]:
            assert rel_err(rs[lay], rs[lrx.LRX_LAYOUT_FULL]).max() <= 1e-9, (NAME[lay], t)
        mask = np.abs(rs[lrx.LRX_LAYOUT_FULL]) > 0.3
        taken += int(mask.sum())
        for wk in wks.values():
            wk.decide(mask=mask)
            wk.apply()
        r_o = chain.propose(k[sample], elec[sample], slot[sample])
        assert rel_err(rs[lrx.LRX_LAYOUT_FULL][sample], r_o).max() <= 1e-9, t
        chain.accept(k[sample], elec[sample], slot[sample], mask[sample])
    say(f"  accepted {taken} of {W * steps}")
    ref = read_inverse(wks[lrx.LRX_LAYOUT_FULL])
    assert rel_err(ref[sample], chain.inv, axis=(1, 2)).max() <= 1e-9
    for lay in lays[1:]:
        np.testing.assert_array_equal(wks[lay].occ.cpu().numpy(), wks[lrx.LRX_LAYOUT_FULL].occ.cpu().numpy())
        m = read_inverse(wks[lay])
        e = rel_err(m, ref, axis=(1, 2))
        say(f"  {NAME[lay]} vs plain: max rel diff {e.max():.2e}")
        assert e.max() <= 1e-9, NAME[lay]
        np.testing.assert_allclose(wks[lay].st.logabs.cpu().numpy()[sample], chain.logabs, atol=1e-8)


def test_pf_layout_c64_bulk():
    """complex64 bulk on both layouts: a 40-step Metropolis chain with ratios and inverses
    held to single-precision bounds (as the full-storage complex64 chain)."""
    for layout in (FUSED, PACKED):
        say(f"pf c64 chain layout={NAME[layout]}")
        g, f, occ, emp = pf_inputs(980 + layout, 256, 128, 4, True)
        steps = 40
        draws = [gen.hop_draws(g, 4, 128, 128, (1,), 1) for _ in range(steps)]
        u01 = [gen.uniforms(g, 4) for _ in range(steps)]
        wk = Walkers(lrx.LRX_PF, torch.complex64, f, occ, emp, 1, 0, refresh_period=20, layout=layout)
        chain = orc.PfChain(f, occ, emp)
        worst_r, worst_m, _, _ = run_chain(wk, chain, draws, u01, check_every=10, tol_ratio=1e-4, tol_inv=5e-3,
                                           bound_fn=pf_bound_fn(f), eps=EPS32, growth=lambda t: 1.0 + t % 20)
        say(f"  c64 {NAME[layout]}: max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
