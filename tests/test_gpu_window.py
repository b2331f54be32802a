"""Persistent window over uneven batches vs the full-recompute oracle (Sec. II.C)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import EPS32, EPS64, RatioTally, det_ratio_bound, ratio_err, rel_err, say
from test_rng_host import philox4x32_10

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as orc  # noqa: E402
from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.uneven import UnevenWalkers  # noqa: E402


def small_classes(g, sizes, walkers):
    out = []
    for n, W in zip(sizes, walkers):
        phi = gen.normal(g, (2 * n, n))
        occ, emp = gen.occupancy(g, W, 2 * n, n)
        out.append({"n": n, "phi": phi, "occ": occ, "empty": emp})
    return out


def oracle_window(classes, draws, u01s, mode):
    """Run the oracle chains through the window; returns per class the ratios,
    the decisions, the ratio error bounds and the chain."""
    res = []
    for cls, (k, e, s), u in zip(classes, draws, u01s):
        chain = orc.DetChain(cls["phi"], cls["occ"], cls["empty"])
        rs, masks, bounds = [], [], []
        for t in range(k.shape[0]):
            inv0, occ0 = chain.inv.copy(), chain.book.occ.copy()
            r = chain.propose(k[t], e[t], s[t])
            after = chain.book.proposed(k[t], e[t], s[t])
            bounds.append(det_ratio_bound(cls["phi"], occ0, after, inv0, k[t], e[t]))
            m = orc.metropolis(r, u[t]) if mode == "mh" else np.isfinite(r) & (r != 0)
            chain.accept(k[t], e[t], s[t], m)
            rs.append(r)
            masks.append(m)
        res.append((np.array(rs), np.array(masks), np.array(bounds), chain))
    return res


@pytest.mark.parametrize("dt,delays,steps", [
    ("f64", (4, 5, 3, 7), 11),     # several flushes inside one launch, ragged n
    ("f64", (16, 16, 16, 16), 16),  # one flush at the end of the window
    ("f64", (2, 3, 2, 4), 9),      # flushes every 2-4 steps
])
def test_window_matches_oracle(dt, delays, steps):
    say(f"window {dt} delays={delays} steps={steps}")
    g = gen.generator(900 + steps)
    sizes, walkers = (24, 64, 100, 130), (5, 4, 3, 2)
    classes = small_classes(g, sizes, walkers)
    k_max, ranks = 4, (1, 2, 3, 4)
    draws = [gen.hop_draws_batch(g, steps, W, n, n, ranks, k_max) for n, W in zip(sizes, walkers)]
    u01 = [g.random((steps, W)) for W in walkers]
    ref = oracle_window(classes, draws, u01, "mh")
    uw = UnevenWalkers(torch.float64 if dt == "f64" else torch.float32, classes, k_max, list(delays), steps,
                       grid=7)
    uw.set_draws(draws)
    uw.window(mode=lrx.LRX_MH_MASK, mask=[m for _, m, _, _ in ref])
    torch.cuda.synchronize()
    tally = RatioTally(f"window {dt}")
    for p, (r_o, m_o, bnd, chain), K in zip(uw.parts, ref, delays):
        r = p.ratio.cpu().numpy()
        for t in range(steps):
            tally.check(r[t], r_o[t], 1e-10, bnd[t], EPS64, 1.0 + t, where=f"n={p.st.n} step {t}")
        np.testing.assert_array_equal(p.accept.cpu().numpy().astype(bool), m_o)
        np.testing.assert_array_equal(p.occ.cpu().numpy(), chain.book.occ)
        np.testing.assert_array_equal(p.empty.cpu().numpy(), chain.book.empty)
        assert p.st.slot == steps % K
        np.testing.assert_allclose(p.st.logabs.cpu().numpy(), chain.logabs, atol=1e-9)
    tally.report()
    for inv, (_, _, _, chain) in zip(uw.inverses(), ref):
        assert rel_err(inv.cpu().numpy(), chain.inv, axis=(1, 2)).max() <= 1e-10


def test_window_fp32_forced_and_second_window():
    """FP32 bulk, every proposal applied, two windows back to back (the second
    starts from a partly filled delay window)."""
    say("window f32")
    g = gen.generator(950)
    sizes, walkers = (64, 128, 256), (6, 4, 3)
    classes = small_classes(g, sizes, walkers)
    steps, k_max = 6, 8
    uw = UnevenWalkers(torch.float32, classes, k_max, [4, 8, 5], steps, grid=5)
    chains = [orc.DetChain(c["phi"], c["occ"], c["empty"]) for c in classes]
    tally = RatioTally("window f32")
    for win in range(2):
        draws = [gen.hop_draws_batch(g, steps, W, n, n, (1, 2, 4, 8), k_max) for n, W in zip(sizes, walkers)]
        uw.set_draws(draws)
        uw.window(mode=lrx.LRX_MH_FORCE)
        torch.cuda.synchronize()
        for p, chain, (k, e, s) in zip(uw.parts, chains, draws):
            r = p.ratio.cpu().numpy()
            for t in range(steps):
                inv0, occ0 = chain.inv.copy(), chain.book.occ.copy()
                r_o = chain.propose(k[t], e[t], s[t])
                bnd = det_ratio_bound(p.table.cpu().numpy(), occ0, chain.book.proposed(k[t], e[t], s[t]), inv0,
                                      k[t], e[t])
                tally.check(r[t], r_o, 1e-4, bnd, EPS32, 1.0 + win * steps + t, where=f"win {win} step {t}")
                chain.accept(k[t], e[t], s[t], np.isfinite(r_o) & (r_o != 0))
            np.testing.assert_array_equal(p.occ.cpu().numpy(), chain.book.occ)
    tally.report()


def test_window_device_rng_decisions():
    """LRX_MH_DEVICE_RNG: each decision is u < min(1, |r|^2) with u from
    Philox-4x32-10 keyed by the walker's position in the class list."""
    say("window device rng")
    g = gen.generator(960)
    sizes, walkers = (32, 48), (7, 5)
    classes = small_classes(g, sizes, walkers)
    steps, seed, ctr = 5, 0x0BAD_5EED_1234_5678, 1000
    uw = UnevenWalkers(torch.float64, classes, 2, [3, 4], steps, grid=3)
    uw.set_draws([gen.hop_draws_batch(g, steps, W, n, n, (1, 2), 2) for n, W in zip(sizes, walkers)])
    uw.window(mode=lrx.LRX_MH_DEVICE_RNG, seed=seed, counter=ctr)
    base = 0
    for p in uw.parts:
        r = p.ratio.cpu().numpy()
        acc = p.accept.cpu().numpy().astype(bool)
        for t in range(steps):
            uu = np.empty(p.st.walkers)
            c_t = ctr + t
            for w in range(p.st.walkers):
                c = philox4x32_10([base + w, c_t & 0xFFFFFFFF, c_t >> 32, 0], (seed & 0xFFFFFFFF, seed >> 32))
                uu[w] = (((c[0] >> 5) << 26) | (c[1] >> 6)) * 2.0 ** -53
            np.testing.assert_array_equal(acc[t], orc.metropolis(r[t], uu))
        base += p.st.walkers


def test_uneven_workload_full_size_sampled():
    """4096 walkers, n in {64, 128, 256, 512, 1024}, k in {1, 2, 4, 8}, FP32 bulk, the
    benchmark's per-class delays, over one whole refresh period (eight windows of 16 steps,
    then the FP64 refresh) and one window past it, with Metropolis decisions from the
    device generator.  Two walkers per class follow the same decisions in the oracle:
    ratios within 1e-4 relative or, above it, within 8 eps32 (1 + steps since refresh)
    times their first-order bound (counted); inverses just before the refresh within
    8 eps32 (1 + 128) sqrt(n) cond_1(A)."""
    wl = gen.WORKLOADS["uneven_n64_1024_fp32"]
    say(f"full-size {wl.name}")
    classes, g = gen.uneven_inputs(wl)
    delays = {64: 4, 128: 8, 256: 8, 512: 16, 1024: 32}
    steps, P = wl.delay, wl.refresh
    uw = UnevenWalkers(torch.float32, classes, wl.k_max, [delays[c["n"]] for c in classes], steps)
    samples = [np.array([0, len(c["walkers"]) - 1]) for c in classes]
    books = [orc.Occupancy(c["occ"][sm], c["empty"][sm]) for c, sm in zip(classes, samples)]
    tally = RatioTally("uneven full-size f32")
    errs = []
    for win in range(P // steps + 1):
        draws = [gen.hop_draws_batch(g, steps, len(c["walkers"]), c["n"], c["n"], wl.ranks, wl.k_max)
                 for c in classes]
        uw.set_draws(draws)
        uw.window(mode=lrx.LRX_MH_DEVICE_RNG, seed=77, counter=win * steps)
        torch.cuda.synchronize()
        for p, cls, sm, book, (k, e, s) in zip(uw.parts, classes, samples, books, draws):
            r = p.ratio.cpu().numpy()[:, sm]
            acc = p.accept.cpu().numpy()[:, sm].astype(bool)
            every = 1 if cls["n"] <= 128 else (4 if cls["n"] <= 256 else 8)
            for t in range(steps):
                since = (win * steps + t) % P
                kk, ee, ss = k[t][sm], e[t][sm], s[t][sm]
                if t % every == 0 or t == steps - 1:
                    la0, ph0, inv0 = orc.slogdet(orc.slater_matrices(cls["phi"], book.occ))
                    prop = book.proposed(kk, ee, ss)
                    la1, ph1, _ = orc.slogdet(orc.slater_matrices(cls["phi"], prop), want_inv=False)
                    r_o = orc.ratio(la1, ph1, la0, ph0)
                    bnd = det_ratio_bound(cls["phi"], book.occ, prop, inv0, kk, ee)
                    er = tally.check(r[t], r_o, 1e-4, bnd, EPS32, 1.0 + since, where=f"n={cls['n']} step {since}")
                    errs.append((cls["n"], since, float(er.max())))
                book.commit(kk, ee, ss, acc[t])
            np.testing.assert_array_equal(p.occ.cpu().numpy()[sm], book.occ)
        if (win + 1) * steps == P:
            # just before the refresh: every class's delay window is empty (K divides 128)
            for p, cls, sm, book in zip(uw.parts, classes, samples, books):
                assert p.st.slot == 0
                inv = p.st.inv.cpu().numpy()[sm].astype(np.float64).transpose(0, 2, 1)
                a = orc.slater_matrices(cls["phi"], book.occ)
                _, _, oinv = orc.slogdet(a)
                cond = np.linalg.norm(a, 1, axis=(1, 2)) * np.linalg.norm(oinv, 1, axis=(1, 2))
                e_inv = rel_err(inv, oinv, axis=(1, 2))
                say(f"  n={cls['n']}: inverse after {P} steps (before the refresh) {e_inv.max():.2e}, "
                    f"cond {cond.max():.1e}")
                assert np.all(e_inv <= 8 * EPS32 * (1.0 + P) * np.sqrt(cls["n"]) * cond), (e_inv, cond)
            uw.refresh(report=False)
    tally.report()
    for n in sorted({x[0] for x in errs}):
        m = [x[2] for x in errs if x[0] == n]
        say(f"  n={n}: ratio rel err max {max(m):.2e} median {float(np.median(m)):.2e} over {len(m)} checks")


def test_autotuned_delays_and_grid(tmp_path, monkeypatch):
    """delays="auto" / grid="auto": the tuned K per class is one of the candidates, the
    choices are cached, and the grid search leaves the walkers' state untouched."""
    from paper_2602_05255_amd import autotune
    monkeypatch.setenv("LRX_TUNE_CACHE", str(tmp_path / "tune.json"))
    say("autotune")
    g = gen.generator(970)
    sizes, walkers, ranks = (64, 200), (40, 24), (1, 2, 4)
    classes = small_classes(g, sizes, walkers)
    steps = 8
    uw = UnevenWalkers(torch.float64, classes, 4, "auto", steps, grid="auto", ranks=ranks)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert uw.grid % cus == 0 and 1 <= uw.grid // cus <= 4
    for p, n in zip(uw.parts, sizes):
        assert p.st.delay in autotune.delay_candidates(n, 4, ranks)
        assert p.st.slot == 0
        # the choice is registered with the library's tuning table
        t = lrx.lrx_autotune_lookup(torch.float64, n, 4)
        assert t["tuned"] and t["delay"] == p.st.delay and t["rows_per_block"] in autotune.rows_candidates(n)
    assert (tmp_path / "tune.json").exists()
    chains = [orc.DetChain(c["phi"], c["occ"], c["empty"]) for c in classes]
    draws = [gen.hop_draws_batch(g, steps, W, n, n, ranks, 4) for n, W in zip(sizes, walkers)]
    uw.set_draws(draws)
    uw.window(mode=lrx.LRX_MH_FORCE)
    tally = RatioTally("autotuned window")
    for p, chain, (k, e, s) in zip(uw.parts, chains, draws):
        r = p.ratio.cpu().numpy()
        for t in range(steps):
            inv0, occ0 = chain.inv.copy(), chain.book.occ.copy()
            r_o = chain.propose(k[t], e[t], s[t])
            bnd = det_ratio_bound(p.table.cpu().numpy(), occ0, chain.book.proposed(k[t], e[t], s[t]), inv0,
                                  k[t], e[t])
            # linear growth over the t updates since the start (no refresh in this test)
            tally.check(r[t], r_o, 1e-10, bnd, EPS64, 1.0 + t, where=f"n={p.st.n} K={p.st.delay} step {t}")
            chain.accept(k[t], e[t], s[t], np.isfinite(r_o) & (r_o != 0))
        np.testing.assert_array_equal(p.occ.cpu().numpy(), chain.book.occ)
    tally.report()
