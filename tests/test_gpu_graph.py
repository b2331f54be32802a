"""The benchmark's production path -- one refresh period of a walker batch split into
four sub-batches on four streams (staggered refreshes, flushes every K steps) captured
into one HIP graph -- replayed several times and followed by the full-recompute oracle.
The decisions are Metropolis with uniforms that the graph reads from device memory, refilled
before every replay, so every replay is a new stretch of the chain; the oracle takes its
own decisions from its own ratios and the same uniforms."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import EPS64, RatioTally, det_ratio_bound, pf_hop_bound, rel_err, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as orc  # noqa: E402
from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.driver import PeriodDriver  # noqa: E402


def _walker_order(off, P):
    """Draw indices a sub-batch with offset `off` uses during one period."""
    return [(t + off) % P for t in range(P)]


@pytest.mark.parametrize("kind,dt,n,ranks,K,P", [
    ("det", torch.float64, 64, (1, 2, 4), 4, 16),
    ("pf", torch.complex128, 48, (1,), 4, 16),
])
def test_graph_period_replays_match_oracle(kind, dt, n, ranks, K, P):
    say(f"graph period {kind} n={n} K={K} P={P}")
    g = gen.generator(4200 + n)
    W, L, parts, replays = 32, 2 * n, 4, 3
    k_max = max(ranks)
    if kind == "det":
        table = gen.normal(g, (L, n))
        chain_cls = orc.DetChain
    else:
        table = gen.skew_from(gen.normal(g, (L, L), True))
        chain_cls = orc.PfChain
    occ, emp = gen.occupancy(g, W, L, n)
    k, e, s = gen.hop_draws_batch(g, P, W, n, L - n, ranks, k_max)
    draws = tuple(torch.as_tensor(x).cuda() for x in (k, e, s))
    log = torch.zeros(P, W, dtype=torch.float64 if kind == "det" else torch.complex128, device="cuda")
    u01 = torch.zeros(P, W, dtype=torch.float64, device="cuda")
    drv = PeriodDriver(lrx.LRX_DET if kind == "det" else lrx.LRX_PF, dt, table, occ, emp, k_max, K, P, draws,
                       streams=parts, ratio_log=log, mode=lrx.LRX_MH_UNIFORMS, u01=u01)
    assert len(set(drv.offsets)) == parts, drv.offsets       # staggered refreshes
    chains = []
    uh = g.random((P, W))
    u01.copy_(torch.as_tensor(uh))
    for (wk, a0, a1, _), off in zip(drv.parts, drv.offsets):
        ch = chain_cls(table, occ[a0:a1], emp[a0:a1])
        for t in range(off):                                  # what prime() does
            r = ch.propose(k[t, a0:a1], e[t, a0:a1], s[t, a0:a1])
            ch.accept(k[t, a0:a1], e[t, a0:a1], s[t, a0:a1], orc.metropolis(r, uh[t, a0:a1]))
        chains.append(ch)
    drv.capture()                                             # one eager period, then the recording
    tally = RatioTally(f"graph {kind}")

    def follow(check):
        got = log.cpu().numpy()
        for (wk, a0, a1, _), off, ch in zip(drv.parts, drv.offsets, chains):
            for t in _walker_order(off, P):
                kk, ee, ss = k[t, a0:a1], e[t, a0:a1], s[t, a0:a1]
                inv0, occ0 = ch.inv.copy(), ch.book.occ.copy()
                r = ch.propose(kk, ee, ss)
                if check:
                    if kind == "det":
                        bound = (lambda: det_ratio_bound(table, occ0, ch.book.proposed(kk, ee, ss), inv0, kk, ee))
                    else:
                        bound = (lambda: pf_hop_bound(table, occ0, ch.book.proposed(kk, ee, ss), inv0, ee))
                    tally.check(got[t, a0:a1], r, 1e-10, bound, EPS64, 1.0 + P, where=f"part {a0} step {t}")
                ch.accept(kk, ee, ss, orc.metropolis(r, uh[t, a0:a1]))

    follow(check=True)                                        # the eager warm-up period
    for rep in range(replays):
        uh = g.random((P, W))                                 # fresh uniforms for this replay
        u01.copy_(torch.as_tensor(uh))
        drv.graph.replay()
        torch.cuda.synchronize()
        follow(check=True)
        for (wk, a0, a1, _), ch in zip(drv.parts, chains):
            np.testing.assert_array_equal(wk.occ.cpu().numpy(), ch.book.occ)
            np.testing.assert_allclose(wk.st.logabs.cpu().numpy(), ch.logabs, atol=1e-9)
            np.testing.assert_allclose(wk.st.phase.cpu().numpy(), ch.phase, atol=1e-9)
        say(f"  replay {rep}: occupancy, log|value| and phase agree")
    tally.report()
    assert tally.checked == (replays + 1) * P * W
    # Inverses: 1e-10, or for an ill-conditioned walker sqrt(n) eps cond_1(A) times the
    # updates since its last refresh (at most P), the error the oracle's own inverse carries
    # too (counted).
    n_cond = 0
    for (wk, a0, a1, _), ch in zip(drv.parts, chains):
        inv = wk.inverse().cpu().numpy()
        o = ch.book.occ
        a = table[o] if kind == "det" else table[o[:, :, None], o[:, None, :]]
        cond = np.linalg.norm(a, 1, axis=(1, 2)) * np.linalg.norm(ch.inv, 1, axis=(1, 2))
        tol = np.maximum(1e-10, np.sqrt(n) * EPS64 * (1.0 + P) * cond)
        n_cond += int(np.sum(tol > 1e-10))
        err = rel_err(inv, ch.inv, axis=(1, 2))
        assert np.all(err <= tol), (err, cond)
    say(f"  inverses: {n_cond} of {W} walkers held to their conditioning bound instead of 1e-10")


def test_graph_uneven_windows_and_refresh_replays_match_oracle():
    """Two persistent windows (several flushes inside each) and the FP64 refresh of every
    size class, captured into one HIP graph and replayed; every ratio of every replay is
    checked against the oracle chain."""
    from paper_2602_05255_amd.uneven import UnevenWalkers
    say("graph uneven windows + refresh")
    g = gen.generator(4300)
    sizes, walkers, delays = (40, 96, 130), (6, 5, 4), (4, 2, 8)
    steps, nwin, k_max, ranks = 8, 2, 4, (1, 2, 4)
    P = steps * nwin
    classes = []
    for n, W in zip(sizes, walkers):
        phi = gen.normal(g, (2 * n, n))
        occ, emp = gen.occupancy(g, W, 2 * n, n)
        classes.append({"n": n, "phi": phi, "occ": occ, "empty": emp})
    uw = UnevenWalkers(torch.float64, classes, k_max, list(delays), steps, grid=6)
    draws = [gen.hop_draws_batch(g, P, W, n, n, ranks, k_max) for n, W in zip(sizes, walkers)]
    dev = [tuple(torch.as_tensor(x).cuda() for x in d) for d in draws]
    logs = [torch.zeros(P, W, dtype=torch.float64, device="cuda") for W in walkers]
    accs = [torch.zeros(P, W, dtype=torch.uint8, device="cuda") for W in walkers]
    u01s = [torch.zeros(P, W, dtype=torch.float64, device="cuda") for W in walkers]

    def period():
        for i in range(nwin):
            sl = slice(i * steps, (i + 1) * steps)
            for p, (k, e, s), lg, ac, uu in zip(uw.parts, dev, logs, accs, u01s):
                p.k, p.elec, p.slot, p.ratio, p.accept, p.u01 = k[sl], e[sl], s[sl], lg[sl], ac[sl], uu[sl]
            lrx.lrx_det_window(uw.parts, steps, lrx.LRX_MH_UNIFORMS, 0, i * steps, uw.work, uw.grid)
        uw.refresh(report=False)

    uh = []

    def fresh_uniforms():
        uh.clear()
        for uu, W in zip(u01s, walkers):
            x = g.random((P, W))
            uu.copy_(torch.as_tensor(x))
            uh.append(x)

    chains = [orc.DetChain(c["phi"], c["occ"], c["empty"]) for c in classes]
    tally = RatioTally("graph uneven")

    def follow():
        for ch, lg, (k, e, s), c, u in zip(chains, logs, draws, classes, uh):
            got = lg.cpu().numpy()
            for t in range(P):
                inv0, occ0 = ch.inv.copy(), ch.book.occ.copy()
                r = ch.propose(k[t], e[t], s[t])
                tally.check(got[t], r, 1e-10,
                            lambda: det_ratio_bound(c["phi"], occ0, ch.book.proposed(k[t], e[t], s[t]), inv0, k[t],
                                                    e[t]), EPS64, 1.0 + t, where=f"n={c['n']} step {t}")
                ch.accept(k[t], e[t], s[t], orc.metropolis(r, u[t]))

    fresh_uniforms()
    s_ = torch.cuda.Stream()
    s_.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_):
        period()                                   # eager warm-up period
    torch.cuda.current_stream().wait_stream(s_)
    torch.cuda.synchronize()
    follow()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        period()
    torch.cuda.synchronize()
    for rep in range(3):
        fresh_uniforms()
        graph.replay()
        torch.cuda.synchronize()
        follow()
        for p, ch in zip(uw.parts, chains):
            np.testing.assert_array_equal(p.occ.cpu().numpy(), ch.book.occ)
            np.testing.assert_allclose(p.st.logabs.cpu().numpy(), ch.logabs, atol=1e-9)
            # the refresh closes the period: the stored inverse is the fresh FP64 one
            inv = p.st.inv.cpu().numpy().transpose(0, 2, 1)
            a = orc.slater_matrices(p.table.cpu().numpy(), ch.book.occ)
            cond = np.linalg.norm(a, 1, axis=(1, 2)) * np.linalg.norm(ch.inv, 1, axis=(1, 2))
            assert np.all(rel_err(inv, ch.inv, axis=(1, 2)) <= np.maximum(1e-10, 8 * EPS64 * cond))
        say(f"  replay {rep}: occupancy, log|det| and inverses agree")
    tally.report()
