"""Determinant path on the GPU vs the full-recompute oracle (Sec. II)."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import (EPS32, EPS64, RatioTally, det_bound_fn, det_ratio_bound, ratio_err, rel_err, run_chain,
                      say)
from test_rng_host import philox4x32_10

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as orc  # noqa: E402
from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.walkers import Walkers  # noqa: E402

DT = {"f64": torch.float64, "f32": torch.float32, "c64": torch.complex64, "c128": torch.complex128}


def draws_for(g, steps, W, n, n_empty, ranks, k_max):
    d = [gen.hop_draws(g, W, n, n_empty, ranks, k_max) for _ in range(steps)]
    u = [gen.uniforms(g, W) for _ in range(steps)]
    return d, u


@pytest.mark.parametrize("dt", ["f64", "c128", "f32", "c64"])
@pytest.mark.parametrize("n", [1, 7, 32, 100, 130, 256])
def test_init_inverse_matches_oracle(dt, n):
    say(f"init_inverse dt={dt} n={n}")
    cplx = dt in ("c64", "c128")
    g = gen.generator(100 + n)
    W, L = 5, 2 * n + 3
    phi = gen.normal(g, (L, n), cplx)
    occ, emp = gen.occupancy(g, W, L, n)
    wk = Walkers(lrx.LRX_DET, DT[dt], phi, occ, emp)
    torch.cuda.synchronize()
    la, ph, inv = orc.slogdet(orc.slater_matrices(phi, occ))
    got = wk.inverse().cpu().numpy()
    tol = 1e-10 if dt in ("f64", "c128") else 1e-5
    cond = np.linalg.cond(orc.slater_matrices(phi, occ))
    em = rel_err(got, inv, axis=(1, 2))
    assert np.all(em <= np.maximum(tol, 64 * cond * np.finfo(np.float64 if tol < 1e-8 else np.float32).eps)), em
    np.testing.assert_allclose(wk.st.logabs.cpu().numpy(), la, rtol=0, atol=1e-9 * max(n, 1))
    np.testing.assert_allclose(wk.st.phase.cpu().numpy(), ph, rtol=0, atol=1e-9 * max(n, 1))
    assert (wk.st.flags.cpu().numpy() == 0).all()


@pytest.mark.parametrize("dt,n", [("f64", 1024), ("c128", 520), ("f64", 616), ("c128", 616)])
def test_init_inverse_large(dt, n):
    """The largest sizes: several 64-column outer panels, each eliminated in
    register-resident blocks (32 columns real / 8 complex above n = 512, with the
    MFMA sub-block update between them; n = 616 ends on a 40-column outer panel,
    so its second block is 8 wide) and applied to the rest of the matrix by the
    MFMA outer update."""
    say(f"init_inverse large dt={dt} n={n}")
    cplx = dt == "c128"
    g = gen.generator(150 + n)
    W, L = 3, 2 * n
    phi = gen.normal(g, (L, n), cplx)
    occ, emp = gen.occupancy(g, W, L, n)
    wk = Walkers(lrx.LRX_DET, DT[dt], phi, occ, emp)
    torch.cuda.synchronize()
    a = orc.slater_matrices(phi, occ)
    la, ph, inv = orc.slogdet(a)
    cond = np.linalg.norm(a, 1, axis=(1, 2)) * np.linalg.norm(inv, 1, axis=(1, 2))
    em = rel_err(wk.inverse().cpu().numpy(), inv, axis=(1, 2))
    assert np.all(em <= np.maximum(1e-10, 8 * EPS64 * cond)), (em, cond)
    np.testing.assert_allclose(wk.st.logabs.cpu().numpy(), la, rtol=0, atol=1e-9 * n)
    np.testing.assert_allclose(wk.st.phase.cpu().numpy(), ph, rtol=0, atol=1e-9 * n)


def test_init_dense_batch_and_singular():
    say("init dense batch with a singular member")
    g = gen.generator(7)
    n, W = 12, 4
    a = g.standard_normal((W, n, n))
    a[2, 5] = 0.0              # a zero row: exactly singular in any elimination order
    st = lrx.State(lrx.LRX_DET, torch.float64, W, n)
    lrx.lrx_det_init_inverse(st, torch.as_tensor(a).cuda(), n, None)
    torch.cuda.synchronize()
    flags = st.flags.cpu().numpy()
    assert flags[2] & lrx.LRX_FLAG_SINGULAR_A
    assert (flags[[0, 1, 3]] == 0).all()
    la, ph, inv = orc.slogdet(a[[0, 1, 3]])
    got = st.inv.cpu().numpy()[[0, 1, 3]].transpose(0, 2, 1)
    assert rel_err(got, inv, axis=(1, 2)).max() <= 1e-10
    assert st.logabs.cpu().numpy()[2] == -np.inf


def test_slater_n32_fp64_every_step():
    """Plain Sherman-Morrison, Phi 64x32, 16 walkers x 200 single hops, FP64, checked every step."""
    wl = gen.WORKLOADS["slater_n32_fp64"]
    say(f"chain {wl.name}")
    phi, occ, emp, g = gen.slater_inputs(wl)
    draws, u01 = draws_for(g, wl.steps, wl.walkers, wl.n, wl.sites - wl.n, wl.ranks, wl.k_max)
    wk = Walkers(lrx.LRX_DET, torch.float64, phi, occ, emp, wl.k_max, wl.delay)
    chain = orc.DetChain(phi, occ, emp)
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, tol_ratio=1e-10, tol_inv=1e-10,
                                         bound_fn=det_bound_fn(phi))
    say(f"  max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
    np.testing.assert_allclose(la, chain.logabs, atol=1e-9)
    np.testing.assert_allclose(ph, chain.phase, atol=1e-12)


@pytest.mark.parametrize("n,k_max,ranks,K,W,steps", [
    (256, 4, (1, 2, 4), 16, 24, 40),     # the scale workload's shape, fewer walkers
    (100, 2, (1, 2), 5, 9, 23),          # ragged n, ragged final window
    (64, 8, (1, 3, 8), 4, 6, 13),        # largest rank, odd ranks
    (33, 1, (1,), 3, 5, 10),             # odd n (unaligned rows)
    (128, 8, (1, 4, 8), 16, 6, 36),      # K k_max = 128 > 64 live slot columns (wider G grouping)
    (600, 4, (1, 2, 4), 16, 3, 24),      # n > 512: four entries a thread in the propose, ragged n
    (200, 8, (8,), 32, 3, 40),           # 256 live slot columns: propose LDS above 64 KB
])
def test_delayed_det_chain_fp64(n, k_max, ranks, K, W, steps):
    say(f"delayed det chain n={n} k_max={k_max} K={K} W={W}")
    g = gen.generator(1000 + n)
    L = 2 * n
    phi = gen.normal(g, (L, n))
    occ, emp = gen.occupancy(g, W, L, n)
    draws, u01 = draws_for(g, steps, W, n, L - n, ranks, k_max)
    wk = Walkers(lrx.LRX_DET, torch.float64, phi, occ, emp, k_max, K)
    chain = orc.DetChain(phi, occ, emp)
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=3, tol_ratio=1e-10, tol_inv=1e-10,
                                         bound_fn=det_bound_fn(phi))
    say(f"  max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
    np.testing.assert_allclose(la, chain.logabs, atol=1e-8)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_complex_det_chain(dt):
    say(f"complex det chain {dt}")
    g = gen.generator(77)
    n, W, L, K, steps = 48, 6, 96, 4, 17
    phi = gen.normal(g, (L, n), True)
    occ, emp = gen.occupancy(g, W, L, n)
    draws, u01 = draws_for(g, steps, W, n, L - n, (1, 2), 2)
    wk = Walkers(lrx.LRX_DET, DT[dt], phi, occ, emp, 2, K)
    chain = orc.DetChain(phi, occ, emp)
    wide = dt == "c128"
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=2, tol_ratio=1e-10 if wide else 1e-4,
                                         tol_inv=1e-10 if wide else 2e-3, bound_fn=det_bound_fn(phi),
                                         eps=EPS64 if wide else EPS32,
                                         growth=None if wide else (lambda t: 1.0 + t))
    say(f"  {dt}: max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
    np.testing.assert_allclose(ph, chain.phase, atol=1e-8 if dt == "c128" else 1e-3)


def test_fp32_bulk_with_fp64_refresh():
    """FP32 bulk updates, FP64 refresh every 16 steps; the error is reported and bounded."""
    say("fp32 bulk chain")
    g = gen.generator(88)
    n, W, L, K, steps = 256, 8, 512, 16, 48
    phi = gen.normal(g, (L, n))
    occ, emp = gen.occupancy(g, W, L, n)
    draws, u01 = draws_for(g, steps, W, n, L - n, (1, 2, 4), 4)
    wk = Walkers(lrx.LRX_DET, torch.float32, phi, occ, emp, 4, K, refresh_period=16)
    chain = orc.DetChain(phi, occ, emp)
    stats = []
    worst_r, worst_m, la, ph = run_chain(wk, chain, draws, u01, check_every=8, tol_ratio=1e-4, tol_inv=5e-3,
                                         stats=stats, bound_fn=det_bound_fn(phi), eps=EPS32,
                                         growth=lambda t: 1.0 + t % 16)
    say(f"  fp32: max rel err ratio {worst_r:.2e} inverse {worst_m:.2e}")
    # refresh restores FP64 log|det| (drift bounded by the refresh period)
    np.testing.assert_allclose(la, chain.logabs, atol=1e-3)


def test_singular_proposal_is_a_noop():
    """A hop that makes A exactly singular gives r = 0 (Sec. II.A); forcing accept is a no-op."""
    say("singular proposal")
    n, W = 4, 2
    L = 6
    phi = np.zeros((L, n))
    phi[:4] = np.eye(4)
    phi[4] = phi[1]              # site 4 duplicates site 1
    phi[5] = np.array([1.0, 2.0, 0.5, 0.25])
    occ = np.array([[0, 1, 2, 3]] * W, dtype=np.int32)
    emp = np.array([[4, 5]] * W, dtype=np.int32)
    wk = Walkers(lrx.LRX_DET, torch.float64, phi, occ, emp)
    before = wk.st.inv.clone()
    la0 = wk.st.logabs.clone()
    wk.set_draws(np.ones(W, np.int32), np.array([[0], [0]], np.int32), np.array([[0], [1]], np.int32))
    r = wk.propose().cpu().numpy()
    assert r[0] == 0.0                       # rows 1 and 0 of the new A are equal
    assert r[1] == pytest.approx(1.0)        # e_0 -> (1, 2, .5, .25): ratio = 1
    wk.decide(mode=lrx.LRX_MH_FORCE)
    assert wk.accept.cpu().numpy().tolist() == [0, 1]
    wk.decide(mask=np.array([1, 1]))         # force both through the update
    wk.apply()
    torch.cuda.synchronize()
    assert torch.equal(wk.st.inv[0], before[0])
    assert wk.st.logabs[0].item() == la0[0].item()
    assert wk.accept.cpu().numpy().tolist() == [0, 1]   # the skipped walker's accept is cleared
    assert wk.occ.cpu().numpy()[0, 0] == 0              # ... so its occupancy is not committed
    assert wk.occ.cpu().numpy()[1, 0] == 5


def test_bad_index_flags_walker():
    say("bad index flag")
    g = gen.generator(9)
    n, W, L = 16, 3, 32
    phi = gen.normal(g, (L, n))
    occ, emp = gen.occupancy(g, W, L, n)
    wk = Walkers(lrx.LRX_DET, torch.float64, phi, occ, emp, 1, 2)
    elec = np.array([[3], [n + 5], [1]], np.int32)      # walker 1 out of range
    wk.set_draws(np.ones(W, np.int32), elec, np.zeros((W, 1), np.int32))
    wk.propose()
    wk.decide(mode=lrx.LRX_MH_FORCE)
    acc = wk.accept.cpu().numpy()
    flags = wk.st.flags.cpu().numpy()
    assert flags[1] & lrx.LRX_FLAG_BADINDEX and acc[1] == 0
    assert flags[0] == 0 and flags[2] == 0
    wk.apply()
    wk.refresh()
    torch.cuda.synchronize()
    assert (wk.st.flags.cpu().numpy() == 0).all()      # refresh clears the flags


def test_refresh_reports_and_removes_drift():
    say("refresh drift")
    g = gen.generator(10)
    n, W, L = 64, 4, 128
    phi = gen.normal(g, (L, n))
    occ, emp = gen.occupancy(g, W, L, n)
    wk = Walkers(lrx.LRX_DET, torch.float64, phi, occ, emp)
    noise = torch.randn_like(wk.st.inv) * 1e-6
    wk.st.inv.add_(noise * wk.st.inv.abs().mean())
    wk.st.logabs.add_(0.5)
    rep = wk.refresh().cpu().numpy()
    assert np.all(rep[:, 0] > 1e-9) and np.all(rep[:, 0] < 1e-4)
    np.testing.assert_allclose(rep[:, 1], 0.5, atol=1e-9)
    _, _, inv = orc.slogdet(orc.slater_matrices(phi, occ))
    assert rel_err(wk.inverse().cpu().numpy(), inv, axis=(1, 2)).max() < 1e-11
    rep2 = wk.refresh().cpu().numpy()
    assert rep2[:, 0].max() < 1e-14 and rep2[:, 1].max() < 1e-12


class _Split:
    """The benchmark's launch shape: the walker batch cut into sub-batches with their own
    states, each driven on its own stream."""

    def __init__(self, parts, phi, occ, emp, wl):
        bounds = np.linspace(0, occ.shape[0], parts + 1).astype(int)
        self.b = list(zip(bounds[:-1], bounds[1:]))
        self.wks = [Walkers(lrx.LRX_DET, torch.float64, phi, occ[a:b], emp[a:b], wl.k_max, wl.delay, wl.refresh)
                    for a, b in self.b]
        self.streams = [torch.cuda.Stream() for _ in self.b] if parts > 1 else [None]

    def _each(self, fn):
        cur = torch.cuda.current_stream()
        out = []
        for wk, st, (a, b) in zip(self.wks, self.streams, self.b):
            if st is None:
                out.append(fn(wk, a, b))
                continue
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                out.append(fn(wk, a, b))
        for st in self.streams:
            if st is not None:
                cur.wait_stream(st)
        return out

    def propose(self, k, elec, slot):
        def f(wk, a, b):
            wk.set_draws(k[a:b], elec[a:b], slot[a:b])
            return wk.propose()
        return torch.cat(self._each(f))

    def accept_all(self):
        def f(wk, a, b):
            wk.decide(mask=np.ones(b - a, bool))
            wk.apply()
        self._each(f)

    def cat(self, fn):
        return np.concatenate([fn(wk) for wk in self.wks])


@pytest.mark.parametrize("parts", [1, 4])
def test_scale_workload_full_size_sampled(parts):
    """Phi 512x256, 1024 walkers, k in {1,2,4}, K=16, FP64 at full size, in one batch and
    in the benchmark's launch shape (four sub-batches of 256 walkers on four streams).
    Sampled walkers, among them both sides of every sub-batch boundary, are recomputed
    by the oracle."""
    wl = gen.WORKLOADS["slater_n256_k124"]
    say(f"full-size {wl.name} parts={parts}")
    phi, occ, emp, g = gen.slater_inputs(wl)
    run = _Split(parts, phi, occ, emp, wl)
    steps = 2 * wl.delay + 5
    sample = np.array([0, 1, 255, 256, 340, 511, 512, 700, 767, 768, 1022, 1023])
    book = orc.Occupancy(occ, emp)
    tally = RatioTally("full-size FP64")
    for t in range(steps):
        k, elec, slot = gen.hop_draws(g, wl.walkers, wl.n, wl.sites - wl.n, wl.ranks, wl.k_max)
        r = run.propose(k, elec, slot).cpu().numpy()
        prop = book.proposed(k, elec, slot)
        la0, ph0, inv0 = orc.slogdet(orc.slater_matrices(phi, book.occ[sample]))
        la1, ph1, _ = orc.slogdet(orc.slater_matrices(phi, prop[sample]), want_inv=False)
        ref = orc.ratio(la1, ph1, la0, ph0)
        # First-order bound per unit error of the stored inverse, which has taken t
        # updates since the last refresh (linear growth: a worst-case sum of their
        # rounding errors).
        since = t % wl.refresh
        tally.check(r[sample], ref, 1e-10,
                    lambda: det_ratio_bound(phi, book.occ[sample], prop[sample], inv0, k[sample], elec[sample]),
                    EPS64, 1.0 + since, where=f"step {t}")
        run.accept_all()
        book.commit(k, elec, slot, np.ones(wl.walkers, bool))
    np.testing.assert_array_equal(run.cat(lambda wk: wk.occ.cpu().numpy()), book.occ)
    inv = run.cat(lambda wk: wk.inverse().cpu().numpy())
    a_fin = orc.slater_matrices(phi, book.occ[sample])
    la, ph, oinv = orc.slogdet(a_fin)
    # The inverse of an ill-conditioned walker carries about sqrt(n) cond_1(A) eps relative
    # error (the oracle's own inverse too), growing at most linearly over the t updates since
    # the last refresh; where that estimate exceeds 1e-10 it is the tolerance (counted).
    tally.report()
    cond = np.linalg.norm(a_fin, 1, axis=(1, 2)) * np.linalg.norm(oinv, 1, axis=(1, 2))
    tol_inv = np.maximum(1e-10, np.sqrt(wl.n) * EPS64 * (1.0 + steps % wl.refresh) * cond)
    err_inv = rel_err(inv[sample], oinv, axis=(1, 2))
    say(f"  inverse: {int(np.sum(tol_inv > 1e-10))} of {len(sample)} sampled walkers above 1e-10 by their "
        f"condition, max rel err {err_inv.max():.2e}")
    assert np.all(err_inv <= tol_inv), (err_inv, cond)
    logabs = run.cat(lambda wk: wk.st.logabs.cpu().numpy())
    np.testing.assert_allclose(logabs[sample], la, atol=1e-8)
    assert np.isfinite(logabs).all()


def test_metropolis_modes():
    say("metropolis")
    W = 4096
    g = gen.generator(12)
    st = lrx.State(lrx.LRX_DET, torch.float64, W, 4)
    ratio = g.standard_normal(W) * 1.5
    ratio[::97] = 0.0
    ratio[5] = np.inf
    rt = torch.as_tensor(ratio).cuda()
    u = g.random(W)
    acc = torch.zeros(W, dtype=torch.uint8, device="cuda")
    lrx.lrx_metropolis(st, rt, torch.as_tensor(u).cuda(), 0, 0, lrx.LRX_MH_UNIFORMS, acc)
    np.testing.assert_array_equal(acc.cpu().numpy().astype(bool), orc.metropolis(ratio, u))
    lrx.lrx_metropolis(st, rt, None, 0, 0, lrx.LRX_MH_FORCE, acc)
    np.testing.assert_array_equal(acc.cpu().numpy().astype(bool), np.isfinite(ratio) & (ratio != 0))
    seed, ctr = 0x1234_5678_9ABC_DEF0, 77
    lrx.lrx_metropolis(st, rt, None, seed, ctr, lrx.LRX_MH_DEVICE_RNG, acc)
    uu = np.empty(W)
    for w in range(W):
        c = philox4x32_10([w, ctr & 0xFFFFFFFF, ctr >> 32, 0], (seed & 0xFFFFFFFF, seed >> 32))
        uu[w] = (((c[0] >> 5) << 26) | (c[1] >> 6)) * 2.0 ** -53
    np.testing.assert_array_equal(acc.cpu().numpy().astype(bool), orc.metropolis(ratio, uu))


@pytest.mark.parametrize("K", [0, 4])
def test_fused_hop_step_matches_oracle(K):
    """propose_hop + accept_hop (device Metropolis with the given uniforms, fused
    occupancy commit) follow the oracle's chain."""
    say(f"fused hop step K={K}")
    g = gen.generator(500 + K)
    n, W, L, steps = 40, 12, 90, 21
    phi = gen.normal(g, (L, n))
    occ, emp = gen.occupancy(g, W, L, n)
    wk = Walkers(lrx.LRX_DET, torch.float64, phi, occ, emp, 4, K)
    chain = orc.DetChain(phi, occ, emp)
    u01 = torch.zeros(W, dtype=torch.float64, device="cuda")
    tally = RatioTally("fused hop")
    for t in range(steps):
        k, elec, slot = gen.hop_draws(g, W, n, L - n, (1, 2, 4), 4)
        u = gen.uniforms(g, W)
        wk.set_draws(k, elec, slot)
        u01.copy_(torch.as_tensor(u))
        wk.step_device(mode=lrx.LRX_MH_UNIFORMS, u01=u01)
        r_gpu = wk.ratio.cpu().numpy()
        inv0, occ0 = chain.inv.copy(), chain.book.occ.copy()
        r_orc = chain.propose(k, elec, slot)
        tally.check(r_gpu, r_orc, 1e-10,
                    lambda: det_ratio_bound(phi, occ0, chain.book.proposed(k, elec, slot), inv0, k, elec),
                    EPS64, 1.0 + t, where=f"step {t}")
        mask = orc.metropolis(r_orc, u)
        np.testing.assert_array_equal(wk.accept.cpu().numpy().astype(bool), mask)
        chain.accept(k, elec, slot, mask)
    tally.report()
    np.testing.assert_array_equal(wk.occ.cpu().numpy(), chain.book.occ)
    inv = wk.inverse().cpu().numpy()
    assert rel_err(inv, chain.inv, axis=(1, 2)).max() <= 1e-10
    np.testing.assert_allclose(wk.st.logabs.cpu().numpy(), chain.logabs, atol=1e-9)
