"""Hand-written adjoint of log det (Phi[occ] + B C^T) vs the oracle and finite differences."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import assert_entries_close, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as orc  # noqa: E402
from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.adjoint import lowrank_logdet  # noqa: E402

DT = {"f64": torch.float64, "c64": torch.complex64, "c128": torch.complex128}


def make(seed, L, n, S, r, cplx, bc_var=0.1):
    g = gen.generator(seed)
    phi = gen.normal(g, (L, n), cplx)
    occ, _ = gen.occupancy(g, S, L, n)
    b = gen.normal(g, (S, n, r), cplx, bc_var)
    c = gen.normal(g, (S, n, r), cplx, bc_var)
    w = gen.normal(g, (S,), cplx)
    return phi, occ, b, c, w


def run_gpu(phi, occ, b, c, w, dt):
    cplx = np.iscomplexobj(phi)
    wide = torch.complex128 if cplx else torch.float64
    P = torch.tensor(phi, dtype=wide, device="cuda", requires_grad=True)
    B = torch.tensor(b, dtype=wide, device="cuda", requires_grad=True)
    C = torch.tensor(c, dtype=wide, device="cuda", requires_grad=True)
    occ_t = torch.as_tensor(occ, dtype=torch.int32, device="cuda")
    ld, ph = lowrank_logdet(P, B, C, occ_t, DT[dt])
    wt = torch.as_tensor(w, dtype=ld.dtype, device="cuda")
    loss = (wt * ld).real.sum()
    loss.backward()
    return ld.detach().cpu().numpy(), ph.cpu().numpy(), P.grad.cpu().numpy(), B.grad.cpu().numpy(), C.grad.cpu().numpy()


def oracle_grads(phi, occ, b, c, w):
    """Torch-convention gradients of sum Re(w_s log det M_s) from the oracle's closed forms."""
    la, ph, gm, gb, gc = orc.lowrank_logdet_and_grads(phi, occ, b, c)
    gw = np.conj(w)
    dphi = np.zeros_like(phi)
    for s in range(occ.shape[0]):
        dphi += orc.scatter_rows(gw[s] * np.conj(gm[s:s + 1]), occ[s:s + 1], phi.shape[0])
    db = gw[:, None, None] * np.conj(gb)
    dc = gw[:, None, None] * np.conj(gc)
    return la, ph, dphi, db, dc


@pytest.mark.parametrize("dt,r", [("c128", 8), ("c128", 3), ("f64", 8), ("c64", 8)])
def test_lowrank_forward_and_gradients_match_oracle(dt, r):
    say(f"adjoint {dt} r={r}")
    cplx = dt.startswith("c")
    phi, occ, b, c, w = make(700 + r, 80, 32, 6, r, cplx)
    ld, ph, dphi, db, dc = run_gpu(phi, occ, b, c, w, dt)
    la, oph, odphi, odb, odc = oracle_grads(phi, occ, b, c, w)
    tol = 1e-10 if dt in ("c128", "f64") else 2e-4
    got_la = ld.real if cplx else ld
    np.testing.assert_allclose(got_la, la, atol=tol * 32)
    np.testing.assert_allclose(ph, oph, atol=tol * 32)
    assert_entries_close(dphi, odphi, tol, "dPhi")
    assert_entries_close(db, odb, tol, "dB")
    assert_entries_close(dc, odc, tol, "dC")


def test_lowrank_gradients_finite_differences_fp64():
    """Central differences of the complex128 loss (full recompute by numpy slogdet) at n = 32."""
    say("adjoint FD")
    phi, occ, b, c, w = make(800, 64, 32, 4, 8, True)
    ld, ph, dphi, db, dc = run_gpu(phi, occ, b, c, w, "c128")

    def loss(phi_, b_, c_):
        m = phi_[occ] + b_ @ np.swapaxes(c_, -1, -2)
        sg, lg = np.linalg.slogdet(m)
        return float(np.sum((w * (lg + np.log(sg))).real))

    h = 1e-6
    for (site, col) in [(occ[0, 3], 5), (occ[2, 17], 0), (occ[3, 31], 31)]:
        for unit, part in ((1.0, "real"), (1j, "imag")):
            d = np.zeros_like(phi)
            d[site, col] = h * unit
            fd = (loss(phi + d, b, c) - loss(phi - d, b, c)) / (2 * h)
            got = dphi[site, col].real if part == "real" else dphi[site, col].imag
            assert abs(fd - got) <= 1e-6 * max(1, abs(fd)), (site, col, part, fd, got)
    for (s, i, q) in [(0, 0, 0), (1, 7, 3), (3, 31, 7)]:
        for unit, part in ((1.0, "real"), (1j, "imag")):
            d = np.zeros_like(b)
            d[s, i, q] = h * unit
            fd_b = (loss(phi, b + d, c) - loss(phi, b - d, c)) / (2 * h)
            fd_c = (loss(phi, b, c + d) - loss(phi, b, c - d)) / (2 * h)
            gb = db[s, i, q].real if part == "real" else db[s, i, q].imag
            gc = dc[s, i, q].real if part == "real" else dc[s, i, q].imag
            assert abs(fd_b - gb) <= 1e-6 * max(1, abs(fd_b))
            assert abs(fd_c - gc) <= 1e-6 * max(1, abs(fd_c))


def test_logpsi_workload_full_size_sampled():
    """Phi 1024x512 complex64, 512 samples, rank-8 B C^T: forward on sampled samples, and
    the full backward with the cotangent restricted to four samples (oracle-checkable)."""
    wl = gen.WORKLOADS["logpsi_grad_n512_c64"]
    say(f"full-size {wl.name}")
    phi, occ, b, c, w = gen.lowrank_inputs(wl)
    keep = np.array([3, 100, 257, 511])
    wsp = np.zeros_like(w)
    wsp[keep] = w[keep]
    ld, ph, dphi, db, dc = run_gpu(phi, occ, b, c, wsp, "c64")
    la, oph, odphi, odb, odc = oracle_grads(phi, occ[keep], b[keep], c[keep], wsp[keep])
    np.testing.assert_allclose(ld.real[keep], la, atol=5e-3)
    assert_entries_close(dphi, odphi, 5e-3, "dPhi")
    assert_entries_close(db[keep], odb, 5e-3, "dB")
    assert_entries_close(dc[keep], odc, 5e-3, "dC")
    others = np.setdiff1d(np.arange(wl.walkers), keep)
    assert np.abs(db[others]).max() == 0 and np.abs(dc[others]).max() == 0


# ---------------------------------------------------------------------------- from a walker state
def _walkers_after_steps(kind, dt, seed, n, L, W, K, steps, k_max=2):
    """A walker batch stepped through a few Metropolis steps (oracle-decided), ending
    mid-window in the delayed form (slot > 0); returns the walkers and the oracle chain."""
    from paper_2602_05255_amd.walkers import Walkers
    g = gen.generator(seed)
    cplx = dt.is_complex
    if kind == "det":
        table = gen.normal(g, (L, n), cplx)
        chain = orc.DetChain
        wk = Walkers(lrx.LRX_DET, dt, table, *gen.occupancy(g, W, L, n), k_max=k_max, delay=K)
        ranks = tuple(range(1, k_max + 1))
    else:
        table = gen.skew_from(gen.normal(g, (L, L), cplx))
        wk = Walkers(lrx.LRX_PF, dt, table, *gen.occupancy(g, W, L, n), k_max=1, delay=K)
        chain = orc.PfChain
        k_max, ranks = 1, (1,)
    ch = chain(table, wk.occ.cpu().numpy(), wk.empty.cpu().numpy())
    for t in range(steps):
        k, e, s = gen.hop_draws(g, W, n, L - n, ranks, k_max)
        wk.set_draws(k, e, s)
        wk.propose()
        r = ch.propose(k, e, s)
        mask = orc.metropolis(r, gen.uniforms(g, W))
        wk.decide(mask=mask)
        wk.apply()
        ch.accept(k, e, s, mask)
    torch.cuda.synchronize()
    return wk, ch, table, g


@pytest.mark.parametrize("dt", [torch.float64, torch.complex128])
def test_det_adjoint_from_delayed_walker_state(dt):
    """log det(Phi[occ] + B C^T) and dPhi, dB, dC from a walker state mid-window (delayed
    form, slot > 0, no flush) against the oracle at the walkers' current occupancy; the
    same from the flushed state; two backward passes are bitwise equal."""
    from paper_2602_05255_amd.adjoint import walker_lowrank_logdet
    say(f"det adjoint from a delayed walker state {dt}")
    n, L, W, K, r = 24, 56, 6, 5, 3
    wk, ch, phi, g = _walkers_after_steps("det", dt, 6100, n, L, W, K, steps=7)
    assert wk.st.slot == 2                     # 7 steps with K = 5: two live slots
    cplx = dt.is_complex
    b = gen.normal(g, (W, n, r), cplx, 0.1)
    c = gen.normal(g, (W, n, r), cplx, 0.1)
    w = gen.normal(g, (W,), cplx)
    occ = wk.occ.cpu().numpy()
    la, oph, odphi, odb, odc = oracle_grads(phi, occ, b, c, w)
    grads = []
    for flushed in (False, True, True):
        if flushed:
            wk.flush()
        P = torch.tensor(phi, dtype=dt, device="cuda", requires_grad=True)
        B = torch.tensor(b, dtype=dt, device="cuda", requires_grad=True)
        C = torch.tensor(c, dtype=dt, device="cuda", requires_grad=True)
        ld, ph = walker_lowrank_logdet(wk, B, C, P)
        loss = (torch.as_tensor(w, dtype=ld.dtype, device="cuda") * ld).real.sum()
        loss.backward()
        got_la = (ld.real if cplx else ld).detach().cpu().numpy()
        np.testing.assert_allclose(got_la, la, atol=1e-10 * n)
        np.testing.assert_allclose(ph.cpu().numpy(), oph, atol=1e-10 * n)
        for got, ref, nm in ((P.grad, odphi, "dPhi"), (B.grad, odb, "dB"), (C.grad, odc, "dC")):
            e = assert_entries_close(got.cpu().numpy(), ref, 1e-10, nm)
            say(f"  slot {wk.st.slot}: {nm} max entry error {e:.2e}")
        grads.append((P.grad.clone(), B.grad.clone(), C.grad.clone()))
    for x, y in zip(grads[1], grads[2]):
        assert torch.equal(x, y), "the backward is not bitwise reproducible"


@pytest.mark.parametrize("dt,r,delayed", [(torch.complex128, 2, False), (torch.complex128, 4, True),
                                          (torch.float64, 2, True), (torch.complex64, 2, False)])
def test_pf_lowrank_adjoint_matches_oracle(dt, r, delayed):
    """log pf(F[occ][:, occ] - U J U^T) and dF, dU from a Pfaffian walker state (flushed,
    or mid-window in the delayed form) against the oracle's full recompute."""
    from paper_2602_05255_amd.adjoint import walker_lowrank_logpf
    say(f"pf low-rank adjoint {dt} r={r} delayed={delayed}")
    n, L, W = 16, 36, 5
    wk, ch, f, g = _walkers_after_steps("pf", dt, 6200 + r, n, L, W, K=4 if delayed else 0,
                                        steps=6 if delayed else 3)
    if delayed:
        assert wk.st.slot == 2
    cplx = dt.is_complex
    u = gen.normal(g, (W, n, r), cplx, 0.2)
    w = gen.normal(g, (W,), cplx)
    occ = wk.occ.cpu().numpy()
    la, oph, gm, gu = orc.lowrank_logpf_and_grads(f, occ, u)
    gw = np.conj(w)
    odf = sum(orc.scatter_pairs(gw[s] * np.conj(gm[s:s + 1]), occ[s:s + 1], L) for s in range(W))
    odu = gw[:, None, None] * np.conj(gu)
    F = torch.tensor(f, dtype=dt, device="cuda", requires_grad=True)
    U = torch.tensor(u, dtype=dt, device="cuda", requires_grad=True)
    lp, ph = walker_lowrank_logpf(wk, U, F)
    loss = (torch.as_tensor(w, dtype=lp.dtype, device="cuda") * lp).real.sum()
    loss.backward()
    tol = 1e-10 if dt != torch.complex64 else 2e-4
    got_la = (lp.real if cplx else lp).detach().cpu().numpy()
    np.testing.assert_allclose(got_la, la, atol=tol * n)
    np.testing.assert_allclose(ph.cpu().numpy(), oph, atol=tol * n)
    e1 = assert_entries_close(U.grad.cpu().numpy(), odu, tol, "dU")
    e2 = assert_entries_close(F.grad.cpu().numpy(), odf, tol, "dF")
    say(f"  dU max entry error {e1:.2e}, dF {e2:.2e}")


def test_pf_lowrank_gradients_finite_differences():
    """Central differences of the GPU forward itself (complex128, fresh state per
    evaluation) against the GPU backward, for entries of U and skew directions of F."""
    from paper_2602_05255_amd.adjoint import lowrank_logpf
    say("pf low-rank FD")
    g = gen.generator(6300)
    n, L, W, r = 12, 30, 3, 4
    f = gen.skew_from(gen.normal(g, (L, L), True))
    occ_np, _ = gen.occupancy(g, W, L, n)
    occ = torch.as_tensor(occ_np, dtype=torch.int32, device="cuda")
    u = gen.normal(g, (W, n, r), True, 0.3)
    w = gen.normal(g, (W,), True)
    wt = torch.as_tensor(w, device="cuda")

    def loss(f_, u_, grad=False):
        F = torch.tensor(f_, dtype=torch.complex128, device="cuda", requires_grad=grad)
        U = torch.tensor(u_, dtype=torch.complex128, device="cuda", requires_grad=grad)
        lp, _ = lowrank_logpf(F, U, occ)
        val = (wt * lp).real.sum()
        if grad:
            val.backward()
            return F.grad.cpu().numpy(), U.grad.cpu().numpy()
        return float(val)

    dF, dU = loss(f, u, grad=True)
    h = 1e-6
    for (s, i, q) in [(0, 0, 0), (1, 5, 3), (2, 11, 1)]:
        for unit, part in ((1.0, "real"), (1j, "imag")):
            d = np.zeros_like(u)
            d[s, i, q] = h * unit
            fd = (loss(f, u + d) - loss(f, u - d)) / (2 * h)
            got = dU[s, i, q].real if part == "real" else dU[s, i, q].imag
            assert abs(fd - got) <= 1e-6 * max(1, abs(fd)), (s, i, q, part, fd, got)
    for (a, b) in [(occ_np[0, 1], occ_np[0, 7]), (occ_np[2, 0], occ_np[1, 3])]:
        for unit, part in ((1.0, "real"), (1j, "imag")):
            d = np.zeros_like(f)
            d[a, b] = h * unit
            d[b, a] = -h * unit
            fd = (loss(f + d, u) - loss(f - d, u)) / (2 * h)
            gab = dF[a, b] - dF[b, a]
            got = gab.real if part == "real" else gab.imag
            assert abs(fd - got) <= 1e-6 * max(1, abs(fd)), (a, b, part, fd, got)


@pytest.mark.parametrize("dt,n", [(torch.complex128, 10), (torch.float64, 64), (torch.complex128, 130),
                                  (torch.complex64, 40)])
def test_batched_pf_ops_match_oracle(dt, n):
    """The stand-alone batched logpf / slogpf / pf of dense skew matrices (Parlett-Reid)
    against the oracle, and the gradient of log pf against (1/2) A^-T (Appendix A, Eq.
    pf_grad, pinned by finite differences on the CPU), entry by entry."""
    from paper_2602_05255_amd.adjoint import logpf, pf, slogpf
    say(f"batched pf ops {dt} n={n}")
    g = gen.generator(6400 + n)
    cplx = dt.is_complex
    W = 5
    a = np.stack([gen.skew_from(gen.normal(g, (n, n), cplx)) for _ in range(W)])
    la, ph = orc.slogpf(a)
    A = torch.tensor(a, dtype=dt, device="cuda", requires_grad=True)
    lp = logpf(A)
    tol = 1e-10 if dt != torch.complex64 else 2e-4
    got = lp.detach().cpu().numpy()
    np.testing.assert_allclose(got.real if cplx else got, la, atol=tol * n)
    phase, labs = slogpf(A.detach())
    np.testing.assert_allclose(phase.cpu().numpy(), ph, atol=tol * n)
    np.testing.assert_allclose(labs.cpu().numpy(), la, atol=tol * n)
    if n <= 64:
        np.testing.assert_allclose(pf(A.detach()).cpu().numpy(), ph * np.exp(la), rtol=tol * n)
    w = gen.normal(g, (W,), cplx)
    loss = (torch.as_tensor(w, dtype=lp.dtype, device="cuda") * lp).real.sum()
    loss.backward()
    inv = orc.skew_inverse(a)
    want = np.conj(w)[:, None, None] * np.conj(0.5 * np.swapaxes(inv, 1, 2))
    e = assert_entries_close(A.grad.cpu().numpy(), want, tol, "dA")
    say(f"  d log pf / dA max entry error {e:.2e}")
