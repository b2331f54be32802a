#!/usr/bin/env python3
"""Benchmark: walker-steps/s of batched low-rank determinant updates on one MI355X.

Default workload (the paper-shaped scale configuration): orbital matrix Phi
512 x 256 iid N(0,1), 1024 walkers, each step moves k ~ U{1,2,4} electrons to
empty sites, delayed updates with K = 16 flushed by an MFMA GEMM, FP64 refresh
every 128 steps.  One benchmark "step" is one refresh period: 128 Markov-chain
steps of every walker (build hop -> ratio -> accept -> delayed update, 8
flushes) plus the FP64 refresh, replayed as one HIP graph.  Mode: forced
accept (every proposal is applied, a deterministic byte count).

The JSON line also carries: the dominant kernel's roofline (HIP events around
the delayed accept kernel), the oracle on the host cores (cpu_baseline), full
recompute on the same GPU (rocSOLVER via torch.linalg.slogdet), the FP32-bulk
variant, and the measured relative error of the LRU state against an FP64 full
recompute on the same GPU.  Only the cpu_baseline leg runs the oracle.
"""
from __future__ import annotations

import argparse
import contextlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "walker-steps/s det & pf LRU vs full recompute, same GPU, at stated rel. error"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3


def counter_traffic(profile, sources, walkers_per_launch):
    """HBM bytes per launch measured by the FETCH_SIZE / WRITE_SIZE counter passes
    recorded in profiles/<profile>, or None when the kernel sources changed since or the
    launch size differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    keys = {}
    for line in open(path):
        part = line.strip().split(":", 1)
        if len(part) == 2:
            keys[part[0].strip()] = part[1].strip()
    if keys.get("source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in keys:
        return None
    if keys.get("walkers_per_launch") != str(int(walkers_per_launch)):
        return None
    return float(keys["traffic_bytes_per_launch"])


DET_SOURCES = ["paper_2602_05255_amd/csrc/lrx_common.hpp", "paper_2602_05255_amd/csrc/lrx_internal.hpp",
               "paper_2602_05255_amd/csrc/lrx_det_impl.hpp", "paper_2602_05255_amd/csrc/lrx_det.hip",
               "include/lrx.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed refresh periods")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="slater_n256_k124")
    ap.add_argument("--walkers", type=int, default=0, help="override the walker count")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-recompute", action="store_true")
    ap.add_argument("--streams", type=int, default=None,
                    help="independent sub-batches of the walker batch, one HIP stream each (1 = one launch "
                         "per step); default 4 for the determinant and Pfaffian workloads, 1 for the n-sweep")
    ap.add_argument("--sizes", default=None, help="n-sweep sizes, comma separated (default 64,...,1024)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    return ap.parse_args()


class Run:
    """One walker batch with its pre-generated draws, stepping one refresh period at a time.

    With streams > 1 the batch is split into that many independent sub-batches (their own
    states), each driven on its own HIP stream (default priority) and forked from / joined to
    the calling stream every period: one sub-batch's latency-bound launches (propose, flush,
    refresh blocks) then run beside another's bandwidth-bound accept.  The walkers and their
    arithmetic are the same as with one stream."""

    def __init__(self, wl, dtype, walkers, seed_offset=0, streams=1):
        import torch
        from paper_2602_05255_amd import inputs as gen
        from paper_2602_05255_amd import lrx
        from paper_2602_05255_amd.walkers import Walkers
        self.torch, self.lrx = torch, lrx
        self.wl = wl
        if wl.kind == "det":
            phi, occ, emp, g = gen.slater_inputs(wl, walkers=walkers, seed_offset=seed_offset)
        else:
            phi, occ, emp, g = gen.pairing_inputs(wl, walkers=walkers, seed_offset=seed_offset)
        self.phi = phi
        self.W = walkers
        self.P = wl.refresh
        t0 = time.time()
        k, e, s = gen.hop_draws_batch(g, self.P, walkers, wl.n, wl.sites - wl.n, wl.ranks, wl.k_max)
        log(f"  draws {self.P} x {walkers}: {time.time() - t0:.1f}s")
        dev = torch.device("cuda")
        self.k = torch.as_tensor(k).to(dev)
        self.e = torch.as_tensor(e).to(dev)
        self.s = torch.as_tensor(s).to(dev)
        kind = lrx.LRX_DET if wl.kind == "det" else lrx.LRX_PF
        bounds = np.linspace(0, walkers, max(1, streams) + 1).astype(int)
        self.parts = []
        for a0, a1 in zip(bounds[:-1], bounds[1:]):
            wk = Walkers(kind, dtype, phi, occ[a0:a1], emp[a0:a1], wl.k_max, wl.delay, refresh_period=0)
            self.parts.append((wk, int(a0), int(a1), torch.cuda.Stream() if streams > 1 else None))
        self.wk = self.parts[0][0]
        self.graph = None
        # Sub-batch p runs offsets[p] steps ahead (a multiple of K), so the sub-batches reach
        # their refresh at different steps and each refresh overlaps the others' steps.
        K = max(1, wl.delay)
        self.offsets = [(p * (self.P // len(self.parts))) // K * K for p in range(len(self.parts))]
        self.primed = False

    @property
    def occ(self):
        return self.torch.cat([wk.occ for wk, _, _, _ in self.parts])

    def _step(self, wk, a0, a1, t, timer):
        lrx = self.lrx
        k, e, s = self.k[t, a0:a1], self.e[t, a0:a1], self.s[t, a0:a1]
        if timer is not None:
            timer.begin("propose", wk.st.slot)
        if wk.kind == lrx.LRX_DET:
            lrx.lrx_det_propose_hop(wk.st, wk.table, wk.sites, wk.occ, wk.empty, wk.n_empty, k, e, s, wk.u,
                                    wk.ratio)
        else:
            lrx.lrx_pf_propose_hop(wk.st, wk.table, wk.sites, wk.occ, wk.empty, wk.n_empty, k, e, s, wk.u,
                                   wk.ratio)
        if timer is not None:
            timer.end("propose")
            timer.begin("accept", wk.st.slot, wk.W)
        if wk.kind == lrx.LRX_DET:
            lrx.lrx_det_accept_hop(wk.st, k, e, s, wk.u, lrx.LRX_MH_FORCE, None, 0, t, wk.accept, wk.occ,
                                   wk.empty, wk.n_empty)
        else:
            lrx.lrx_pf_accept_hop(wk.st, k, e, s, wk.u, lrx.LRX_MH_FORCE, None, 0, t, wk.accept, wk.occ,
                                  wk.empty, wk.n_empty)
        if timer is not None:
            timer.end("accept")
        if wk.delay and wk.st.slot == wk.delay:
            if timer is not None:
                timer.begin("flush", wk.st.slot)
            wk.flush()
            if timer is not None:
                timer.end("flush")

    def prime(self):
        """Advance every sub-batch by its offset (once, before the first period)."""
        if self.primed:
            return
        for (wk, a0, a1, _), off in zip(self.parts, self.offsets):
            for t in range(off):
                self._step(wk, a0, a1, t, None)
        self.torch.cuda.synchronize()
        self.primed = True

    def period(self, timer=None):
        """One refresh period: P steps of every sub-batch with forced accept, flushes every
        K, and each sub-batch's refresh after its own P-th step.  With a timer every launch
        runs on the calling stream (one at a time, so that each launch's own duration is
        measured); otherwise the sub-batches run on their streams."""
        torch = self.torch
        self.prime()
        split = timer is None and len(self.parts) > 1
        cur = torch.cuda.current_stream()
        if split:
            for _, _, _, st in self.parts:
                st.wait_stream(cur)
        for t in range(self.P):
            for (wk, a0, a1, st), off in zip(self.parts, self.offsets):
                local = (t + off) % self.P
                with torch.cuda.stream(st) if split else contextlib.nullcontext():
                    self._step(wk, a0, a1, local, None if split else timer)
                    if local == self.P - 1:
                        if timer is not None:
                            timer.begin("refresh", 0)
                        wk.refresh(report=False)
                        if timer is not None:
                            timer.end("refresh")
        if split:
            for _, _, _, st in self.parts:
                cur.wait_stream(st)

    def capture(self):
        torch = self.torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.period()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.period()
        torch.cuda.synchronize()
        self.graph = g

    def step(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self.period()


class EventTimer:
    """HIP events around selected launches on the current stream."""

    def __init__(self, torch):
        self.torch = torch
        self.rec = []
        self.cur = {}

    def begin(self, name, tau, walkers=0):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        self.cur[name] = (ev, tau, walkers)

    def end(self, name):
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record()
        b, tau, walkers = self.cur.pop(name)
        self.rec.append((name, tau, walkers, b, ev))

    def results(self):
        self.torch.cuda.synchronize()
        out = {}
        for name, tau, walkers, b, e in self.rec:
            out.setdefault(name, []).append((tau, b.elapsed_time(e) * 1e-3, walkers))
        return out


def accept_bytes(wl, s, W, tau):
    """Algorithmic HBM bytes of one delayed accept launch (all walkers accepted).
    DET: read A_0^-1 (n^2), the tau live b-slot rows (n k_max tau), u and C
    (2 n k_max); write slot tau of a and b (2 n k_max).
    PF: read A_0^-1 (n^2), x, col and the 2 tau a-slot columns; write the two
    new a-slot columns."""
    n, km = wl.n, wl.k_max
    if wl.kind == "pf":
        return W * s * (n * n + 2 * n * tau + 4 * n)
    return W * s * (n * n + n * km * tau + 4 * n * km)


def queue_filler(torch, ms=150.0):
    """About `ms` of GPU work (FP64 GEMMs) on the current stream, enqueued at once."""
    a = torch.ones(4096, 4096, dtype=torch.float64, device="cuda") / 4096.0
    reps = max(1, int(ms / 3.0))             # one 4096^3 FP64 GEMM is about 3 ms here or more
    for _ in range(reps):
        a = a @ a


def measure(wl, dtype, walkers, args, torch, label):
    run = Run(wl, dtype, walkers, streams=args.streams)
    elem = torch.empty((), dtype=dtype).element_size()
    wl_launch = walkers / len(run.parts)      # walkers per launch (one sub-batch)
    # roofline pass: eager, HIP events around every accept launch of one period.  A filler
    # (FP64 GEMMs) keeps the GPU busy while the host enqueues the period, so that no event
    # pair brackets host launch time.
    run.period()
    torch.cuda.synchronize()
    queue_filler(torch)
    timer = EventTimer(torch)
    run.period(timer)
    res = timer.results()
    acc = res["accept"]
    bytes_tot = sum(accept_bytes(wl, elem, wp, tau) for tau, _, wp in acc)
    t_tot = sum(dt for _, dt, _ in acc)
    fl = res.get("flush", [])
    flush_t = np.mean([dt for _, dt, _ in fl]) if fl else None
    refresh_t = np.mean([dt for _, dt, _ in res["refresh"]])
    if not args.no_graph:
        run.capture()
    for _ in range(args.warmup):
        run.step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        run.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu = e0.elapsed_time(e1) * 1e-3
    T = max(wall, gpu)
    value = walkers * run.P * args.steps / T
    # flush roofline: algorithmic flops per walker 2 n^2 K k_max (DET, real), 8 n^2 2K / 2
    # (PF complex, upper half); bytes RW of M0 + the slot panels
    n, K, km = wl.n, wl.delay, wl.k_max
    flush = None
    if flush_t:
        if wl.kind == "pf":
            fflops = wl_launch * 8.0 * n * n * 2 * K / 2
            fbytes = wl_launch * elem * (1.5 * n * n + 2 * n * K)
            elem_peak = FP32_PEAK_TFS if elem <= 8 else FP64_PEAK_TFS
        else:
            kbar = float(np.mean(wl.ranks))    # live slot columns per step (padding is skipped)
            fflops = wl_launch * 2.0 * n * n * K * kbar * (4 if elem == 16 else 1)
            fbytes = wl_launch * elem * (2 * n * n + 2 * n * K * kbar)
            elem_peak = FP64_PEAK_TFS if elem == 8 else FP32_PEAK_TFS
        flush = {"avg_us": flush_t * 1e6, "tflops": fflops / flush_t / 1e12,
                 "gbs": fbytes / flush_t / 1e9,
                 "mfma_frac": fflops / flush_t / 1e12 / elem_peak,
                 "hbm_frac": fbytes / flush_t / 1e9 / HBM_PEAK_GBS}
    log(f"  [{label}] {value:.4g} walker-steps/s, {T / args.steps * 1e3:.3f} ms per period; accept "
        f"{t_tot / len(acc) * 1e6:.1f} us avg, {bytes_tot / t_tot / 1e9:.0f} GB/s; refresh {refresh_t * 1e3:.2f} ms")
    return run, {
        "value": value, "ms_per_step": T / args.steps * 1e3,
        "accept_avg_us": t_tot / len(acc) * 1e6, "accept_gbs": bytes_tot / t_tot / 1e9,
        "accept_bytes_per_launch": bytes_tot / len(acc),
        "refresh_ms": refresh_t * 1e3, "flush": flush,
    }


def rel_error(run, torch, sample):
    """Max relative error of the LRU inverse and log|det| (log|pf|) on sampled walkers against the
    full FP64 / complex128 recompute on the same GPU (torch.linalg: rocSOLVER LU).  For the
    Pfaffian, log|pf| = log|det| / 2 (the phase is checked against the oracle by the tests)."""
    wk = run.wk                      # the first sub-batch; sample spread over its walkers
    sample = np.linspace(0, wk.W - 1, len(sample)).astype(int)
    idx = torch.as_tensor(sample, device=wk.occ.device)
    inv = wk.inverse()[idx]
    occ = wk.occ[idx].long()
    wide = torch.complex128 if run.wl.complex_ else torch.float64
    src = torch.as_tensor(run.phi).to(device=inv.device, dtype=wide)
    if run.wl.kind == "pf":
        a = src[occ[:, :, None], occ[:, None, :]]
        _, la = torch.linalg.slogdet(a)
        la = 0.5 * la
        rinv = torch.linalg.inv(a)
        rinv = 0.5 * (rinv - rinv.transpose(1, 2))
    else:
        a = src[occ]
        _, la = torch.linalg.slogdet(a)
        rinv = torch.linalg.inv(a)
    e_inv = torch.linalg.matrix_norm(inv.to(wide) - rinv) / torch.linalg.matrix_norm(rinv)
    e_la = (wk.st.logabs[idx] - la).abs()
    return {"inverse_max": float(e_inv.max()), "logdet_abs_max": float(e_la.max()), "walkers": len(sample),
            "against": "FP64 full recompute on the same GPU (torch.linalg)"}


def cpu_baseline(wl, seconds):
    """The oracle (full recompute: LU + inverse per walker-step) on the host cores."""
    import oracle as orc
    from paper_2602_05255_amd import inputs as gen
    orc.build(force=False)
    W = 64
    phi, occ, emp, g = gen.slater_inputs(wl, walkers=W, seed_offset=7)
    chain = orc.DetChain(phi, occ, emp)
    done, t0 = 0, time.perf_counter()
    while True:
        k, e, s = gen.hop_draws(g, W, wl.n, wl.sites - wl.n, wl.ranks, wl.k_max)
        chain.propose(k, e, s)
        chain.accept(k, e, s, np.ones(W, bool))
        done += W
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": done / el, "unit": "walker-steps/s", "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{W} walkers x {done // W} steps of the {wl.name} workload (n={wl.n}), "
                      f"full FP64 LU + inverse per walker-step, {el:.1f}s"}


def recompute(wl, run, torch, reps=5):
    """Full recompute on the same GPU: gather Phi[occ] + torch.linalg.slogdet (rocSOLVER), FP64."""
    phi = torch.as_tensor(run.phi).cuda()
    occ = run.occ.long()
    out = {}
    chunk = 128     # batched getrf on the whole 1024-matrix batch fails to allocate its workspace
    for name, fn in (("slogdet", lambda a: torch.linalg.slogdet(a)),
                     ("slogdet+inv", lambda a: (torch.linalg.slogdet(a), torch.linalg.inv(a)))):
        def batch():
            for c0 in range(0, run.W, chunk):
                fn(phi[occ[c0:c0 + chunk]])
        try:
            batch()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                batch()
            torch.cuda.synchronize()
        except RuntimeError as exc:        # report, do not fail the benchmark line
            out[name] = {"error": str(exc).splitlines()[0]}
            continue
        dt = (time.perf_counter() - t0) / reps
        n = wl.n
        flops = run.W * (2 * n ** 3 / 3 + (2 * n ** 3 if "inv" in name else 0))
        out[name] = {"walker_steps_per_s": run.W / dt, "ms_per_batch": dt * 1e3, "tflops": flops / dt / 1e12}
    return out


def bench_secondary(wl, args, torch, dtype):
    """A secondary workload (e.g. the Pfaffian one): same timing, no CPU/recompute legs."""
    W = args.walkers or wl.walkers
    log(f"workload {wl.name}: W={W} n={wl.n} L={wl.sites} K={wl.delay} refresh={wl.refresh}")
    run, r = measure(wl, dtype, W, args, torch, str(dtype).replace("torch.", ""))
    err = rel_error(run, torch, np.linspace(0, W - 1, 4).astype(int))
    log(f"  error vs full recompute: {err}")
    return {"metric": METRIC, "value": r["value"], "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": str(dtype).replace("torch.", ""), "data": "synthetic",
            "config": {"workload": wl.name, "walkers": W, "n": wl.n, "sites": wl.sites, "delay": wl.delay,
                       "refresh_every": wl.refresh, "mode": "forced-accept",
                       "streams": args.streams},
            "accept_avg_us": r["accept_avg_us"], "accept_gbs": r["accept_gbs"], "refresh_ms": r["refresh_ms"],
            "flush": r["flush"], "rel_error": err}


def bench_adjoint(wl, args, torch):
    """Forward + hand-written backward of log det(Phi[occ] + B C^T) for all samples."""
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd.adjoint import lowrank_logdet
    phi, occ, b, c, w = gen.lowrank_inputs(wl)
    dev = "cuda"
    P = torch.tensor(phi, dtype=torch.complex128, device=dev, requires_grad=True)
    B = torch.tensor(b, dtype=torch.complex64, device=dev, requires_grad=True)
    C = torch.tensor(c, dtype=torch.complex64, device=dev, requires_grad=True)
    occ_t = torch.as_tensor(occ, dtype=torch.int32, device=dev)
    wt = torch.as_tensor(w, dtype=torch.complex128, device=dev)

    def one():
        ld, _ = lowrank_logdet(P, B, C, occ_t, torch.complex64)
        loss = (wt * ld).real.sum()
        loss.backward()
        return loss

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    S, n = occ.shape
    return {"metric": "samples/s (log det + hand-written backward)", "value": S / dt, "unit": "samples/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
            "data": "synthetic", "config": {"workload": wl.name, "samples": S, "n": n, "sites": phi.shape[0],
                                            "rank": b.shape[-1]},
            "note": "includes the complex128 factorisation of every A_s = Phi[occ_s] (init) in each step"}


def bench_uneven(wl, args, torch):
    """Uneven batch: every size class advanced by one persistent launch per window
    of K steps; one benchmark step is one refresh period (P / K windows, then the
    FP64 refresh of every class)."""
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd import lrx
    from paper_2602_05255_amd.uneven import UnevenWalkers
    classes, g = gen.uneven_inputs(wl, walkers=args.walkers or None)
    K, P = wl.delay, wl.refresh
    nwin = P // K
    t0 = time.time()
    from paper_2602_05255_amd import autotune
    log(f"  autotune cache {autotune.cache_path()}")
    uw = UnevenWalkers(torch.float32, classes, wl.k_max, "auto", K, ranks=wl.ranks)
    gt = gen.generator(gen.SEED_BASE + 11)    # draws for the grid search only
    uw.set_draws([gen.hop_draws_batch(gt, K, p.st.walkers, c["n"], c["n"], wl.ranks, wl.k_max)
                  for c, p in zip(classes, uw.parts)])
    autotune.tune_grid(uw)
    big = []
    for c, p in zip(classes, uw.parts):
        k, e, s = gen.hop_draws_batch(g, P, len(c["walkers"]), c["n"], c["n"], wl.ranks, wl.k_max)
        big.append(tuple(torch.as_tensor(x).cuda() for x in (k, e, s)))
    log(f"  setup {time.time() - t0:.1f}s; classes " +
        ", ".join(f"n={p.st.n}:W={p.st.walkers}:K={p.st.delay}" for p in uw.parts) + f"; grid {uw.grid}")

    def window(i):
        for p, (k, e, s) in zip(uw.parts, big):
            p.k, p.elec, p.slot = k[i * K:(i + 1) * K], e[i * K:(i + 1) * K], s[i * K:(i + 1) * K]
        lrx.lrx_det_window(uw.parts, K, lrx.LRX_MH_FORCE, 0, i * K, uw.order, uw.queue, uw.grid)

    def period():
        for i in range(nwin):
            window(i)
        uw.refresh(report=False)

    # eager pass with events around every window launch and the refresh
    period()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nwin + 2)]
    ev[0].record()
    for i in range(nwin):
        window(i)
        ev[i + 1].record()
    uw.refresh(report=False)
    ev[-1].record()
    torch.cuda.synchronize()
    win_s = [ev[i].elapsed_time(ev[i + 1]) * 1e-3 for i in range(nwin)]
    refresh_s = ev[nwin].elapsed_time(ev[-1]) * 1e-3
    graph = None
    if not args.no_graph:
        s_ = torch.cuda.Stream()
        s_.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_):
            period()
        torch.cuda.current_stream().wait_stream(s_)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            period()
        torch.cuda.synchronize()
    step = graph.replay if graph is not None else period
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    T = max(time.perf_counter() - t0, e0.elapsed_time(e1) * 1e-3)
    W = uw.walkers
    value = W * P * args.steps / T
    # algorithmic bytes of one window (all proposals applied): per walker and step
    # read A_0^-1 (n^2) and the live b-slot rows (n kbar tau), u and C (2 n kbar),
    # write the new slot (2 n kbar); per walker and flush the flush reads and
    # writes A_0^-1 and reads the Kc kbar live slot columns of a and b.
    kbar = float(np.mean(wl.ranks))
    es = 4
    wbytes = 0.0
    for p in uw.parts:      # each class with its own (autotuned) delay Kc, flushed K / Kc times per window
        n, Kc = p.st.n, p.st.delay
        per_step = n * n + n * kbar * (Kc - 1) / 2.0 + 4 * n * kbar
        wbytes += p.st.walkers * es * (K * per_step + (K / Kc) * (2 * n * n + 2 * n * Kc * kbar))
    win = float(np.mean(win_s))
    log(f"  [uneven f32] {value:.4g} walker-steps/s, {T / args.steps * 1e3:.2f} ms per period; window "
        f"{win * 1e3:.3f} ms ({wbytes / win / 1e9:.0f} GB/s algorithmic); refresh {refresh_s * 1e3:.1f} ms")
    return {"metric": METRIC, "value": value, "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": T / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "walkers": W, "sizes": list(wl.extra["sizes"]),
                       "class_walkers": {int(p.st.n): int(p.st.walkers) for p in uw.parts},
                       "ranks": list(wl.ranks), "window_steps": K, "refresh_every": P, "mode": "forced-accept",
                       "delay_per_class": {int(p.st.n): int(p.st.delay) for p in uw.parts},
                       "delay_and_grid": "autotuned", "graph": graph is not None, "grid": uw.grid},
            "roofline": {"bound": "hbm", "kernel": "det_window_kernel", "achieved": wbytes / win / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": wbytes / win / 1e9 / HBM_PEAK_GBS,
                         "traffic": None, "avg_us": win * 1e6, "bytes_per_launch": wbytes},
            "refresh_ms": refresh_s * 1e3}


def bench_nsweep(wl, args, torch):
    """Single-hop determinant LRU against full recompute on the same GPU, n = 64 .. 1024
    (the shape of the paper's speedup-vs-n figure).  Per n: the delayed LRU (K near the
    byte-model optimum, forced accept, FP64 refresh every 128 steps amortised) in FP64 and
    FP32 bulk, and torch.linalg.slogdet of the gathered Phi[occ] (rocSOLVER LU) in FP64."""
    from paper_2602_05255_amd import inputs as gen
    sizes = [int(x) for x in args.sizes.split(",")] if args.sizes else list(wl.extra["sizes"])
    W = args.walkers or wl.walkers
    rows = []
    for n in sizes:
        wn = gen.nsweep_workload(n)
        log(f"n-sweep n={n}: W={W} L={wn.sites} K={wn.delay} refresh={wn.refresh}")
        run64, r64 = measure(wn, torch.float64, W, args, torch, f"f64 n={n}")
        err64 = rel_error(run64, torch, np.linspace(0, W - 1, 4).astype(int))
        rc = recompute(wn, run64, torch, reps=3)
        del run64
        torch.cuda.empty_cache()
        row = {"n": n, "delay": wn.delay,
               "lru_f64": r64["value"], "accept_gbs_f64": r64["accept_gbs"],
               "accept_hbm_frac_f64": r64["accept_gbs"] / HBM_PEAK_GBS, "refresh_ms": r64["refresh_ms"],
               "rel_error_f64": err64, "recompute": rc}
        if not args.no_fp32:
            run32, r32 = measure(wn, torch.float32, W, args, torch, f"f32 n={n}")
            row["lru_f32"] = r32["value"]
            row["accept_gbs_f32"] = r32["accept_gbs"]
            del run32
            torch.cuda.empty_cache()
        # this library's own full recompute: the FP64 refresh (gather, Gauss-Jordan inverse
        # and log|det| of every walker), timed inside the LRU run
        own = W / (r64["refresh_ms"] * 1e-3)
        row["recompute_own_gj"] = {"walker_steps_per_s": own, "what": "slogdet + inverse, FP64 Gauss-Jordan refresh"}
        row["speedup_f64_vs_own_gj"] = r64["value"] / own
        if "lru_f32" in row:
            row["speedup_f32_bulk_vs_own_gj"] = row["lru_f32"] / own
        rs = rc.get("slogdet", {}).get("walker_steps_per_s")
        if rs:
            row["speedup_f64"] = r64["value"] / rs
            row["recompute_tflops"] = rc["slogdet"]["tflops"]
            row["recompute_fp64_frac"] = rc["slogdet"]["tflops"] / FP64_PEAK_TFS
            if "lru_f32" in row:
                row["speedup_f32_bulk"] = row["lru_f32"] / rs
        log(f"  n={n}: LRU f64 {r64['value']:.4g}/s, recompute rocSOLVER {rs if rs else float('nan'):.4g}/s "
            f"(speedup {row.get('speedup_f64', float('nan')):.1f}x, f32 bulk {row.get('speedup_f32_bulk', float('nan')):.1f}x), "
            f"own GJ {own:.4g}/s (speedup {row['speedup_f64_vs_own_gj']:.1f}x, "
            f"f32 bulk {row.get('speedup_f32_bulk_vs_own_gj', float('nan')):.1f}x)")
        rows.append(row)
    top = rows[-1]
    return {"metric": METRIC, "value": top["lru_f64"], "unit": "walker-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": wl.name, "walkers": W, "sizes": sizes, "ranks": [1],
                       "delay_per_n": {str(r["n"]): r["delay"] for r in rows}, "refresh_every": wl.refresh,
                       "mode": "forced-accept"},
            "speedup_vs_recompute_at_largest_n": top.get("speedup_f64"),
            "speedup_vs_own_gj_recompute_at_largest_n": top.get("speedup_f64_vs_own_gj"), "sweep": rows}


def copy_calibration(torch, nbytes=1 << 30, reps=5):
    """A plain device copy of nbytes (read nbytes, write nbytes): the reference
    that scales the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    return {"copy_bytes": nbytes, "reps": reps + 1, "us": dt * 1e6, "gbs_read_plus_write": 2 * nbytes / dt / 1e9}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): walkers are independent chains, "
              "so the path shards by walker with no exchange; multi-GPU runs are not part of this build.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd import lrx  # noqa: F401  (fails loudly without liblrx.so)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        print(json.dumps(copy_calibration(torch)), flush=True)
        return
    wl = gen.WORKLOADS[args.workload]
    if args.streams is None:
        args.streams = {"slater_n256_k124": 4, "pfaffian_n512_c64": 4}.get(wl.name, 1)
    if wl.name == "logpsi_grad_n512_c64":
        print(json.dumps(bench_adjoint(wl, args, torch)), flush=True)
        return
    if wl.kind == "pf":
        print(json.dumps(bench_secondary(wl, args, torch, torch.complex64)), flush=True)
        return
    if wl.name == "uneven_n64_1024_fp32":
        print(json.dumps(bench_uneven(wl, args, torch)), flush=True)
        return
    if wl.name == "nsweep_det_k1":
        print(json.dumps(bench_nsweep(wl, args, torch)), flush=True)
        return
    assert wl.kind == "det" and wl.n > 0, "the default benchmark drives a uniform-n determinant workload"
    W = args.walkers or wl.walkers
    log(f"workload {wl.name}: W={W} n={wl.n} L={wl.sites} ranks={wl.ranks} K={wl.delay} refresh={wl.refresh}")

    run64, r64 = measure(wl, torch.float64, W, args, torch, "f64")
    sample = np.linspace(0, W - 1, 8).astype(int)
    err64 = rel_error(run64, torch, sample)
    log(f"  f64 error vs full recompute: {err64}")
    rc = None if args.no_recompute else recompute(wl, run64, torch)
    del run64
    torch.cuda.empty_cache()
    fp32 = None
    if not args.no_fp32:
        run32, r32 = measure(wl, torch.float32, W, args, torch, "f32")
        err32 = rel_error(run32, torch, sample)
        log(f"  f32 error vs full recompute: {err32}")
        fp32 = {"value": r32["value"], "ms_per_step": r32["ms_per_step"], "rel_error": err32,
                "accept_gbs": r32["accept_gbs"], "refresh_ms": r32["refresh_ms"]}
        del run32
    cpu = None if args.no_cpu else cpu_baseline(wl, args.cpu_seconds)

    achieved = r64["accept_gbs"]
    line = {
        "metric": METRIC, "value": r64["value"], "unit": "walker-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "walkers": W, "n": wl.n, "sites": wl.sites, "ranks": list(wl.ranks),
                   "delay": wl.delay, "refresh_every": wl.refresh, "mc_steps_per_bench_step": wl.refresh,
                   "mode": "forced-accept", "graph": not args.no_graph, "streams": args.streams},
        "roofline": {"bound": "hbm", "kernel": "det_accept_kernel (delayed)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic("det_accept_kernel_slater_n256_k124_counters.md", DET_SOURCES,
                                                W // max(1, args.streams)),
                     "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "avg_us": r64["accept_avg_us"], "bytes_per_launch": r64["accept_bytes_per_launch"]},
        "cpu_baseline": cpu,
        "rel_error": err64,
        "recompute": rc,
        "speedup_vs_recompute": (r64["value"] / rc["slogdet"]["walker_steps_per_s"])
        if rc and "walker_steps_per_s" in rc.get("slogdet", {}) else None,
        "flush": r64["flush"], "refresh_ms": r64["refresh_ms"],
        "fp32": fp32,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
