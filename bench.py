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


def source_code_bytes(text: bytes) -> bytes:
    """The code of a C/C++/HIP source for the counter-profile hash: comments removed and
    blank lines dropped, so that documentation edits do not void the recorded counters
    (any change to the code itself does)."""
    import re
    code = re.sub(rb"/\*.*?\*/", b"", text, flags=re.S)
    code = re.sub(rb"//[^\n]*", b"", code)
    return b"\n".join(line.rstrip() for line in code.split(b"\n") if line.strip())


def counter_traffic(profile, sources, walkers_per_launch, key=None):
    """HBM bytes measured by the FETCH_SIZE / WRITE_SIZE counter passes recorded in
    profiles/<profile>, or None when the kernel sources changed since.  With
    walkers_per_launch: bytes per launch of that many walkers (None when the recorded
    launch size differs); with key (walkers_per_launch None): bytes per walker of the
    recorded launch configuration `key`."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(source_code_bytes(fh.read()))
    keys = {}
    for line in open(path):
        part = line.strip().split(":", 1)
        if len(part) == 2:
            keys[part[0].strip()] = part[1].strip()
    if keys.get("source_sha256") != h.hexdigest():
        return None
    if key is not None:
        if keys.get("launch_config") != key or "traffic_bytes_per_walker" not in keys:
            return None
        return float(keys["traffic_bytes_per_walker"])
    if "traffic_bytes_per_launch" not in keys or keys.get("walkers_per_launch") != str(int(walkers_per_launch)):
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
    ap.add_argument("--workload", default="uneven_n64_1024_fp32",
                    help="default: the uneven batch as the headline with every other configuration as extra keys")
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
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: the uneven batch only, without the other configurations")
    ap.add_argument("--roofline-only", action="store_true",
                    help="uneven batch: set-up and the event-timed roofline pass only (for kernel traces)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    return ap.parse_args()


class Run:
    """One walker batch of a uniform-n workload with its pre-generated draws for one refresh
    period, driven by the package's PeriodDriver (sub-batches on their own streams,
    staggered refreshes, one HIP graph per period).  Workloads without a refresh (the plain
    Sherman-Morrison chain) use their step count as the period and never refresh."""

    def __init__(self, wl, dtype, walkers, seed_offset=0, streams=1, layout=0):
        import torch
        from paper_2602_05255_amd import inputs as gen
        from paper_2602_05255_amd import lrx
        from paper_2602_05255_amd.driver import PeriodDriver
        self.torch, self.lrx = torch, lrx
        self.wl = wl
        if wl.kind == "det":
            phi, occ, emp, g = gen.slater_inputs(wl, walkers=walkers, seed_offset=seed_offset)
        else:
            phi, occ, emp, g = gen.pairing_inputs(wl, walkers=walkers, seed_offset=seed_offset)
        self.phi = phi
        self.W = walkers
        self.P = wl.refresh if wl.refresh else wl.steps
        t0 = time.time()
        k, e, s = gen.hop_draws_batch(g, self.P, walkers, wl.n, wl.sites - wl.n, wl.ranks, wl.k_max)
        log(f"  draws {self.P} x {walkers}: {time.time() - t0:.1f}s")
        draws = tuple(torch.as_tensor(x).cuda() for x in (k, e, s))
        kind = lrx.LRX_DET if wl.kind == "det" else lrx.LRX_PF
        self.drv = PeriodDriver(kind, dtype, phi, occ, emp, wl.k_max, wl.delay, self.P, draws, streams=streams,
                                refresh=bool(wl.refresh), layout=layout)
        self.parts = self.drv.parts
        self.wk = self.parts[0][0]

    @property
    def occ(self):
        return self.drv.occ

    def period(self, timer=None, probe=None):
        self.drv.period(timer, probe)

    def capture(self):
        self.drv.capture()

    def step(self):
        self.drv.step()


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
    """Algorithmic HBM bytes of one accept launch (all walkers accepted), kbar = mean rank.
    Delayed DET: read A_0^-1 (n^2), the tau live b-slot rows (n kbar tau), u and C
    (2 n kbar); write slot tau of a and b (2 n kbar).
    Delayed PF: read A_0^-1 (n^2), x, col and the 2 tau a-slot columns; write the two
    new a-slot columns.
    Plain DET (K = 0): read and write A^-1 (2 n^2), read u, C (2 n kbar), read R^-1.
    Plain PF: three passes over A^-1 (3 n^2)."""
    n = wl.n
    kbar = float(np.mean(wl.ranks))
    if wl.kind == "pf":
        return W * s * (3 * n * n if not wl.delay else n * n + 2 * n * tau + 4 * n)
    if not wl.delay:
        return W * s * (2 * n * n + 3 * n * kbar)
    return W * s * (n * n + n * kbar * tau + 4 * n * kbar)


def queue_filler(torch, ms=150.0):
    """About `ms` of GPU work (FP64 GEMMs) on the current stream, enqueued at once."""
    a = torch.ones(4096, 4096, dtype=torch.float64, device="cuda") / 4096.0
    reps = max(1, int(ms / 3.0))             # one 4096^3 FP64 GEMM is about 3 ms here or more
    for _ in range(reps):
        a = a @ a


def filled_pass(torch, fn, ms=100.0, tries=4):
    """fn() enqueues a pass whose launches carry HIP event pairs.  The pass is queued
    behind a GEMM filler so that the GPU is still busy when the host has finished
    enqueueing it: then no event pair brackets host launch time.  If the filler had
    drained by then (its end event complete), the pass is repeated behind a filler
    twice as long.  Returns (fn's result, filler ms, True if the last try stayed
    covered)."""
    out = None
    for _ in range(tries):
        queue_filler(torch, ms)
        mark = torch.cuda.Event()
        mark.record()
        out = fn()
        drained = mark.query()
        torch.cuda.synchronize()
        if not drained:
            return out, ms, True
        ms *= 2.0
    return out, ms / 2.0, False


def measure(wl, dtype, walkers, args, torch, label):
    run = Run(wl, dtype, walkers, streams=args.streams)
    elem = torch.empty((), dtype=dtype).element_size()
    wl_launch = walkers / len(run.parts)      # walkers per launch (one sub-batch)
    # roofline pass: eager, HIP events around every accept launch of one period.  A filler
    # (FP64 GEMMs) keeps the GPU busy while the host enqueues the period, so that no event
    # pair brackets host launch time.
    run.period()
    torch.cuda.synchronize()

    def timed_period():
        timer = EventTimer(torch)
        run.period(timer)
        return timer

    timer, _, covered = filled_pass(torch, timed_period)
    res = timer.results()
    acc = res["accept"]
    bytes_tot = sum(accept_bytes(wl, elem, wp, tau) for tau, _, wp in acc)
    t_tot = sum(dt for _, dt, _ in acc)
    fl = res.get("flush", [])
    flush_t = np.mean([dt for _, dt, _ in fl]) if fl else None
    refresh_t = np.mean([dt for _, dt, _ in res["refresh"]]) if "refresh" in res else float("nan")
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


def _recompute_state(torch, wide, table, occ, kind):
    """FP64 / complex128 full recompute on the same GPU (torch.linalg: rocSOLVER LU) of the
    inverse and log|det| (log|pf| = log|det| / 2) at the given occupancies."""
    src = torch.as_tensor(table).to(device=occ.device, dtype=wide)
    o = occ.long()
    if kind == "pf":
        a = src[o[:, :, None], o[:, None, :]]
        _, la = torch.linalg.slogdet(a)
        inv = torch.linalg.inv(a)
        return 0.5 * (inv - inv.transpose(1, 2)), 0.5 * la
    a = src[o]
    _, la = torch.linalg.slogdet(a)
    return torch.linalg.inv(a), la


def state_error(torch, wk, idx, table, kind, complex_):
    """Relative Frobenius error of the stored inverse and absolute error of the tracked
    log|value| of walkers idx (state flushed) against the same-GPU full recompute."""
    wide = torch.complex128 if complex_ else torch.float64
    rinv, la = _recompute_state(torch, wide, table, wk.occ[idx], kind)
    inv = wk.st.inv[idx].to(wide)
    if kind == "det":
        inv = inv.transpose(1, 2)          # the state holds A^-T
    e_inv = (torch.linalg.matrix_norm(inv - rinv) / torch.linalg.matrix_norm(rinv)).cpu().numpy()
    e_la = (wk.st.logabs[idx] - la).abs().cpu().numpy()
    return e_inv, e_la


def summarize_errors(rows, against, walkers):
    """rows: (steps_since_refresh, e_inv[], e_la[]).  The headline figures are those at the
    largest steps-since-refresh (the state just before its refresh), with the profile."""
    prof = []
    for since in sorted({r[0] for r in rows}):
        ei = np.concatenate([r[1] for r in rows if r[0] == since])
        el = np.concatenate([r[2] for r in rows if r[0] == since])
        prof.append([int(since), float(ei.max()), float(np.median(ei)), float(el.max()), float(np.median(el))])
    last = prof[-1]
    return {"steps_since_refresh": last[0], "inverse_max": last[1], "inverse_median": last[2],
            "logdet_abs_max": last[3], "logdet_abs_median": last[4], "walkers": walkers, "against": against,
            "profile_columns": ["steps_since_refresh", "inverse_max", "inverse_median", "logdet_abs_max",
                                "logdet_abs_median"],
            "profile": prof}


def error_profile(run, torch, nsample=16):
    """Error of the LRU state against the same-GPU FP64 / complex128 recompute at every
    flush boundary of one eager period of the first sub-batch: steps since its refresh
    K, 2K, ..., P (the last just before the refresh).  The first sub-batch has offset 0,
    so after the timed periods it stands right after its refresh."""
    from paper_2602_05255_amd import lrx
    wk0 = run.parts[0][0]
    idx = torch.as_tensor(np.linspace(0, wk0.W - 1, min(nsample, wk0.W)).astype(int), device="cuda")
    every = run.wl.delay if run.wl.delay else max(1, run.P // 8)

    def one(mode, what):
        rows = []

        def probe(p, wk, since):
            if p == 0 and (since % every == 0 or since == run.P):
                e_inv, e_la = state_error(torch, wk, idx, run.phi, run.wl.kind, run.wl.complex_)
                rows.append((since, e_inv, e_la))
        saved = run.drv.mode, run.drv.seed
        run.drv.mode, run.drv.seed = mode, 0x5EED
        run.period(probe=probe)
        run.drv.mode, run.drv.seed = saved
        torch.cuda.synchronize()
        return summarize_errors(rows, f"FP64/complex128 full recompute on the same GPU (torch.linalg), {what}, "
                                      "sampled walkers of one sub-batch at each flush boundary of a period",
                                len(idx))
    err = one(lrx.LRX_MH_DEVICE_RNG, "Metropolis chain")
    err["forced_accept"] = one(lrx.LRX_MH_FORCE, "forced-accept chain")
    return err


def cpu_baseline(wl, seconds):
    """The oracle (full recompute: LU + inverse per walker-step) on the host cores, on a
    bounded sample of the workload's walkers (all OpenMP threads of the host)."""
    import oracle as orc
    from paper_2602_05255_amd import inputs as gen
    orc.build(force=False)
    if wl.n == 0:      # uneven batch: the same number of sampled walkers from every size class
        classes, g = gen.uneven_inputs(wl, seed_offset=7)
        per = 8
        chains = []
        for c in classes:
            chains.append((orc.DetChain(c["phi"], c["occ"][:per], c["empty"][:per]), c["n"]))
        done, t0 = 0, time.perf_counter()
        while True:
            for ch, n in chains:
                k, e, s = gen.hop_draws(g, per, n, n, wl.ranks, wl.k_max)
                ch.propose(k, e, s)
                ch.accept(k, e, s, np.ones(per, bool))
                done += per
            el = time.perf_counter() - t0
            if el >= seconds:
                break
        sizes = ",".join(str(n) for _, n in chains)
        return {"value": done / el, "unit": "walker-steps/s", "cores": orc.num_threads(), "kind": "oracle",
                "sample": f"{per} walkers from each size class n in {{{sizes}}} x {done // (per * len(chains))} "
                          f"steps of the {wl.name} workload, k in {list(wl.ranks)}, full FP64 LU + inverse per "
                          f"walker-step (the class mix of the workload), {el:.1f}s"}
    W = 64 if wl.n > 64 else wl.walkers
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


def recompute(wl, run, torch, reps=3, chunks=(1, 16, 128), sample=128, with_inverse=True):
    """Full recompute on the same GPU: gather the matrices at the walkers' occupancies, then
    torch.linalg.slogdet (rocSOLVER LU; for the Pfaffian the skew matrix's |det| = pf^2, a
    lower bound on any O(n^3) Pfaffian, without the sign), FP64 / complex128.  rocSOLVER's
    batched LU is timed in batches of each size in `chunks` on the first `sample` walkers and
    the fastest rate is kept (large batches starve it at large n).  A second figure adds
    torch.linalg.inv."""
    wide = torch.complex128 if wl.complex_ else torch.float64
    src = torch.as_tensor(run.phi).to(device="cuda", dtype=wide)
    occ = run.occ.long()[:min(sample, run.W)]
    nw = occ.shape[0]
    n = wl.n

    def gather(o):
        return src[o[:, :, None], o[:, None, :]] if wl.kind == "pf" else src[o]
    out = {}
    variants = [("slogdet", lambda a: torch.linalg.slogdet(a))]
    if with_inverse:
        variants.append(("slogdet+inv", lambda a: (torch.linalg.slogdet(a), torch.linalg.inv(a))))
    for name, fn in variants:
        best = None
        for chunk in chunks:
            if chunk > nw:
                continue

            def batch():
                for c0 in range(0, nw - nw % chunk, chunk):
                    fn(gather(occ[c0:c0 + chunk]))
            try:
                batch()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    batch()
                torch.cuda.synchronize()
            except RuntimeError as exc:        # report, do not fail the benchmark line
                out.setdefault("errors", []).append(f"{name} chunk {chunk}: {str(exc).splitlines()[0]}")
                continue
            done = (nw - nw % chunk) * reps
            rate = done / (time.perf_counter() - t0)
            if best is None or rate > best[0]:
                best = (rate, chunk)
        if best is None:
            continue
        cplx = 4 if wl.complex_ else 1
        flops = cplx * (2 * n ** 3 / 3 + (2 * n ** 3 if "inv" in name else 0))
        out[name] = {"walker_steps_per_s": best[0], "batch": best[1], "tflops": best[0] * flops / 1e12,
                     "walkers_timed": nw}
    return out


def with_steps(args, steps, warmup):
    a = argparse.Namespace(**vars(args))
    a.steps, a.warmup = steps, warmup
    return a


def bench_uniform(wl, dtype, args, torch, label, walkers=None, streams=None, recompute_leg=False):
    """A uniform-n determinant or Pfaffian workload: timed periods (one HIP graph each), the
    accept roofline, the flush and refresh times, the error profile against the same-GPU
    recompute, and optionally the full recompute comparator."""
    W = walkers or args.walkers or wl.walkers
    a = argparse.Namespace(**vars(args))
    a.streams = streams if streams is not None else a.streams
    log(f"workload {wl.name} [{label}]: W={W} n={wl.n} L={wl.sites} ranks={wl.ranks} K={wl.delay} "
        f"refresh={wl.refresh} streams={a.streams}")
    run, r = measure(wl, dtype, W, a, torch, label)
    err = error_profile(run, torch)
    log(f"  [{label}] error vs recompute before refresh: inverse max {err['inverse_max']:.2e} median "
        f"{err['inverse_median']:.2e}; log|value| max {err['logdet_abs_max']:.2e}")
    out = {"value": r["value"], "unit": "walker-steps/s", "ms_per_period": r["ms_per_step"],
           "steps_per_period": run.P, "walkers": W, "streams": a.streams, "dtype": label,
           "accept": {"avg_us": r["accept_avg_us"], "gbs": r["accept_gbs"], "hbm_frac": r["accept_gbs"] / HBM_PEAK_GBS,
                      "bytes_per_launch": r["accept_bytes_per_launch"]},
           "flush": r["flush"], "refresh_ms": r["refresh_ms"], "rel_error": err}
    if recompute_leg:
        out["recompute"] = recompute(wl, run, torch)
        rs = out["recompute"].get("slogdet", {}).get("walker_steps_per_s")
        out["speedup_vs_recompute"] = r["value"] / rs if rs else None
        if wl.refresh:
            own = run.parts[0][2] / (r["refresh_ms"] * 1e-3)    # walkers of one sub-batch per refresh
            out["recompute_own_refresh"] = {"walker_steps_per_s": own,
                                            "what": "this library's FP64/complex128 refresh of one sub-batch "
                                                    "(log|value| + inverse), timed alone"}
            out["speedup_vs_own_refresh"] = r["value"] / own
    del run
    torch.cuda.empty_cache()
    return out


def bench_plain_chain(wl, args, torch):
    """The plain Sherman-Morrison chain (16 walkers, n = 32, FP64, K = 0): latency bound, so
    the figure is microseconds per Markov-chain step of the whole batch."""
    a = with_steps(args, max(3, args.steps // 4), 2)
    a.streams = 1
    run, r = measure(wl, torch.float64, wl.walkers, a, torch, "f64 plain")
    err = error_profile(run, torch)
    out = {"us_per_step": r["ms_per_step"] * 1e3 / run.P, "walker_steps_per_s": r["value"],
           "walkers": wl.walkers, "steps_per_graph": run.P, "rel_error": err}
    log(f"  [plain n=32] {out['us_per_step']:.2f} us per step of 16 walkers")
    return out


def bench_single_hop(n, args, torch, walkers=1024):
    """Single-hop (k = 1) determinant LRU at one n against full recompute on the same GPU:
    the delayed LRU in FP64 and with FP32 bulk (FP64 refresh every 128 steps amortised), the
    library's own FP64 Gauss-Jordan refresh (log|det| + inverse), and rocSOLVER slogdet at
    its best batch size."""
    from paper_2602_05255_amd import inputs as gen
    wn = gen.nsweep_workload(n)
    a = with_steps(args, max(2, args.steps // 8), 1)
    a.streams = 1
    r64 = bench_uniform(wn, torch.float64, a, torch, f"f64 n={n}", walkers=walkers, streams=1, recompute_leg=True)
    r32 = bench_uniform(wn, torch.float32, a, torch, f"f32 n={n}", walkers=walkers, streams=1)
    own = r64["recompute_own_refresh"]["walker_steps_per_s"]
    rs = r64["recompute"].get("slogdet", {}).get("walker_steps_per_s")
    out = {"n": n, "walkers": walkers, "delay": wn.delay, "lru_f64": r64, "lru_f32_bulk": r32,
           "speedup_f64_vs_own_gj": r64["value"] / own, "speedup_f32_bulk_vs_own_gj": r32["value"] / own,
           "speedup_f64_vs_rocsolver": r64["value"] / rs if rs else None,
           "speedup_f32_bulk_vs_rocsolver": r32["value"] / rs if rs else None}
    log(f"  n={n}: LRU f64 {r64['value']:.4g}/s, f32 bulk {r32['value']:.4g}/s; own GJ {own:.4g}/s; "
        f"rocSOLVER {rs if rs else float('nan'):.4g}/s")
    return out


def bench_adjoint(wl, args, torch):
    """Forward + hand-written backward of log det(Phi[occ] + B C^T) for all 512 samples
    (complex64 bulk), from the samples' walker state (the checkpoint: factorised once, as a
    sampler holds it) and, for comparison, with a fresh complex128 factorisation of every
    A_s = Phi[occ_s] inside each step."""
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd import lrx
    from paper_2602_05255_amd.adjoint import lowrank_logdet, walker_lowrank_logdet
    from paper_2602_05255_amd.walkers import Walkers
    phi, occ, b, c, w = gen.lowrank_inputs(wl)
    dev = "cuda"
    L = phi.shape[0]
    emp = np.stack([np.setdiff1d(np.arange(L), o) for o in occ]).astype(np.int32)
    wk = Walkers(lrx.LRX_DET, torch.complex64, phi, occ, emp)
    P = torch.tensor(phi, dtype=torch.complex128, device=dev, requires_grad=True)
    B = torch.tensor(b, dtype=torch.complex64, device=dev, requires_grad=True)
    C = torch.tensor(c, dtype=torch.complex64, device=dev, requires_grad=True)
    occ_t = torch.as_tensor(occ, dtype=torch.int32, device=dev)
    wt = torch.as_tensor(w, dtype=torch.complex128, device=dev)

    def from_state():
        ld, _ = walker_lowrank_logdet(wk, B, C, P)
        (wt * ld).real.sum().backward()

    def with_init():
        ld, _ = lowrank_logdet(P, B, C, occ_t, torch.complex64)
        (wt * ld).real.sum().backward()

    out = {}
    for name, fn in (("from_state", from_state), ("with_factorisation", with_init)):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        out[name] = {"ms_per_step": ms, "samples_per_s": occ.shape[0] / (ms * 1e-3)}
    S, n = occ.shape
    log(f"  [adjoint] fwd+bwd from the walker state {out['from_state']['ms_per_step']:.2f} ms; with the "
        f"factorisation {out['with_factorisation']['ms_per_step']:.2f} ms (512 samples)")
    return {"metric": "samples/s (log det + hand-written backward)", "value": out["from_state"]["samples_per_s"],
            "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": out["from_state"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "c64", "data": "synthetic",
            "config": {"workload": wl.name, "samples": S, "n": n, "sites": L, "rank": b.shape[-1]},
            "modes": out,
            "note": "from_state: the forward reads A^-1 from the samples' walker state (the checkpoint); "
                    "with_factorisation: a complex128 Gauss-Jordan factorisation of every A_s in each step"}


def bench_uneven(wl, args, torch):
    """Uneven batch (4096 walkers, n in {64..1024}, FP32 bulk): one benchmark step is one
    refresh period (128 Markov-chain steps of every walker and the FP64 refresh of every
    class), replayed as one HIP graph.  Each size class runs on the schedule the
    autotuner measured fastest for it: the persistent window kernel (windows of 16
    steps, one launch for all such classes, on a side stream) or per-step launches
    (four sub-batches on their own streams with staggered refreshes)."""
    from paper_2602_05255_amd import autotune
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd import lrx
    from paper_2602_05255_amd.uneven import UnevenBatch
    classes, g = gen.uneven_inputs(wl, walkers=args.walkers or None)
    K, P = wl.delay, wl.refresh
    t0 = time.time()
    log(f"  autotune cache {autotune.cache_path()}")
    plan = [autotune.tune_class(torch.float32, c["n"], wl.k_max, wl.ranks) for c in classes]
    t_tune = time.time() - t0
    draws = []
    for c in classes:
        k, e, s_ = gen.hop_draws_batch(g, P, len(c["walkers"]), c["n"], c["n"], wl.ranks, wl.k_max)
        draws.append(tuple(torch.as_tensor(x).cuda() for x in (k, e, s_)))
    batch = UnevenBatch(torch.float32, classes, wl.k_max, plan, K, P, draws, substreams=4)
    if batch.uw is not None:
        autotune.tune_grid(batch.uw)
    batch.prime()
    torch.cuda.synchronize()
    log(f"  setup {time.time() - t0:.1f}s (autotune {t_tune:.1f}s); plan " +
        ", ".join(f"n={c['n']}:W={len(c['walkers'])}:K={p['delay']}:" +
                  ("window" if p["window"] else f"steps/rows={p['rows_per_block'] or 'auto'}")
                  for c, p in zip(classes, plan)) +
        (f"; window grid {batch.uw.grid}" if batch.uw is not None else ""))
    # roofline pass: every launch of one period of each per-step class timed alone with
    # HIP events (queue filler ahead so that no event pair brackets host time); window
    # launches of the window classes timed the same way
    per_class = {}
    es = 4
    kbar = float(np.mean(wl.ranks))
    for i, d in zip(batch.step_idx, batch.drivers):
        n = classes[i]["n"]
        wn = gen.Workload(f"uneven_n{n}", "det", 2 * n, n, d.W, wl.ranks, wl.k_max, plan[i]["delay"], P,
                          False, "f32")
        def timed_period():
            timer = EventTimer(torch)
            d.period(timer)
            return timer

        timer, _, covered = filled_pass(torch, timed_period)
        res = timer.results()
        acc = res["accept"]
        byt = sum(accept_bytes(wn, es, wp, tau) for tau, _, wp in acc)
        tt = sum(dt for _, dt, _ in acc)
        fl = res.get("flush", [])
        per_class[n] = {"schedule": "per-step", "delay": plan[i]["delay"], "rows_per_block": plan[i]["rows_per_block"],
                        "accept_us": tt / len(acc) * 1e6, "accept_gbs": byt / tt / 1e9,
                        "accept_bytes_per_launch": byt / len(acc), "accept_total_ms": tt * 1e3,
                        "accept_launches": len(acc), "walkers_per_launch": d.W / len(d.parts),
                        "events_covered": covered,
                        "propose_total_ms": sum(dt for _, dt, _ in res["propose"]) * 1e3,
                        "flush_total_ms": sum(dt for _, dt, _ in fl) * 1e3,
                        "refresh_total_ms": sum(dt for _, dt, _ in res.get("refresh", [])) * 1e3}
    if batch.uw is not None:
        def timed_windows():
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(P // K + 2)]
            ev[0].record()
            for i in range(P // K):
                batch._window(i, lrx.LRX_MH_FORCE)
                ev[i + 1].record()
            batch.uw.refresh(report=False)
            ev[-1].record()
            return ev

        ev, _, _ = filled_pass(torch, timed_windows)
        win = [ev[i].elapsed_time(ev[i + 1]) * 1e-3 for i in range(P // K)]
        wbytes = 0.0
        for p in batch.uw.parts:
            n, Kc = p.st.n, p.st.delay
            per_step = n * n + n * kbar * (Kc - 1) / 2.0 + 4 * n * kbar
            wbytes += p.st.walkers * es * (K * per_step + (K / Kc) * (2 * n * n + 2 * n * Kc * kbar))
        per_class["window_classes"] = {
            "schedule": "persistent window", "sizes": [int(p.st.n) for p in batch.uw.parts],
            "delays": [int(p.st.delay) for p in batch.uw.parts], "grid": batch.uw.grid,
            "window_ms": float(np.mean(win)) * 1e3, "window_gbs": wbytes / float(np.mean(win)) / 1e9,
            "refresh_ms": ev[P // K].elapsed_time(ev[-1])}
    if args.roofline_only:
        return {"roofline_pass": per_class}
    # the whole period in one HIP graph
    s_ = torch.cuda.Stream()
    s_.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s_):
        batch.period()
    torch.cuda.current_stream().wait_stream(s_)
    torch.cuda.synchronize()
    graph = None
    if not args.no_graph:
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            batch.period()
        torch.cuda.synchronize()
    step = graph.replay if graph is not None else batch.period
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
    W = batch.walkers
    value = W * P * args.steps / T
    # error profiles: one eager period each with Metropolis decisions (device generator)
    # and with forced accept; at every point where a class or sub-batch has an empty
    # delay window and a multiple of 32 steps since its refresh, 4 sampled walkers
    # against the same-GPU FP64 recompute
    def profile(mode, what):
        rows, by_n = [], {}

        def probe(kind, part, since):
            if since % 32:
                return
            parts = part.parts if kind == "window" else [part]
            for q in parts:
                Wq = q.st.walkers if kind == "window" else q.W
                idx = torch.as_tensor(np.linspace(0, Wq - 1, 4).astype(int), device="cuda")
                a_, b_ = state_error(torch, q, idx, q.table, "det", False)
                rows.append((since, a_, b_))
                by_n.setdefault(int(q.st.n), []).append((since, a_))
        batch.period(mode, probe)
        torch.cuda.synchronize()
        out = summarize_errors(rows, f"FP64 full recompute on the same GPU (torch.linalg), {what}, 4 sampled "
                                     "walkers per class or sub-batch at every 32 steps since its refresh", 4)
        # per size class, at its largest steps since refresh: max and median inverse error, and
        # the share of sampled walker-states (all probe points) above 1e-3 relative
        cls = {}
        for n_, rs in sorted(by_n.items()):
            last = max(r[0] for r in rs)
            e_last = np.concatenate([r[1] for r in rs if r[0] == last])
            e_all = np.concatenate([r[1] for r in rs])
            cls[n_] = {"steps_since_refresh": int(last), "inverse_max": float(e_last.max()),
                       "inverse_median": float(np.median(e_last)),
                       "share_above_1e-3": float(np.mean(e_all > 1e-3)), "samples": int(e_all.size)}
        out["by_class"] = cls
        return out
    err = profile(lrx.LRX_MH_DEVICE_RNG, "Metropolis chain")
    err["forced_accept"] = profile(lrx.LRX_MH_FORCE, "forced-accept chain")
    dom = max((v for v in per_class.values() if v.get("schedule") == "per-step"),
              key=lambda v: v["accept_total_ms"], default=None)
    dom_n = [n for n, v in per_class.items() if v is dom][0] if dom is not None else None
    log(f"  [uneven f32] {value:.4g} walker-steps/s, {T / args.steps * 1e3:.2f} ms per period; " +
        "; ".join(f"n={n}: accept {v['accept_gbs']:.0f} GB/s" for n, v in per_class.items() if "accept_gbs" in v))
    line = {"metric": METRIC, "value": value, "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": T / args.steps * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": wl.name, "walkers": W, "sizes": list(wl.extra["sizes"]),
                       "class_walkers": {int(c["n"]): len(c["walkers"]) for c in classes},
                       "ranks": list(wl.ranks), "refresh_every": P, "mc_steps_per_bench_step": P,
                       "mode": "forced-accept", "bulk": "f32", "refresh": "f64",
                       "schedule_per_class": {int(c["n"]): ("persistent window" if p["window"] else "per-step")
                                              for c, p in zip(classes, plan)},
                       "delay_per_class": {int(c["n"]): p["delay"] for c, p in zip(classes, plan)},
                       "delay_schedule_and_tiles": "autotuned", "graph": graph is not None,
                       "substreams_per_step_class": 4, "window_steps": K},
            "per_class": per_class, "rel_error": err}
    if dom is not None:
        wpl = dom["walkers_per_launch"]
        tw = counter_traffic(f"det_accept_kernel_{wl.name}_counters.md", DET_SOURCES, None,
                             key=f"n{dom_n}_K{dom['delay']}_rows{dom['rows_per_block']}")
        line["roofline"] = {"bound": "hbm", "kernel": f"det_accept_kernel (delayed, FP32, n={dom_n})",
                            "achieved": dom["accept_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": dom["accept_gbs"] / HBM_PEAK_GBS,
                            "traffic": tw * wpl if tw is not None else None,
                            "avg_us": dom["accept_us"], "bytes_per_launch": dom["accept_bytes_per_launch"],
                            "walkers_per_launch": wpl, "events_covered": dom["events_covered"]}
    else:
        wc = per_class["window_classes"]
        line["roofline"] = {"bound": "hbm", "kernel": "det_window_kernel", "achieved": wc["window_gbs"],
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": wc["window_gbs"] / HBM_PEAK_GBS,
                            "traffic": None, "avg_us": wc["window_ms"] * 1e3, "bytes_per_launch": None}
    return line


def bench_delay_sweep(args, torch, kinds=("det", "pf")):
    """Delayed against plain updates (the paper's delay-length benchmark): 16384 walkers,
    n = 128, 128 consecutive single-hop updates of every walker (forced accept, no refresh),
    FP64, for each delay K; one HIP graph of the 128 steps per K.  Reports the time per
    128 updates, the speedup of each delay over the plain update, the fastest K, and the
    K the library's byte model proposes (lrx_autotune_lookup default)."""
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd import lrx
    out = {}
    for kind in kinds:
        base = gen.WORKLOADS[f"delay_sweep_n128_{kind}"]
        W = args.walkers or base.walkers
        rows = []
        for K in (0, 2, 4, 8, 16, 32, 64):
            wl = gen.Workload(base.name, kind, base.sites, base.n, W, base.ranks, base.k_max, K, 0, False, "f64",
                              steps=base.steps, seed=base.seed)
            run = Run(wl, torch.float64, W, streams=1)
            run.capture()
            for _ in range(2):
                run.step()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            reps = 3
            e0.record()
            for _ in range(reps):
                run.step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            rows.append({"delay": K, "ms_per_128_updates": ms, "walker_steps_per_s": W * wl.steps / (ms * 1e-3)})
            log(f"  delay sweep {kind} K={K}: {ms:.2f} ms per 128 updates of {W} walkers")
            del run
            torch.cuda.empty_cache()
        plain = rows[0]["ms_per_128_updates"]
        for r in rows:
            r["speedup_vs_plain"] = plain / r["ms_per_128_updates"]
        best = min(rows[1:], key=lambda r: r["ms_per_128_updates"])
        model = lrx.lrx_autotune_lookup(torch.float64, base.n, 1)["delay"]
        out[kind] = {"walkers": W, "n": base.n, "updates": base.steps, "dtype": "f64", "rows": rows,
                     "best_delay": best["delay"], "best_speedup_vs_plain": best["speedup_vs_plain"],
                     "byte_model_delay": model,
                     "paper_best_delay": 16 if kind == "det" else 4,
                     "paper_note": "the paper finds T = 16 (det) and T = 4 (pf) best for 16384 matrices of n = 128 "
                                   "and reports an additional 20-40 % speedup of delayed over plain updates "
                                   "(NVIDIA A100-80GB, JAX)"}
    return out


def bench_pf_layouts(args, torch, steps=64):
    """The Pfaffian workload's shape (256 walkers, n = 512, L = 1024, complex64 bulk), single
    hops, forced accept, no refresh: 64 consecutive steps (one HIP graph) on the plain
    update (three passes over A^-1), the fused delay-one update (one read + write pass),
    the same on packed skew storage (upper 64 x 64 tiles), and the delayed update with
    K = 32 on full and on packed storage.  Bytes per accepted step (algorithmic): plain 3 n^2,
    fused 2 n^2, packed 2 * tiles * 64^2, delayed n^2 + 2 n^2 / K (flush), packed delayed
    tiles * 64^2 (1 + 2 / K), plus the slot columns."""
    from paper_2602_05255_amd import inputs as gen
    from paper_2602_05255_amd import lrx
    base = gen.WORKLOADS["pfaffian_n512_c64"]
    W, n = args.walkers or base.walkers, base.n
    es = 8
    nt = (n + 63) // 64
    tiles = nt * (nt + 1) // 2
    variants = [("plain", lrx.LRX_LAYOUT_FULL, 0, 3.0 * n * n),
                ("fused", lrx.LRX_LAYOUT_FUSED, 0, 2.0 * n * n),
                ("packed", lrx.LRX_LAYOUT_PACKED, 0, 2.0 * tiles * 64 * 64),
                ("delayed_K32", lrx.LRX_LAYOUT_FULL, 32, n * n + 2.0 * n * n / 32 + 2.0 * n * 16),
                ("packed_delayed_K32", lrx.LRX_LAYOUT_PACKED, 32,
                 tiles * 64 * 64 + 2.0 * tiles * 64 * 64 / 32 + 2.0 * n * 16)]
    rows = []
    for name, layout, K, per_step in variants:
        wl = gen.Workload(base.name, "pf", base.sites, n, W, (1,), 1, K, 0, True, "c64", steps=steps, seed=base.seed)
        run = Run(wl, torch.complex64, W, streams=1, layout=layout)
        run.capture()
        for _ in range(2):
            run.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record()
        for _ in range(reps):
            run.step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = W * steps * per_step * es / (ms * 1e-3) / 1e9
        rows.append({"variant": name, "layout": int(layout), "delay": K, "ms_per_64_steps": ms,
                     "walker_steps_per_s": W * steps / (ms * 1e-3), "bytes_per_step": per_step * es,
                     "achieved_gbs_algorithmic": gbs})
        log(f"  pf layouts {name}: {ms:.3f} ms per {steps} steps, {gbs:.0f} GB/s algorithmic")
        del run
        torch.cuda.empty_cache()
    plain = rows[0]["ms_per_64_steps"]
    for r in rows:
        r["speedup_vs_plain"] = plain / r["ms_per_64_steps"]
    return {"walkers": W, "n": n, "sites": base.sites, "dtype": "c64", "steps": steps, "mode": "forced-accept",
            "rows": rows}


def bench_nsweep(wl, args, torch):
    """Single-hop determinant LRU against full recompute on the same GPU, n = 64 .. 1024
    (the shape of the paper's speedup-vs-n figure), one bench_single_hop per n."""
    sizes = [int(x) for x in args.sizes.split(",")] if args.sizes else list(wl.extra["sizes"])
    rows = [bench_single_hop(n, args, torch, walkers=args.walkers or wl.walkers) for n in sizes]
    top = rows[-1]
    return {"metric": METRIC, "value": top["lru_f64"]["value"], "unit": "walker-steps/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": wl.name, "walkers": args.walkers or wl.walkers, "sizes": sizes, "ranks": [1],
                       "refresh_every": wl.refresh, "mode": "forced-accept"},
            "sweep": rows}


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


def headline_line(res, args, extras):
    """The JSON line: the uneven batch (the largest single-GPU configuration) as the headline,
    the other configurations as extra keys."""
    line = {k: res[k] for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                                "roofline")}
    line.update({k: v for k, v in extras.items()})
    return line


def run_extra(name, fn):
    """One secondary configuration; a failure is reported in the line instead of ending the run."""
    t0 = time.time()
    try:
        out = fn()
    except Exception as exc:       # noqa: BLE001 -- keep the headline line whatever happens here
        import traceback
        traceback.print_exc()
        out = {"error": f"{type(exc).__name__}: {exc}"}
    log(f"  [{name}] done in {time.time() - t0:.1f}s")
    return out


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
    if args.workload == "pf_layouts_n512_c64":
        print(json.dumps({"workload": "pf_layouts_n512_c64", **bench_pf_layouts(args, torch)}), flush=True)
        return
    wl = gen.WORKLOADS[args.workload]
    if args.streams is None:
        args.streams = {"slater_n256_k124": 4, "pfaffian_n512_c64": 4}.get(wl.name, 1)
    if wl.name == "logpsi_grad_n512_c64":
        print(json.dumps(bench_adjoint(wl, args, torch)), flush=True)
        return
    if wl.name == "nsweep_det_k1":
        print(json.dumps(bench_nsweep(wl, args, torch)), flush=True)
        return
    if wl.name.startswith("delay_sweep_n128"):
        print(json.dumps({"workload": "delay_sweep_n128", **bench_delay_sweep(args, torch, (wl.kind,))}), flush=True)
        return
    if wl.name != "uneven_n64_1024_fp32":
        # one uniform workload on its own
        dt = {"f64": torch.float64, "f32": torch.float32, "c64": torch.complex64,
              "c128": torch.complex128}[wl.bulk]
        if wl.name == "slater_n32_fp64":
            print(json.dumps({"workload": wl.name, **bench_plain_chain(wl, args, torch)}), flush=True)
            return
        r = bench_uniform(wl, dt, args, torch, wl.bulk, recompute_leg=not args.no_recompute)
        print(json.dumps({"metric": METRIC, "workload": wl.name, **r}), flush=True)
        return

    # Default: the uneven batch is the headline; every other configuration rides along.
    t_start = time.time()
    res = bench_uneven(wl, args, torch)
    if args.roofline_only:
        print(json.dumps({"workload": wl.name, **res}), flush=True)
        return
    torch.cuda.empty_cache()
    extras = {"rel_error": res["rel_error"], "per_class": res["per_class"]}
    short = with_steps(args, max(3, args.steps // 4), max(1, min(args.warmup, 2)))
    c2 = gen.WORKLOADS["slater_n256_k124"]
    cfg = {}
    if args.headline_only:
        print(json.dumps(headline_line(res, args, extras)), flush=True)
        return
    cfg["slater_n256_k124"] = run_extra("slater_n256_k124", lambda: {
        "f64": bench_uniform(c2, torch.float64, short, torch, "f64", streams=4, recompute_leg=not args.no_recompute),
        "f32": bench_uniform(c2, torch.float32, short, torch, "f32", streams=4)})
    c3 = gen.WORKLOADS["pfaffian_n512_c64"]
    cfg["pfaffian_n512_c64"] = run_extra("pfaffian_n512_c64", lambda: bench_uniform(
        c3, torch.complex64, short, torch, "c64", streams=4, recompute_leg=not args.no_recompute))
    cfg["single_hop_n1024"] = run_extra("single_hop_n1024", lambda: bench_single_hop(1024, args, torch))
    cfg["delay_sweep_n128"] = run_extra("delay_sweep_n128", lambda: bench_delay_sweep(short, torch))
    cfg["pf_layouts_n512_c64"] = run_extra("pf_layouts_n512_c64", lambda: bench_pf_layouts(short, torch))
    cfg["slater_n32_fp64"] = run_extra("slater_n32_fp64", lambda: bench_plain_chain(
        gen.WORKLOADS["slater_n32_fp64"], args, torch))
    cfg["logpsi_grad_n512_c64"] = run_extra("logpsi_grad_n512_c64", lambda: bench_adjoint(
        gen.WORKLOADS["logpsi_grad_n512_c64"], short, torch))
    extras["configs"] = cfg
    extras["cpu_baseline"] = None if args.no_cpu else cpu_baseline(wl, args.cpu_seconds)
    extras["bench_wall_s"] = time.time() - t_start
    print(json.dumps(headline_line(res, args, extras)), flush=True)


if __name__ == "__main__":
    main()
