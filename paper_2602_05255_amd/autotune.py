"""Autotuner for the persistent uneven-batch window.

Picks, per (device, bulk dtype, n, k_max), the delay K of a size class (the
window length between flushes: longer windows move fewer bytes in the flush
but make every accept read more slot rows, Sec. II.C), its schedule (the
persistent window kernel, one work-group per walker, or per-step launches that
spread a walker over several work-groups) and, for per-step launches, the
accept tile height (rows of M per work-group); and per batch the number of
work-groups of the persistent launch.  Candidates are timed on the
device with the real kernels (HIP events around whole windows, all proposals
applied) and the winners are cached in a JSON file keyed by the device name,
so a process tunes a shape once.

The search starts from the byte-model optimum K* = sqrt(2 n / kbar) and tries
the powers of two around it that the C ABI accepts (K k_max <= 256).
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

from . import inputs as gen
from . import lrx

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "lrx", "autotune.json")
# Measured results shipped with the package (the same JSON layout as the cache, keyed by
# device name): consulted when the user cache has no entry, so that a device of a tuned
# model starts from the same schedule every time instead of re-timing it.
SEED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_seed.json")


def cache_path():
    return os.environ.get("LRX_TUNE_CACHE", DEFAULT_CACHE)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _entry(table, key):
    """The entry for key from the cache table, else from the shipped seed (None if neither)."""
    if key in table:
        return table[key]
    if os.environ.get("LRX_TUNE_NO_SEED"):
        return None
    return _load(SEED).get(key)


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_key(device):
    """Architecture and compute-unit count (the marketing name is not reliable: some
    tools report it empty)."""
    prop = torch.cuda.get_device_properties(device)
    arch = str(getattr(prop, "gcnArchName", "") or torch.cuda.get_device_name(device)).split(":")[0]
    return f"{arch.replace(' ', '_')}|cu{prop.multi_processor_count}"


def delay_candidates(n, k_max, ranks):
    kbar = float(np.mean(ranks))
    k_star = math.sqrt(2.0 * n / kbar)
    base = 2 ** int(round(math.log2(max(k_star, 1.0))))
    cands = sorted({max(2, base // 2), base, base * 2, base * 4})
    return [K for K in cands if K * k_max <= 256 and K <= lrx.LRX_MAX_DELAY]


def _time_windows(uw, reps):
    """Seconds per walker-step over `reps` windows (forced accept, refresh excluded).  The
    windows are launched directly (not through uw.window), so the batch's window count and
    refresh schedule are left alone."""
    lrx.lrx_det_window(uw.parts, uw.steps, lrx.LRX_MH_FORCE, 0, 0, uw.work, uw.grid)      # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        lrx.lrx_det_window(uw.parts, uw.steps, lrx.LRX_MH_FORCE, 0, (r + 1) * uw.steps, uw.work, uw.grid)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (reps * uw.steps * uw.walkers)


def rows_candidates(n):
    """Accept work-group heights tried for the per-step schedule: the library's heuristic (0)
    and 32, 64, 128, 256, 512 rows below n."""
    return [0] + [r for r in (32, 64, 128, 256, 512) if r < n]


def _time_steps(wk, draws, steps, reps):
    """Seconds per walker-step of the per-step schedule (propose_hop, accept_hop, flush;
    forced accept) over `reps` passes of `steps` steps."""
    k, e, s = draws

    def one_pass():
        for t in range(steps):
            lrx.lrx_det_propose_hop(wk.st, wk.table, wk.sites, wk.occ, wk.empty, wk.n_empty, k[t], e[t], s[t],
                                    wk.u, wk.ratio)
            lrx.lrx_det_accept_hop(wk.st, k[t], e[t], s[t], wk.u, lrx.LRX_MH_FORCE, None, 0, t, wk.accept, wk.occ,
                                   wk.empty, wk.n_empty)
            if wk.st.slot == wk.delay:
                wk.flush()
    one_pass()                                        # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        one_pass()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (reps * steps * wk.W)


def tune_class(dtype, n, k_max, ranks, walkers=512, device="cuda", cache=None, seed=7):
    """Schedule of one size class, timed on the device: the delay K, and either the
    persistent window kernel (one work-group per walker for the whole window) or per-step
    launches with the accept work-group height (rows of M per work-group) that ran
    fastest.  Cached in JSON and registered with the library's tuning table
    (lrx_autotune_store), which the per-step accept launches read."""
    from .uneven import UnevenWalkers
    from .walkers import Walkers
    path = cache or cache_path()
    table = _load(path)
    dname = str(dtype).replace("torch.", "")
    key = f"{_device_key(device)}|{dname}|n={n}|kmax={k_max}|ranks={list(ranks)}|v3"
    hit = _entry(table, key) or {}
    if all(f in hit for f in ("delay", "rows_per_block", "window")):
        out = {"delay": int(hit["delay"]), "rows_per_block": int(hit["rows_per_block"]), "window": bool(hit["window"])}
        lrx.lrx_autotune_store(dtype, n, k_max, out["delay"], out["rows_per_block"], 0, out["window"])
        return out
    g = gen.generator(gen.SEED_BASE + seed)
    phi = gen.normal(g, (2 * n, n))
    occ, emp = gen.occupancy(g, walkers, 2 * n, n)
    results = {}
    for K in delay_candidates(n, k_max, ranks):
        kk, ee, ss = gen.hop_draws_batch(g, 2 * K, walkers, n, n, ranks, k_max)
        uw = UnevenWalkers(dtype, [{"phi": phi, "occ": occ, "empty": emp}], k_max, [K], 2 * K, device=device)
        uw.set_draws([(kk, ee, ss)])
        results[("window", K, 0)] = _time_windows(uw, reps=2)
        del uw
        wk = Walkers(lrx.LRX_DET, dtype, phi, occ, emp, k_max, K, device=device)
        dev = tuple(torch.as_tensor(x).to(device) for x in (kk, ee, ss))
        for rpb in rows_candidates(n):
            lrx.lrx_autotune_store(dtype, n, k_max, K, rpb, 0, 0)
            results[("step", K, rpb)] = _time_steps(wk, dev, 2 * K, reps=2)
        del wk
    best = min(results, key=results.get)
    out = {"delay": int(best[1]), "rows_per_block": int(best[2]), "window": best[0] == "window"}
    table = _load(path)
    table[key] = dict(out, s_per_walker_step={f"{m},K={K},rows={r}": v for (m, K, r), v in results.items()},
                      tuned_at=time.strftime("%Y-%m-%d %H:%M:%S"))
    _store(path, table)
    lrx.lrx_autotune_store(dtype, n, k_max, out["delay"], out["rows_per_block"], 0, out["window"])
    return out


def tune_delay(dtype, n, k_max, ranks, walkers=512, device="cuda", cache=None, seed=7):
    """Best delay K for one size class (see tune_class)."""
    return tune_class(dtype, n, k_max, ranks, walkers, device, cache, seed)["delay"]


def tune_grid(uw, candidates=(1, 2, 3, 4), cache=None):
    """Work-groups per compute unit of the persistent launch for this batch (cached)."""
    path = cache or cache_path()
    table = _load(path)
    dev = uw.device
    shape = ",".join(f"{p.st.n}x{p.st.walkers}/K{p.st.delay}" for p in uw.parts)
    key = f"{_device_key(dev)}|grid|{str(uw.parts[0].st.dtype).replace('torch.', '')}|kmax={uw.k_max}|{shape}"
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    hit = _entry(table, key)
    if hit is not None and "wgs_per_cu" in hit:
        uw.grid = int(hit["wgs_per_cu"]) * cus
        return uw.grid
    # the trial windows advance the chains; keep the caller's state out of it
    snap = [(p.st.buffers["inv"].clone(), p.st.buffers["fa"].clone(), p.st.buffers["fb"].clone(),
             p.st.buffers["stash"].clone(), p.st.logabs.clone(), p.st.phase.clone(), p.st.flags.clone(),
             p.occ.clone(), p.empty.clone(), p.st.c.slot) for p in uw.parts]
    results = {}
    for c in candidates:
        uw.grid = c * cus
        results[c] = _time_windows(uw, reps=2)
    best = min(results, key=results.get)
    for p, (inv, fa, fb, st, la, ph, fl, occ, emp, slot) in zip(uw.parts, snap):
        p.st.buffers["inv"].copy_(inv)
        p.st.buffers["fa"].copy_(fa)
        p.st.buffers["fb"].copy_(fb)
        p.st.buffers["stash"].copy_(st)
        p.st.logabs.copy_(la)
        p.st.phase.copy_(ph)
        p.st.flags.copy_(fl)
        p.occ.copy_(occ)
        p.empty.copy_(emp)
        p.st.c.slot = slot
    uw.grid = best * cus
    table = _load(path)
    table[key] = {"wgs_per_cu": int(best), "s_per_walker_step": {str(c): v for c, v in results.items()},
                  "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, table)
    return uw.grid
