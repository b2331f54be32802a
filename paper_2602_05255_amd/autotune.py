"""Autotuner for the persistent uneven-batch window.

Picks, per (device, bulk dtype, n, k_max), the delay K of a size class (the
window length between flushes: longer windows move fewer bytes in the flush
but make every accept read more slot rows, Sec. II.C), and per batch the
number of work-groups of the persistent launch.  Candidates are timed on the
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


def cache_path():
    return os.environ.get("LRX_TUNE_CACHE", DEFAULT_CACHE)


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _device_key(device):
    return torch.cuda.get_device_name(device).replace(" ", "_")


def delay_candidates(n, k_max, ranks):
    kbar = float(np.mean(ranks))
    k_star = math.sqrt(2.0 * n / kbar)
    base = 2 ** int(round(math.log2(max(k_star, 1.0))))
    cands = sorted({max(2, base // 2), base, base * 2, base * 4})
    return [K for K in cands if K * k_max <= 256 and K <= lrx.LRX_MAX_DELAY]


def _time_windows(uw, reps):
    """Seconds per walker-step over `reps` windows (forced accept, refresh excluded)."""
    uw.window(mode=lrx.LRX_MH_FORCE, counter=0)      # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        lrx.lrx_det_window(uw.parts, uw.steps, lrx.LRX_MH_FORCE, 0, (r + 1) * uw.steps, uw.order, uw.queue,
                           uw.grid)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / (reps * uw.steps * uw.walkers)


def tune_delay(dtype, n, k_max, ranks, walkers=512, device="cuda", cache=None, seed=7):
    """Best delay K for one size class (cached)."""
    from .uneven import UnevenWalkers
    path = cache or cache_path()
    table = _load(path)
    key = f"{_device_key(device)}|{str(dtype).replace('torch.', '')}|n={n}|kmax={k_max}|ranks={list(ranks)}"
    if key in table and "delay" in table[key]:
        return int(table[key]["delay"])
    g = gen.generator(gen.SEED_BASE + seed)
    phi = gen.normal(g, (2 * n, n))
    occ, emp = gen.occupancy(g, walkers, 2 * n, n)
    results = {}
    for K in delay_candidates(n, k_max, ranks):
        uw = UnevenWalkers(dtype, [{"phi": phi, "occ": occ, "empty": emp}], k_max, [K], 2 * K, device=device)
        k, e, s = gen.hop_draws_batch(g, 2 * K, walkers, n, n, ranks, k_max)
        uw.set_draws([(k, e, s)])
        results[K] = _time_windows(uw, reps=3)
        del uw
    best = min(results, key=results.get)
    table = _load(path)
    table[key] = {"delay": int(best), "s_per_walker_step": {str(K): v for K, v in results.items()},
                  "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, table)
    return int(best)


def tune_grid(uw, candidates=(1, 2, 3, 4), cache=None):
    """Work-groups per compute unit of the persistent launch for this batch (cached)."""
    path = cache or cache_path()
    table = _load(path)
    dev = uw.device
    shape = ",".join(f"{p.st.n}x{p.st.walkers}/K{p.st.delay}" for p in uw.parts)
    key = f"{_device_key(dev)}|grid|{str(uw.parts[0].st.dtype).replace('torch.', '')}|kmax={uw.k_max}|{shape}"
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    if key in table and "wgs_per_cu" in table[key]:
        uw.grid = int(table[key]["wgs_per_cu"]) * cus
        return uw.grid
    # the trial windows advance the chains; keep the caller's state out of it
    snap = [(p.st.buffers["inv"].clone(), p.st.buffers["fa"].clone(), p.st.buffers["fb"].clone(),
             p.st.buffers["stash"].clone(), p.st.logabs.clone(), p.st.phase.clone(), p.occ.clone(),
             p.empty.clone(), p.st.c.slot) for p in uw.parts]
    results = {}
    for c in candidates:
        uw.grid = c * cus
        results[c] = _time_windows(uw, reps=2)
    best = min(results, key=results.get)
    for p, (inv, fa, fb, st, la, ph, occ, emp, slot) in zip(uw.parts, snap):
        p.st.buffers["inv"].copy_(inv)
        p.st.buffers["fa"].copy_(fa)
        p.st.buffers["fb"].copy_(fb)
        p.st.buffers["stash"].copy_(st)
        p.st.logabs.copy_(la)
        p.st.phase.copy_(ph)
        p.occ.copy_(occ)
        p.empty.copy_(emp)
        p.st.c.slot = slot
    uw.grid = best * cus
    table = _load(path)
    table[key] = {"wgs_per_cu": int(best), "s_per_walker_step": {str(c): v for c, v in results.items()},
                  "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}
    _store(path, table)
    return uw.grid
