"""Uneven walker batches: several size classes n advanced together.

Each size class n is a uniform determinant state (its own delay K, chosen by
the autotuner).  Two schedules exist per class:

* the persistent window (``UnevenWalkers``): ``lrx_det_window`` moves every
  walker of every such class through ``steps`` delayed steps in one launch,
  one work-group per walker, flushing each walker in-kernel when its class's
  delay window fills;
* per-step launches (``PeriodDriver``): propose_hop / accept_hop / flush
  kernels spread every walker over several work-groups, the class cut into
  sub-batches on their own streams with staggered refreshes.

``UnevenBatch`` runs a whole refresh period of every class, each class on the
schedule the autotuner picked for its size, with the window classes on a side
stream beside the per-step classes, so one HIP graph holds the period.  The
periodic FP64 refresh is ``lrx_det_refresh`` per class or sub-batch.  Device
buffers are torch tensors; all arithmetic runs in liblrx.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lrx

_INT = torch.int32


class UnevenWalkers:
    def __init__(self, dtype, classes, k_max, delays, steps, refresh_period=0, grid=None, device="cuda",
                 ranks=None):
        """classes: list of dicts {phi [2n][n] float64, occ [W][n], empty [W][n_empty]};
        delays: K per class (int or list), or "auto" (autotuned per size class for the
        proposal ranks `ranks`); steps: steps per window; grid: work-groups of the
        persistent launch, None (two per compute unit) or "auto" (autotuned)."""
        rk = tuple(ranks) if ranks is not None else tuple(2 ** i for i in range(int(np.log2(k_max)) + 1))
        if delays == "auto":
            from . import autotune
            delays = [autotune.tune_class(dtype, int(np.asarray(c["occ"]).shape[1]), k_max, rk, device=device)["delay"]
                      for c in classes]
        if isinstance(delays, int):
            delays = [delays] * len(classes)
        self.delays = [int(K) for K in delays]
        self.device = torch.device(device)
        self.steps, self.k_max, self.refresh_period = int(steps), int(k_max), int(refresh_period)
        self.parts = []
        for cls, K in zip(classes, delays):
            occ = np.asarray(cls["occ"], dtype=np.int32)
            emp = np.asarray(cls["empty"], dtype=np.int32)
            W, n = occ.shape
            st = lrx.State(lrx.LRX_DET, dtype, W, n, k_max, int(K), device)
            table = torch.as_tensor(np.ascontiguousarray(cls["phi"], dtype=np.float64)).to(self.device)
            occ_t = torch.as_tensor(occ).to(self.device)
            emp_t = torch.as_tensor(emp).to(self.device)
            lrx.lrx_det_init_inverse(st, table, table.shape[0], occ_t)
            S, KM = self.steps, k_max
            part = lrx.WindowClass(
                st, table, occ_t, emp_t,
                k=torch.ones(S, W, dtype=_INT, device=self.device),
                elec=torch.zeros(S, W, KM, dtype=_INT, device=self.device),
                slot=torch.zeros(S, W, KM, dtype=_INT, device=self.device),
                u=torch.zeros(W, KM, n, dtype=st.dtype, device=self.device),
                ratio=torch.zeros(S, W, dtype=torch.float64, device=self.device),
                accept=torch.zeros(S, W, dtype=torch.uint8, device=self.device))
            part.report = torch.zeros(W, 2, dtype=torch.float64, device=self.device)
            self.parts.append(part)
        self.work = torch.zeros(lrx.lrx_window_work_bytes(self.parts, self.steps), dtype=torch.uint8,
                                device=self.device)
        cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        self.grid = 2 * cus if grid in (None, "auto") else int(grid)
        self.windows = 0
        if grid == "auto":
            from . import autotune
            autotune.tune_grid(self)

    @property
    def walkers(self):
        return sum(p.st.walkers for p in self.parts)

    def set_draws(self, draws):
        """draws: per class (k [steps][W], elec [steps][W][k_max], slot [steps][W][k_max]) host arrays."""
        for p, (k, e, s) in zip(self.parts, draws):
            p.k.copy_(torch.as_tensor(np.ascontiguousarray(k, dtype=np.int32)))
            p.elec.copy_(torch.as_tensor(np.ascontiguousarray(e, dtype=np.int32)))
            p.slot.copy_(torch.as_tensor(np.ascontiguousarray(s, dtype=np.int32)))

    def window(self, mode=lrx.LRX_MH_FORCE, seed=0, counter=0, u01=None, mask=None):
        """One persistent launch of ``steps`` steps for every walker of every class.

        mode LRX_MH_MASK takes the per-class decisions ``mask`` ([steps][W] host
        arrays); LRX_MH_UNIFORMS takes per-class ``u01`` ([steps][W])."""
        for i, p in enumerate(self.parts):
            if mode == lrx.LRX_MH_MASK:
                p.accept.copy_(torch.as_tensor(np.asarray(mask[i], dtype=np.uint8)))
            if mode == lrx.LRX_MH_UNIFORMS:
                if p.u01 is None:
                    p.u01 = torch.zeros(self.steps, p.st.walkers, dtype=torch.float64, device=self.device)
                p.u01.copy_(torch.as_tensor(np.asarray(u01[i], dtype=np.float64)))
        lrx.lrx_det_window(self.parts, self.steps, mode, seed, counter, self.work, self.grid)
        self.windows += 1
        if self.refresh_period and (self.windows * self.steps) % self.refresh_period == 0:
            self.refresh(report=False)

    def flush(self):
        for p in self.parts:
            if p.st.slot:
                lrx.lrx_det_flush_delayed(p.st)

    def refresh(self, report=True):
        self.flush()
        for p in self.parts:
            lrx.lrx_det_refresh(p.st, p.table, p.table.shape[0], p.occ, p.report if report else None)
        return [p.report for p in self.parts]

    def inverses(self):
        """A^-1 per class in FP64 (flushing pending slots first)."""
        self.flush()
        return [p.st.inv.to(torch.float64).transpose(1, 2) for p in self.parts]


class UnevenBatch:
    """Every size class of an uneven batch for whole refresh periods, each class on its
    tuned schedule: the persistent window (classes in ``window_classes``) or per-step
    launches with ``substreams`` staggered sub-batches per class.

    draws: per class (k [P][W], elec [P][W][k_max], slot [P][W][k_max]) device int32
    tensors for the P = period steps (indexed by the step's position in the period)."""

    def __init__(self, dtype, classes, k_max, plan, window_steps, period, draws, substreams=4, grid=None,
                 device="cuda"):
        from .driver import PeriodDriver
        self.device = torch.device(device)
        self.P, self.K = int(period), int(window_steps)
        self.plan = plan
        win = [i for i, p in enumerate(plan) if p["window"]]
        step = [i for i, p in enumerate(plan) if not p["window"]]
        self.win_idx, self.step_idx = win, step
        self.uw = None
        if win:
            self.uw = UnevenWalkers(dtype, [classes[i] for i in win], k_max, [plan[i]["delay"] for i in win],
                                    self.K, grid=grid, device=device)
            self.win_draws = [draws[i] for i in win]
        self.drivers = []
        for i in step:
            c = classes[i]
            self.drivers.append(PeriodDriver(lrx.LRX_DET, dtype, c["phi"], c["occ"], c["empty"], k_max,
                                             plan[i]["delay"], self.P, draws[i], streams=substreams))
        self.side = torch.cuda.Stream(device=self.device) if win and step else None
        self.walkers = sum(int(np.asarray(c["occ"]).shape[0]) for c in classes)

    def _window(self, i, mode):
        K = self.K
        for p, (k, e, s) in zip(self.uw.parts, self.win_draws):
            p.k, p.elec, p.slot = k[i * K:(i + 1) * K], e[i * K:(i + 1) * K], s[i * K:(i + 1) * K]
        lrx.lrx_det_window(self.uw.parts, K, mode, 0x5EED, i * K, self.uw.work, self.uw.grid)

    def prime(self):
        for d in self.drivers:
            d.prime()

    def period(self, mode=lrx.LRX_MH_FORCE, probe=None):
        """One refresh period of every class.  probe(kind, part, since) is called (eager
        runs) whenever a class or sub-batch stands with an empty delay window: kind
        "window" (part = the UnevenWalkers, since = steps into the period) or "step"
        (part = the Walkers of a sub-batch, since = its steps since refresh)."""
        cur = torch.cuda.current_stream()
        if self.uw is not None:
            ctx = torch.cuda.stream(self.side) if (self.side is not None and probe is None) else None
            if ctx is not None:
                self.side.wait_stream(cur)
                ctx.__enter__()
            for i in range(self.P // self.K):
                self._window(i, mode)
                if probe is not None and all(p.st.slot == 0 for p in self.uw.parts):
                    probe("window", self.uw, (i + 1) * self.K)
            self.uw.refresh(report=False)
            if ctx is not None:
                ctx.__exit__(None, None, None)
        for d in self.drivers:
            saved = d.mode
            d.mode = mode
            d.period(probe=(lambda p, wk, since: probe("step", wk, since)) if probe is not None else None)
            d.mode = saved
        if self.side is not None and probe is None:
            cur.wait_stream(self.side)
