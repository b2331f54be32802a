"""Uneven walker batches: several size classes advanced by one persistent launch.

Each size class n is a uniform determinant state (its own delay K, chosen by
the autotuner).  ``UnevenWalkers.window()`` enqueues ``lrx_det_window``: one
launch that moves every walker of every class through ``steps`` delayed steps,
flushing each walker's slots inside the kernel when its class's window fills.
The periodic FP64 refresh is one ``lrx_det_refresh`` per class.  Device
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
        if delays == "auto":
            from . import autotune
            rk = tuple(ranks) if ranks is not None else tuple(2 ** i for i in range(int(np.log2(k_max)) + 1))
            delays = [autotune.tune_delay(dtype, int(np.asarray(c["occ"]).shape[1]), k_max, rk, device=device)
                      for c in classes]
        if isinstance(delays, int):
            delays = [delays] * len(classes)
        self.delays = [int(K) for K in delays]
        self.device = torch.device(device)
        self.steps, self.k_max, self.refresh_period = int(steps), int(k_max), int(refresh_period)
        self.parts, self.tables = [], []
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
        self.order = lrx.lrx_window_plan(self.parts, self.steps).to(self.device)
        self.queue = torch.zeros(1, dtype=_INT, device=self.device)
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
        lrx.lrx_det_window(self.parts, self.steps, mode, seed, counter, self.order, self.queue, self.grid)
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
