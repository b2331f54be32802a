"""Walker-batch driver: sequences the C-ABI calls of one Markov-chain step.

A step (Sec. II.A-II.C for determinants, III.A-III.C for Pfaffians) is
  build_hop -> propose_ratio -> accept decision -> accept_update -> hop_commit
  [-> flush_delayed when the delay window is full] [-> refresh every P steps].
This module only holds device buffers (torch) and calls ``lrx``; every
arithmetic step runs in the HIP kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lrx

_INT = torch.int32


class Walkers:
    """A batch of walkers sharing one orbital (DET) or pairing (PF) matrix."""

    def __init__(self, kind, dtype, table, occ, empty, k_max=1, delay=0, refresh_period=0,
                 device="cuda", layout=0):
        occ = np.asarray(occ)
        empty = np.asarray(empty)
        self.kind = kind
        self.W, self.n = occ.shape
        self.n_empty = empty.shape[1]
        self.k_max, self.delay, self.refresh_period = k_max, delay, refresh_period
        self.st = lrx.State(kind, dtype, self.W, self.n, k_max, delay, device, layout)
        self.device = torch.device(device)
        self.table = torch.as_tensor(np.ascontiguousarray(table)).to(self.device, self.st.wide)
        self.sites = int(self.table.shape[0])
        self.occ = torch.as_tensor(occ.astype(np.int32)).to(self.device)
        self.empty = torch.as_tensor(empty.astype(np.int32)).to(self.device)
        W, KM = self.W, k_max
        self.k = torch.ones(W, dtype=_INT, device=self.device)
        self.elec = torch.zeros(W, KM, dtype=_INT, device=self.device)
        self.slot = torch.zeros(W, KM, dtype=_INT, device=self.device)
        if kind == lrx.LRX_DET:
            self.u = torch.zeros(W, KM, self.n, dtype=self.st.dtype, device=self.device)
        else:
            self.u = torch.zeros(W, self.n, dtype=self.st.dtype, device=self.device)
        self.ratio = torch.zeros(W, dtype=self.st.wide, device=self.device)
        self.accept = torch.zeros(W, dtype=torch.uint8, device=self.device)
        self.u01 = torch.zeros(W, dtype=torch.float64, device=self.device)
        self.report = torch.zeros(W, 2, dtype=torch.float64, device=self.device)
        self.steps = 0
        self.use_draws(self.k, self.elec, self.slot)
        self.init()

    # ------------------------------------------------------------------ pieces
    def init(self):
        f = lrx.lrx_det_init_inverse if self.kind == lrx.LRX_DET else lrx.lrx_pf_init_inverse
        f(self.st, self.table, self.sites, self.occ)

    def refresh(self, report=True):
        if self.st.slot:
            self.flush()
        f = lrx.lrx_det_refresh if self.kind == lrx.LRX_DET else lrx.lrx_pf_refresh
        f(self.st, self.table, self.sites, self.occ, self.report if report else None)
        return self.report

    def set_draws(self, k, elec, slot):
        """Copy one step's proposal draws (host arrays) into the step buffers."""
        for dst, src in ((self.k, k), (self.elec, elec), (self.slot, slot)):
            dst.copy_(torch.as_tensor(np.ascontiguousarray(src, dtype=np.int32)))
        self.use_draws(self.k, self.elec, self.slot)

    def use_draws(self, k, elec, slot):
        """Point the step at device draw tensors (no copy): k [W], elec/slot [W][k_max] int32."""
        self._k, self._elec, self._slot = k, elec, slot

    def propose(self):
        k, elec, slot = self._k, self._elec, self._slot
        if self.kind == lrx.LRX_DET:
            lrx.lrx_det_build_hop(self.st, self.table, self.sites, self.occ, self.empty, self.n_empty,
                                  k, elec, slot, self.u)
            lrx.lrx_det_propose_ratio(self.st, k, elec, self.u, self.ratio)
        else:
            lrx.lrx_pf_build_hop(self.st, self.table, self.sites, self.occ, self.empty, self.n_empty,
                                 k, elec, slot, self.u)
            lrx.lrx_pf_propose_ratio(self.st, k, elec, self.u, self.ratio)
        return self.ratio

    def decide(self, mode=lrx.LRX_MH_FORCE, u01=None, mask=None, seed=0, counter=0):
        """Fill the accept bytes: a host/device mask, or lrx_metropolis in ``mode``."""
        if mask is not None:
            if isinstance(mask, torch.Tensor):
                self.accept.copy_(mask.to(torch.uint8), non_blocking=True)
            else:
                self.accept.copy_(torch.as_tensor(np.asarray(mask, dtype=np.uint8)))
            return self.accept
        if u01 is not None:
            self.u01.copy_(torch.as_tensor(np.asarray(u01, dtype=np.float64)) if not isinstance(u01, torch.Tensor)
                           else u01)
        lrx.lrx_metropolis(self.st, self.ratio, self.u01 if mode == lrx.LRX_MH_UNIFORMS else None, seed,
                           counter, mode, self.accept)
        return self.accept

    def apply(self):
        k, elec, slot = self._k, self._elec, self._slot
        if self.kind == lrx.LRX_DET:
            lrx.lrx_det_accept_update(self.st, k, elec, self.u, self.accept)
        else:
            lrx.lrx_pf_accept_update(self.st, k, elec, self.u, self.accept)
        lrx.lrx_hop_commit(self.W, self.n, self.n_empty, self.k_max, k, elec, slot,
                           self.accept, self.occ, self.empty)
        self.steps += 1
        if self.delay and self.st.slot == self.delay:
            self.flush()
        if self.refresh_period and self.steps % self.refresh_period == 0:
            self.refresh(report=False)

    def step_device(self, mode=lrx.LRX_MH_FORCE, u01=None, seed=0, counter=0):
        """One step with the decision taken on the device, for determinants and Pfaffians
        alike in two fused calls: propose_hop (hop vector and ratio) and accept_hop
        (decision, update and occupancy commit)."""
        k, elec, slot = self._k, self._elec, self._slot
        if self.kind == lrx.LRX_DET:
            lrx.lrx_det_propose_hop(self.st, self.table, self.sites, self.occ, self.empty, self.n_empty,
                                    k, elec, slot, self.u, self.ratio)
            lrx.lrx_det_accept_hop(self.st, k, elec, slot, self.u, mode, u01, seed, counter, self.accept,
                                   self.occ, self.empty, self.n_empty)
        else:
            lrx.lrx_pf_propose_hop(self.st, self.table, self.sites, self.occ, self.empty, self.n_empty,
                                   k, elec, slot, self.u, self.ratio)
            lrx.lrx_pf_accept_hop(self.st, k, elec, slot, self.u, mode, u01, seed, counter, self.accept,
                                  self.occ, self.empty, self.n_empty)
        self.steps += 1
        if self.delay and self.st.slot == self.delay:
            self.flush()
        if self.refresh_period and self.steps % self.refresh_period == 0:
            self.refresh(report=False)

    def flush(self):
        if self.kind == lrx.LRX_DET:
            lrx.lrx_det_flush_delayed(self.st)
        else:
            lrx.lrx_pf_flush_delayed(self.st)

    # ------------------------------------------------------------------ views
    def inverse(self):
        """A^-1 of every walker in the wide dtype (flushing pending factors first; packed
        Pfaffian states are read out through lrx_pf_read_inverse)."""
        if self.st.slot:
            self.flush()
        if self.st.layout == lrx.LRX_LAYOUT_PACKED:
            out = torch.empty(self.W, self.n, self.n, dtype=self.st.dtype, device=self.device)
            lrx.lrx_pf_read_inverse(self.st, out)
            return out.to(self.st.wide)
        m = self.st.inv.to(self.st.wide)
        return m.transpose(1, 2) if self.kind == lrx.LRX_DET else m
