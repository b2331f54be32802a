"""Period driver: a walker batch stepped one refresh period at a time, capturable
into one HIP graph.

A period is P Markov-chain steps of every walker -- per step the fused
propose_hop (hop vectors and ratio, Sec. II.A / III.A) and accept_hop
(decision, delayed or plain update, occupancy commit), a flush whenever the
delay window fills (Eqs. delayed_Ainv, pf_delayed_Ainv) -- followed by the
FP64 / complex128 refresh (the stability remark of Sec. II.A).  The proposal
draws of the P steps are device tensors indexed by the step's position in the
period, so replaying a captured period proposes new hops from the walkers'
current occupancies.

With ``streams > 1`` the batch is split into that many independent sub-batches
(own states), each driven on its own default-priority HIP stream forked from
and joined to the calling stream every period; sub-batch p runs ``offsets[p]``
steps ahead (a whole number of delay windows) so the sub-batches reach their
refresh at different steps.  Every launch is a liblrx call; this module only
sequences them.
"""
from __future__ import annotations

import contextlib

import numpy as np
import torch

from . import lrx
from .walkers import Walkers


class PeriodDriver:
    def __init__(self, kind, dtype, table, occ, empty, k_max, delay, period, draws, streams=1,
                 mode=lrx.LRX_MH_FORCE, seed=0, ratio_log=None, refresh=True, u01=None, layout=0):
        """draws: device int32 tensors (k [P][W], elec [P][W][k_max], slot [P][W][k_max]);
        period: P (steps per period); ratio_log: optional device tensor [P][W] receiving the
        ratio of every walker at each step (indexed by the step's position in the period);
        refresh: refresh every sub-batch once per period (False: never); u01: device float64
        [P][W] uniforms read at run time by mode LRX_MH_UNIFORMS (refill it between replays
        of a captured period); layout: storage / update scheme of the states (LRX_LAYOUT_*)."""
        occ = np.asarray(occ)
        empty = np.asarray(empty)
        self.kind, self.P, self.W = kind, int(period), occ.shape[0]
        self.k, self.e, self.s = draws
        self.mode, self.seed, self.ratio_log, self.do_refresh, self.u01 = mode, seed, ratio_log, refresh, u01
        bounds = np.linspace(0, self.W, max(1, streams) + 1).astype(int)
        self.parts = []
        for a0, a1 in zip(bounds[:-1], bounds[1:]):
            wk = Walkers(kind, dtype, table, occ[a0:a1], empty[a0:a1], k_max, delay, refresh_period=0, layout=layout)
            self.parts.append((wk, int(a0), int(a1), torch.cuda.Stream() if streams > 1 else None))
        K = max(1, delay)
        self.offsets = [(p * (self.P // len(self.parts))) // K * K for p in range(len(self.parts))]
        self.primed = False
        self.graph = None
        self.counter = 0

    @property
    def occ(self):
        return torch.cat([wk.occ for wk, _, _, _ in self.parts])

    def _step(self, wk, a0, a1, t, timer):
        k, e, s = self.k[t, a0:a1], self.e[t, a0:a1], self.s[t, a0:a1]
        if timer is not None:
            timer.begin("propose", wk.st.slot)
        if wk.kind == lrx.LRX_DET:
            lrx.lrx_det_propose_hop(wk.st, wk.table, wk.sites, wk.occ, wk.empty, wk.n_empty, k, e, s, wk.u,
                                    wk.ratio)
        else:
            lrx.lrx_pf_propose_hop(wk.st, wk.table, wk.sites, wk.occ, wk.empty, wk.n_empty, k, e, s, wk.u,
                                   wk.ratio)
        if self.ratio_log is not None:
            self.ratio_log[t, a0:a1].copy_(wk.ratio)
        if timer is not None:
            timer.end("propose")
            timer.begin("accept", wk.st.slot, wk.W)
        accept_hop = lrx.lrx_det_accept_hop if wk.kind == lrx.LRX_DET else lrx.lrx_pf_accept_hop
        u01 = self.u01[t, a0:a1] if (self.u01 is not None and self.mode == lrx.LRX_MH_UNIFORMS) else None
        accept_hop(wk.st, k, e, s, wk.u, self.mode, u01, self.seed, t, wk.accept, wk.occ, wk.empty, wk.n_empty)
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
        torch.cuda.synchronize()
        self.primed = True

    def period(self, timer=None, probe=None):
        """One refresh period.  With a timer every launch runs on the calling stream (one at
        a time, so that each launch's own duration is measured); otherwise the sub-batches
        run on their streams.  probe(part_index, wk, steps_since_refresh) is called (eager
        runs only) after every step that leaves a sub-batch's delay window empty."""
        self.prime()
        split = timer is None and probe is None and len(self.parts) > 1
        cur = torch.cuda.current_stream()
        if split:
            for _, _, _, st in self.parts:
                st.wait_stream(cur)
        for t in range(self.P):
            for p, ((wk, a0, a1, st), off) in enumerate(zip(self.parts, self.offsets)):
                local = (t + off) % self.P
                with torch.cuda.stream(st) if split else contextlib.nullcontext():
                    self._step(wk, a0, a1, local, None if split else timer)
                    if probe is not None and wk.st.slot == 0:
                        probe(p, wk, local + 1)
                    if local == self.P - 1 and self.do_refresh:
                        if timer is not None:
                            timer.begin("refresh", 0)
                        wk.refresh(report=False)
                        if timer is not None:
                            timer.end("refresh")
        if split:
            for _, _, _, st in self.parts:
                cur.wait_stream(st)

    def capture(self):
        """Record one period into a HIP graph (after one eager warm-up period)."""
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
