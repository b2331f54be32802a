"""Seeded synthetic inputs shared by the GPU path's tests/benchmark and the oracle.

This module holds random-number draws and the shapes of the workloads only; it
contains none of the method's arithmetic.  Every random number the method
consumes (which electrons hop, to which empty sites, the Metropolis uniforms)
is drawn here and passed to both sides as data.

Workloads follow the paper's synthetic benchmarks (Sec. IV: batched random
matrices, rank k = 1 hops, n up to 1024) and the physics of Sec. II.B / III.B:
an orbital matrix Phi (L sites x n orbitals) or a skew pairing matrix F
(L x L); each walker occupies n of the L sites, and a step moves k distinct
electrons to k distinct sites that were empty at the start of the step.

Complex normal CN(0, s2): real and imaginary parts iid N(0, s2/2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2602_05255


def generator(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def normal(rng: np.random.Generator, shape, complex_: bool = False, var: float = 1.0):
    """iid N(0, var) real, or CN(0, var) complex, in double precision."""
    if not complex_:
        return rng.standard_normal(shape) * np.sqrt(var)
    s = np.sqrt(var / 2.0)
    return rng.standard_normal(shape) * s + 1j * (rng.standard_normal(shape) * s)


def skew_from(g):
    """F = (G - G^T)/2: the synthetic pairing matrix of the Pfaffian workload."""
    return 0.5 * (g - g.T)


def occupancy(rng: np.random.Generator, walkers: int, sites: int, n: int):
    """Random n-subsets of the sites.

    Returns (occ [W][n], empty [W][sites-n]) as int32; occupied sites are in
    ascending order, so electron label i sits on the i-th smallest occupied site.
    """
    occ = np.empty((walkers, n), dtype=np.int32)
    emp = np.empty((walkers, sites - n), dtype=np.int32)
    for w in range(walkers):
        perm = rng.permutation(sites)
        occ[w] = np.sort(perm[:n])
        emp[w] = np.sort(perm[n:])
    return occ, emp


def hop_draws(rng: np.random.Generator, walkers: int, n: int, n_empty: int,
              ranks, k_max: int):
    """One step's proposal draws for every walker.

    k[w] is drawn uniformly from ``ranks``; elec[w][:k] are k distinct electron
    labels and slot[w][:k] k distinct indices into the walker's empty-site list.
    Entries c >= k repeat entry 0 (padding; consumers ignore them).
    """
    ranks = np.asarray(ranks, dtype=np.int32)
    k = ranks[rng.integers(0, len(ranks), size=walkers)].astype(np.int32)
    elec = np.empty((walkers, k_max), dtype=np.int32)
    slot = np.empty((walkers, k_max), dtype=np.int32)
    for w in range(walkers):
        kw = int(k[w])
        e = rng.choice(n, size=kw, replace=False)
        s = rng.choice(n_empty, size=kw, replace=False)
        elec[w, :kw] = e
        slot[w, :kw] = s
        elec[w, kw:] = e[0]
        slot[w, kw:] = s[0]
    return k, elec, slot


def _first_distinct(rng: np.random.Generator, lead, m: int, k: int):
    """For every index of the leading shape, k distinct values of range(m) drawn uniformly
    without replacement, in draw order: the first k distinct entries of an iid uniform
    sequence (sequential sampling without replacement).  Rows whose candidate sequence holds
    fewer than k distinct values are redrawn from a random permutation."""
    c = min(m, 2 * k + 8) if m > 2 * k + 8 else m
    if c == m:                                     # small ranges: a random permutation per row
        return np.argsort(rng.random(tuple(lead) + (m,)), axis=-1)[..., :k]
    cand = rng.integers(0, m, size=tuple(lead) + (c,))
    eq = cand[..., :, None] == cand[..., None, :]
    new = ~np.any(np.tril(eq, -1), axis=-1)        # not equal to any earlier candidate of the row
    pos = np.argsort(~new, axis=-1, kind="stable")[..., :k]
    out = np.take_along_axis(cand, pos, axis=-1)
    short = new.sum(axis=-1) < k
    if short.any():
        idx = np.nonzero(short)
        out[idx] = np.argsort(rng.random((len(idx[0]), m)), axis=-1)[:, :k]
    return out


def hop_draws_batch(rng: np.random.Generator, steps: int, walkers: int, n: int, n_empty: int,
                    ranks, k_max: int):
    """``steps`` steps of proposal draws at once (same distribution as hop_draws).

    k[t][w] is drawn uniformly from ``ranks``; the k_max electrons and empty-list slots
    of a walker-step are distinct uniform draws without replacement, of which the first
    k are used.  Returns int32 arrays k [steps][W], elec [steps][W][k_max],
    slot [steps][W][k_max]; entries c >= k repeat entry 0 (padding).
    """
    ranks = np.asarray(ranks, dtype=np.int32)
    k = ranks[rng.integers(0, len(ranks), size=(steps, walkers))].astype(np.int32)
    elec = _first_distinct(rng, (steps, walkers), n, k_max).astype(np.int32)
    slot = _first_distinct(rng, (steps, walkers), n_empty, k_max).astype(np.int32)
    pad = np.arange(k_max)[None, None, :] >= k[:, :, None]
    elec = np.where(pad, elec[:, :, :1], elec)
    slot = np.where(pad, slot[:, :, :1], slot)
    return k, elec.astype(np.int32), slot.astype(np.int32)


def uniforms(rng: np.random.Generator, walkers: int):
    return rng.random(walkers)


@dataclass
class Workload:
    """A named synthetic workload (one of the paper-shaped configurations)."""
    name: str
    kind: str                 # "det" or "pf"
    sites: int                # L
    n: int                    # matrix dimension (electrons)
    walkers: int
    ranks: tuple              # ranks k drawn per walker-step
    k_max: int
    delay: int                # K (0 = plain Sherman-Morrison / Woodbury)
    refresh: int              # refresh period in steps (0 = never)
    complex_: bool
    bulk: str                 # bulk dtype: "f64", "f32", "c64", "c128"
    steps: int = 0
    seed: int = SEED_BASE
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # Plain Slater LRU, FP64: Phi 64x32, 16 walkers x 200 single hops, no delay.
    "slater_n32_fp64": Workload("slater_n32_fp64", "det", 64, 32, 16, (1,), 1, 0, 0,
                                False, "f64", steps=200, seed=SEED_BASE + 1),
    # Determinant LRU at scale: Phi 512x256, 1024 walkers, k in {1,2,4}, K=16, refresh 128.
    "slater_n256_k124": Workload("slater_n256_k124", "det", 512, 256, 1024, (1, 2, 4), 4, 16, 128,
                                 False, "f64", steps=128, seed=SEED_BASE + 2),
    # Pfaffian LRU: F = (G - G^T)/2, G 1024x1024 CN(0,1); n=512; 256 walkers; K=32; refresh 64.
    "pfaffian_n512_c64": Workload("pfaffian_n512_c64", "pf", 1024, 512, 256, (1,), 1, 32, 64,
                                  True, "c64", steps=64, seed=SEED_BASE + 3),
    # Uneven batch: 4096 walkers, n in {64..1024}, L = 2n, k in {1,2,4,8}, FP32 bulk.
    "uneven_n64_1024_fp32": Workload("uneven_n64_1024_fp32", "det", 0, 0, 4096, (1, 2, 4, 8), 8, 16, 128,
                                     False, "f32", steps=128, seed=SEED_BASE + 4,
                                     extra={"sizes": (64, 128, 256, 512, 1024)}),
    # n-sweep of the single-hop determinant LRU (the shape of the paper's speedup-vs-n figure):
    # 1024 walkers, k = 1, L = 2n, n in {64 .. 1024}; one workload per n from nsweep_workload.
    "nsweep_det_k1": Workload("nsweep_det_k1", "det", 0, 0, 1024, (1,), 1, 0, 128,
                              False, "f64", steps=128, seed=SEED_BASE + 6,
                              extra={"sizes": (64, 128, 256, 512, 1024)}),
    # Delayed vs plain updates (the paper's delay-length benchmark): 16384 walkers, n = 128,
    # L = 256, single hops, 128 consecutive updates with no refresh; delay K swept.
    "delay_sweep_n128_det": Workload("delay_sweep_n128_det", "det", 256, 128, 16384, (1,), 1, 16, 0,
                                     False, "f64", steps=128, seed=SEED_BASE + 7),
    "delay_sweep_n128_pf": Workload("delay_sweep_n128_pf", "pf", 256, 128, 16384, (1,), 1, 4, 0,
                                    False, "f64", steps=128, seed=SEED_BASE + 8),
    # Differentiated log-psi: c64 Phi 1024x512 + rank-8 B C^T per sample, 512 samples.
    "logpsi_grad_n512_c64": Workload("logpsi_grad_n512_c64", "det", 1024, 512, 512, (8,), 8, 0, 0,
                                     True, "c64", seed=SEED_BASE + 5, extra={"rank": 8, "bc_var": 0.1}),
}


def nsweep_delay(n: int, kbar: float = 1.0) -> int:
    """Delay for the n-sweep: the power of two nearest (in log scale) to the byte-model
    optimum K* = sqrt(2 n / kbar), capped at 64."""
    k_star = math.sqrt(2.0 * n / kbar)
    return int(min(64, 2 ** round(math.log2(k_star))))


def nsweep_workload(n: int) -> Workload:
    """One size of the n-sweep: Phi (2n x n) N(0,1), 1024 walkers, single hops, FP64 refresh every 128."""
    base = WORKLOADS["nsweep_det_k1"]
    return Workload(f"nsweep_det_k1_n{n}", "det", 2 * n, n, base.walkers, (1,), 1, nsweep_delay(n),
                    base.refresh, False, "f64", steps=base.steps, seed=base.seed + n)


def slater_inputs(wl: Workload, walkers: int | None = None, seed_offset: int = 0):
    """(Phi [L][n], occ [W][n], empty [W][L-n]) for a uniform-n determinant workload."""
    rng = generator(wl.seed + seed_offset)
    w = wl.walkers if walkers is None else walkers
    phi = normal(rng, (wl.sites, wl.n), wl.complex_)
    occ, emp = occupancy(rng, w, wl.sites, wl.n)
    return phi, occ, emp, rng


def pairing_inputs(wl: Workload, walkers: int | None = None, seed_offset: int = 0):
    """(F [L][L] skew, occ, empty) for the Pfaffian workload."""
    rng = generator(wl.seed + seed_offset)
    w = wl.walkers if walkers is None else walkers
    f = skew_from(normal(rng, (wl.sites, wl.sites), wl.complex_))
    occ, emp = occupancy(rng, w, wl.sites, wl.n)
    return f, occ, emp, rng


def uneven_sizes(rng: np.random.Generator, walkers: int, sizes):
    """Per-walker matrix dimension drawn uniformly from ``sizes``."""
    sizes = np.asarray(sizes, dtype=np.int32)
    return sizes[rng.integers(0, len(sizes), size=walkers)]


def uneven_inputs(wl: Workload, walkers: int | None = None, seed_offset: int = 0):
    """Size classes of the uneven workload: per-walker n drawn from the size list,
    one Phi (2n x n, N(0,1)) per size, random occupancies.  Returns (classes, rng)
    with classes a list of dicts {n, phi, occ, empty, walkers} in size order."""
    rng = generator(wl.seed + seed_offset)
    w = wl.walkers if walkers is None else walkers
    sizes = uneven_sizes(rng, w, wl.extra["sizes"])
    classes = []
    for n in sorted(set(int(x) for x in sizes)):
        ids = np.nonzero(sizes == n)[0]
        phi = normal(rng, (2 * n, n))
        occ, emp = occupancy(rng, len(ids), 2 * n, n)
        classes.append({"n": n, "phi": phi, "occ": occ, "empty": emp, "walkers": ids})
    return classes, rng


def lowrank_inputs(wl: Workload, samples: int | None = None, sites: int | None = None,
                   n: int | None = None, seed_offset: int = 0):
    """Phi [L][n], occ [S][n], B, C [S][n][r] (CN(0, 0.1)), loss weights w [S] (CN(0, 1))."""
    rng = generator(wl.seed + seed_offset)
    s = wl.walkers if samples is None else samples
    L = wl.sites if sites is None else sites
    nn = wl.n if n is None else n
    r = wl.extra["rank"]
    phi = normal(rng, (L, nn), wl.complex_)
    occ, _ = occupancy(rng, s, L, nn)
    b = normal(rng, (s, nn, r), wl.complex_, wl.extra["bc_var"])
    c = normal(rng, (s, nn, r), wl.complex_, wl.extra["bc_var"])
    wts = normal(rng, (s,), wl.complex_)
    return phi, occ, b, c, wts
