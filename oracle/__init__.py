"""lrx oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU reference for the low-rank determinant
and Pfaffian updates of "lrux: Fast low-rank updates of determinants and
Pfaffians in JAX" (arXiv 2602.05255).  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it;
the product package never does, and this module imports nothing from it.

The method's results all have a plain definition:

* the determinant ratio of Sec. II.A (Eqs. det_ratio, det_R) is
  det(A_t) / det(A_{t-1});
* the Sherman-Morrison / Woodbury updates (Eqs. det_inv, pf_inv) and the
  delayed reconstructions (Eqs. delayed_Ainv, pf_delayed_Ainv) produce A_t^-1;
* the Pfaffian ratio (Eqs. pf_ratio, pf_R) is pf(A_t) / pf(A_{t-1});
* the gradient of log det M is M^-T, and that of log pf A is (1/2) A^-T
  (Appendix A, Eq. pf_grad).

So every step here recomputes from scratch: a new matrix is gathered from the
orbital (or pairing) matrix at the current occupancy, then factorised by the C
routines in ``lrx_oracle.c`` (LU with partial pivoting; Parlett-Reid).  No
delayed or low-rank logic exists in the oracle.

Conventions (readings of the paper, listed in the design notes):

* rows of the Slater matrix are electron labels fixed at initialisation:
  ``A[w][i] = Phi[occ[w][i]]``; a hop of electron i replaces row i in place;
* the Pfaffian matrix is ``A[w][i][j] = F[occ[w][i]][occ[w][j]]``;
* complex means transpose, never conjugate transpose;
* Metropolis acceptance is ``u < min(1, |r|^2)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lrx_oracle.c")
_LIB = os.path.join(_HERE, "liblrx_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP contraction off, OpenMP over batch)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.orc_slogdet.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
        lib.orc_slogdet.restype = ctypes.c_int
        lib.orc_slogpf.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        lib.orc_slogpf.restype = ctypes.c_int
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def _as_batch(a):
    a = np.asarray(a)
    squeeze = a.ndim == 2
    if squeeze:
        a = a[None]
    if a.ndim != 3 or a.shape[1] != a.shape[2]:
        raise ValueError("expected a batch of square matrices")
    cplx = np.iscomplexobj(a)
    a = np.ascontiguousarray(a, dtype=np.complex128 if cplx else np.float64)
    return a, cplx, squeeze


def _phase_out(ph, cplx):
    return ph[:, 0] + 1j * ph[:, 1] if cplx else ph[:, 0].copy()


def slogdet(a, want_inv: bool = True):
    """log|det A|, phase (sign or unit complex) and A^-1 by LU with partial pivoting.

    Singular matrices give logabs = -inf, phase 0 and a NaN inverse.
    """
    a, cplx, squeeze = _as_batch(a)
    b, n = a.shape[0], a.shape[1]
    la = np.empty(b)
    ph = np.empty((b, 2))
    inv = np.empty_like(a) if want_inv else None
    _load().orc_slogdet(int(cplx), b, n, _ptr(a), _ptr(la), _ptr(ph),
                        _ptr(inv) if want_inv else None)
    phase = _phase_out(ph, cplx)
    if squeeze:
        return la[0], phase[0], (inv[0] if want_inv else None)
    return la, phase, inv


def det(a):
    la, ph, _ = slogdet(a, want_inv=False)
    return ph * np.exp(la)


def slogpf(a):
    """log|pf A| and phase of skew-symmetric matrices by Parlett-Reid (Appendix A)."""
    a, cplx, squeeze = _as_batch(a)
    b, n = a.shape[0], a.shape[1]
    la = np.empty(b)
    ph = np.empty((b, 2))
    _load().orc_slogpf(int(cplx), b, n, _ptr(a), _ptr(la), _ptr(ph))
    phase = _phase_out(ph, cplx)
    if squeeze:
        return la[0], phase[0]
    return la, phase


def pf(a):
    la, ph = slogpf(a)
    return ph * np.exp(la)


def ratio(la_new, ph_new, la_old, ph_old):
    """det(A_t)/det(A_{t-1}) (or the Pfaffian analogue) from log-magnitudes and phases."""
    return np.exp(np.asarray(la_new) - np.asarray(la_old)) * (np.asarray(ph_new) / np.asarray(ph_old))


def skew_inverse(a):
    """Inverse of a skew-symmetric matrix by LU, then (M - M^T)/2 (exact skew symmetry)."""
    _, _, inv = slogdet(a, want_inv=True)
    return 0.5 * (inv - np.swapaxes(inv, -1, -2))


# --------------------------------------------------------------------------
# Occupancy bookkeeping for electron hops (the oracle's own copy).
# --------------------------------------------------------------------------
class Occupancy:
    """Per-walker list of occupied sites (index = electron label) and of empty sites.

    A hop moves electron ``elec[c]`` to the empty-list entry ``slot[c]`` for
    c < k; the vacated site takes that empty-list entry's place.
    """

    def __init__(self, occ, empty):
        self.occ = np.array(occ, dtype=np.int64, copy=True)
        self.empty = np.array(empty, dtype=np.int64, copy=True)

    def proposed(self, k, elec, slot):
        """Occupancy after the proposal of every walker (no state change)."""
        occ = self.occ.copy()
        for w in range(occ.shape[0]):
            for c in range(int(k[w])):
                occ[w, elec[w, c]] = self.empty[w, slot[w, c]]
        return occ

    def commit(self, k, elec, slot, accept):
        for w in range(self.occ.shape[0]):
            if not accept[w]:
                continue
            for c in range(int(k[w])):
                i, j = elec[w, c], slot[w, c]
                self.occ[w, i], self.empty[w, j] = self.empty[w, j], self.occ[w, i]


def slater_matrices(phi, occ):
    """A[w][i][:] = Phi[occ[w][i]][:] (rows labelled by electrons)."""
    return np.ascontiguousarray(np.asarray(phi)[np.asarray(occ)])


def pairing_matrices(f, occ):
    """A[w][i][j] = F[occ[w][i]][occ[w][j]]."""
    f = np.asarray(f)
    occ = np.asarray(occ)
    return np.ascontiguousarray(f[occ[:, :, None], occ[:, None, :]])


def metropolis(r, u01):
    """Accept iff u < min(1, |r|^2); a zero or non-finite ratio is rejected."""
    r = np.asarray(r)
    p = np.abs(r) ** 2
    ok = np.isfinite(p) & (p > 0)
    return ok & (np.asarray(u01) < np.minimum(1.0, np.where(ok, p, 0.0)))


class DetChain:
    """Full-recompute Slater-determinant chain: every quantity from a fresh LU."""

    def __init__(self, phi, occ0, empty0):
        self.phi = np.asarray(phi)
        self.book = Occupancy(occ0, empty0)
        self.logabs, self.phase, self.inv = slogdet(slater_matrices(self.phi, self.book.occ))

    def propose(self, k, elec, slot):
        occ = self.book.proposed(k, elec, slot)
        la, ph, inv = slogdet(slater_matrices(self.phi, occ))
        self._pending = (la, ph, inv)
        return ratio(la, ph, self.logabs, self.phase)

    def accept(self, k, elec, slot, mask):
        la, ph, inv = self._pending
        mask = np.asarray(mask, dtype=bool)
        self.logabs = np.where(mask, la, self.logabs)
        self.phase = np.where(mask, ph, self.phase)
        self.inv = np.where(mask[:, None, None], inv, self.inv)
        self.book.commit(k, elec, slot, mask)


class PfChain:
    """Full-recompute Pfaffian chain: Parlett-Reid for pf, LU for the inverse."""

    def __init__(self, f, occ0, empty0):
        self.f = np.asarray(f)
        self.book = Occupancy(occ0, empty0)
        a = pairing_matrices(self.f, self.book.occ)
        self.logabs, self.phase = slogpf(a)
        self.inv = skew_inverse(a)

    def propose(self, k, elec, slot):
        occ = self.book.proposed(k, elec, slot)
        a = pairing_matrices(self.f, occ)
        la, ph = slogpf(a)
        self._pending = (la, ph, a)
        return ratio(la, ph, self.logabs, self.phase)

    def accept(self, k, elec, slot, mask):
        la, ph, a = self._pending
        mask = np.asarray(mask, dtype=bool)
        self.logabs = np.where(mask, la, self.logabs)
        self.phase = np.where(mask, ph, self.phase)
        if mask.any():
            inv_new = skew_inverse(a[mask])
            inv = self.inv.copy()
            inv[mask] = inv_new
            self.inv = inv
        self.book.commit(k, elec, slot, mask)


def lowrank_logdet_and_grads(phi, occ, b, c):
    """log det M_s for M_s = Phi[occ_s] + B_s C_s^T, and its holomorphic gradients.

    Returns (logabs[S], phase[S], G[S][n][n], GB[S][n][r], GC[S][n][r]) where
    G = d log det M / dM = M^-T, GB = d/dB = M^-T C and GC = d/dC = M^-1 B.
    """
    a = slater_matrices(phi, occ) + np.asarray(b) @ np.swapaxes(np.asarray(c), -1, -2)
    la, ph, inv = slogdet(a)
    g = np.swapaxes(inv, -1, -2)
    return la, ph, g, g @ np.asarray(c), inv @ np.asarray(b)


def det_general_matrix(a, ev, xu, eu, xv):
    """A_1 = A_0 + v u^T for the mixed dense / one-hot tuples of Sec. II.B ("Matrix
    updates"): u = [xu | e_eu], v = [e_ev | xv], assembled as dense n x k matrices
    and multiplied out.  a [W][n][n]; ev [W][kr], xu [W][kr][n]; eu [W][kc], xv [W][kc][n]
    (kr or kc may be 0)."""
    a = np.asarray(a)
    W, n, _ = a.shape
    kr = 0 if ev is None else np.asarray(ev).shape[1]
    kc = 0 if eu is None else np.asarray(eu).shape[1]
    cplx = np.iscomplexobj(a) or (kr and np.iscomplexobj(np.asarray(xu))) or (kc and np.iscomplexobj(np.asarray(xv)))
    out = a.astype(np.complex128 if cplx else np.float64)
    for w in range(W):
        u = np.zeros((n, kr + kc), dtype=out.dtype)
        v = np.zeros_like(u)
        for c in range(kr):
            u[:, c] = xu[w][c]
            v[ev[w][c], c] = 1.0
        for e in range(kc):
            u[eu[w][e], kr + e] = 1.0
            v[:, kr + e] = xv[w][e]
        out[w] = out[w] + v @ u.T
    return out


def pf_general_matrix(a, cols, x):
    """A_1 = A_0 - u J u^T with u = [x | e_cols] (Sec. III.B, update of k rows and k
    columns), assembled as a dense n x 2k matrix and multiplied out."""
    a = np.asarray(a)
    x = np.asarray(x)
    W, n, _ = a.shape
    k = np.asarray(cols).shape[1]
    jm = skew_eye(k)
    out = a.copy()
    for w in range(W):
        u = np.zeros((n, 2 * k), dtype=np.result_type(a, x))
        for c in range(k):
            u[:, c] = x[w][c]
            u[cols[w][c], k + c] = 1.0
        out[w] = a[w] - u @ jm @ u.T
    return out


def skew_eye(k):
    """The 2k x 2k skew identity J = [[0, 1], [-1, 0]] (blocks of size k) of Sec. III.A."""
    j = np.zeros((2 * k, 2 * k))
    j[:k, k:] = np.eye(k)
    j[k:, :k] = -np.eye(k)
    return j


def lowrank_logpf_and_grads(f, occ, u):
    """log pf M_s for M_s = F[occ_s][:, occ_s] - U_s J U_s^T (the low-rank skew update of
    Sec. III.A) and its holomorphic gradients.

    Returns (logabs[S], phase[S], G[S][n][n], GU[S][n][2k]) with G = d log pf M / dM,
    G_ij = (1/2) (M^-1)_ji (Appendix A, Eq. pf_grad), and GU = d log pf M / dU by the
    chain rule through M_kl = A_kl - sum_cd U_kc J_cd U_ld:
    GU = -(G U J^T) - (G^T U J).  Every quantity comes from a fresh Parlett-Reid
    Pfaffian and LU inverse of M.
    """
    u = np.asarray(u)
    k = u.shape[-1] // 2
    jm = skew_eye(k)
    m = pairing_matrices(f, occ) - u @ jm @ np.swapaxes(u, -1, -2)
    la, ph = slogpf(m)
    _, _, inv = slogdet(m)
    g = 0.5 * np.swapaxes(inv, -1, -2)
    gu = -(g @ u @ jm.T) - (np.swapaxes(g, -1, -2) @ u @ jm)
    return la, ph, g, gu


def scatter_pairs(g, occ, n_sites):
    """dF[a][b] = sum over (walker, i, j with occ_i = a, occ_j = b) of G[w][i][j] (adjoint of
    the gather A[w][i][j] = F[occ[w][i]][occ[w][j]])."""
    g = np.asarray(g)
    occ = np.asarray(occ)
    out = np.zeros((n_sites, n_sites), dtype=g.dtype)
    for w in range(occ.shape[0]):
        out[np.ix_(occ[w], occ[w])] += g[w]
    return out


def scatter_rows(g, occ, n_sites):
    """dPhi[s] = sum over (walker, electron i with occ = s) of G[w][i] (adjoint of the gather)."""
    g = np.asarray(g)
    out = np.zeros((n_sites, g.shape[-1]), dtype=g.dtype)
    occ = np.asarray(occ)
    for w in range(occ.shape[0]):
        for i in range(occ.shape[1]):
            out[occ[w, i]] += g[w, i]
    return out
