"""Python binding of liblrx (ctypes).  Argument marshalling only.

Every function here has the name of the C entry point it wraps (see
``include/lrx.h``), takes torch tensors that already live on the GPU, checks
their dtype/shape/contiguity, and passes raw device pointers plus the current
HIP stream.  All arithmetic runs in the HIP kernels of ``liblrx.so``; there is
no fallback: importing this module raises if the library is missing.

``State`` allocates the caller-owned device buffers of one walker batch with
torch (the library itself never allocates) and keeps the C ``lrx_state``.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblrx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"liblrx.so not built at {LIB_PATH}: run `python -m paper_2602_05255_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# Constants mirrored from lrx.h.
LRX_OK, LRX_EINVAL, LRX_EUNSUPPORTED, LRX_ESHAPE, LRX_ENEEDFLUSH, LRX_EODD, LRX_EHIP, LRX_EKIND = range(8)
LRX_DET, LRX_PF = 0, 1
LRX_F32, LRX_F64, LRX_C64, LRX_C128 = 0, 1, 2, 3
LRX_FLAG_SINGULAR_R, LRX_FLAG_NONFINITE, LRX_FLAG_SINGULAR_A, LRX_FLAG_BADINDEX = 1, 2, 4, 8
LRX_MH_UNIFORMS, LRX_MH_DEVICE_RNG, LRX_MH_FORCE, LRX_MH_MASK = 0, 1, 2, 3
LRX_MAX_N, LRX_MAX_KMAX_DET, LRX_MAX_KMAX_PF, LRX_MAX_DELAY = 1024, 8, 4, 64
LRX_MAX_CLASSES = 8
LRX_LAYOUT_FULL, LRX_LAYOUT_FUSED, LRX_LAYOUT_PACKED = 0, 1, 2
LRX_PACK_TILE = 64
LRX_MAX_WINDOW_STEPS = 256
LRX_NOALLOC_SCRATCH_WORDS = 64

DTYPE_CODE = {torch.float32: LRX_F32, torch.float64: LRX_F64,
              torch.complex64: LRX_C64, torch.complex128: LRX_C128}
CODE_DTYPE = {v: k for k, v in DTYPE_CODE.items()}
WIDE = {LRX_F32: torch.float64, LRX_F64: torch.float64,
        LRX_C64: torch.complex128, LRX_C128: torch.complex128}


class lrx_shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32), ("walkers", ctypes.c_int32),
                ("n", ctypes.c_int32), ("k_max", ctypes.c_int32), ("delay", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class lrx_sizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_size_t) for f in
                ("inv", "fa", "fb", "stash", "logabs", "phase", "flags", "work", "stash_stride")]


class lrx_state(ctypes.Structure):
    _fields_ = [("shape", lrx_shape), ("slot", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("inv", ctypes.c_void_p), ("fa", ctypes.c_void_p), ("fb", ctypes.c_void_p),
                ("stash", ctypes.c_void_p), ("logabs", ctypes.c_void_p), ("phase", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("work", ctypes.c_void_p)]


class lrx_tune(ctypes.Structure):
    _fields_ = [("delay", ctypes.c_int32), ("rows_per_block", ctypes.c_int32), ("wgs_per_cu", ctypes.c_int32),
                ("window", ctypes.c_int32), ("tuned", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lrx_window_class(ctypes.Structure):
    _fields_ = [("state", ctypes.POINTER(lrx_state)), ("table", ctypes.c_void_p), ("sites", ctypes.c_int32),
                ("n_empty", ctypes.c_int32), ("occ", ctypes.c_void_p), ("empty", ctypes.c_void_p),
                ("k", ctypes.c_void_p), ("elec", ctypes.c_void_p), ("slot", ctypes.c_void_p),
                ("u01", ctypes.c_void_p), ("u", ctypes.c_void_p), ("ratio", ctypes.c_void_p),
                ("accept", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "lrx_version": ([], ctypes.c_int),
    "lrx_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "lrx_state_sizes": ([ctypes.POINTER(lrx_shape), ctypes.POINTER(lrx_sizes)], ctypes.c_int),
    "lrx_validate": ([ctypes.POINTER(lrx_state)], ctypes.c_int),
    "lrx_det_init_inverse": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P], ctypes.c_int),
    "lrx_det_refresh": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P, _P], ctypes.c_int),
    "lrx_det_build_hop": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P, _I, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_det_propose_ratio": ([ctypes.POINTER(lrx_state), _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_det_accept_update": ([ctypes.POINTER(lrx_state), _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_det_flush_delayed": ([ctypes.POINTER(lrx_state), _P], ctypes.c_int),
    "lrx_det_propose_hop": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P, _I, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_det_accept_hop": ([ctypes.POINTER(lrx_state), _P, _P, _P, _P, _I, _P, ctypes.c_uint64, ctypes.c_uint64,
                            _P, _P, _P, _I, _P], ctypes.c_int),
    "lrx_det_lowrank_fwd": ([ctypes.POINTER(lrx_state), _I, _P, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_det_lowrank_work_bytes": ([ctypes.POINTER(lrx_shape), _I, _I, ctypes.POINTER(ctypes.c_size_t)],
                                   ctypes.c_int),
    "lrx_det_lowrank_bwd": ([ctypes.POINTER(lrx_state), _I, _P, _I, _P, _P, _P, _P, _P, _P, _P, _P,
                             ctypes.c_size_t, _P], ctypes.c_int),
    "lrx_pf_lowrank_fwd": ([ctypes.POINTER(lrx_state), _I, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_lowrank_work_bytes": ([ctypes.POINTER(lrx_shape), _I, _I, ctypes.POINTER(ctypes.c_size_t)],
                                  ctypes.c_int),
    "lrx_pf_lowrank_bwd": ([ctypes.POINTER(lrx_state), _I, _P, _I, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P],
                           ctypes.c_int),
    "lrx_pf_grad": ([ctypes.POINTER(lrx_state), _P, _P, _P], ctypes.c_int),
    "lrx_pf_init_inverse": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P], ctypes.c_int),
    "lrx_pf_refresh": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P, _P], ctypes.c_int),
    "lrx_pf_build_hop": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P, _I, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_propose_ratio": ([ctypes.POINTER(lrx_state), _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_accept_update": ([ctypes.POINTER(lrx_state), _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_propose_hop": ([ctypes.POINTER(lrx_state), _P, _I, _P, _P, _I, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_accept_hop": ([ctypes.POINTER(lrx_state), _P, _P, _P, _P, _I, _P, ctypes.c_uint64, ctypes.c_uint64,
                           _P, _P, _P, _I, _P], ctypes.c_int),
    "lrx_pf_flush_delayed": ([ctypes.POINTER(lrx_state), _P], ctypes.c_int),
    "lrx_pf_read_inverse": ([ctypes.POINTER(lrx_state), _P, _P], ctypes.c_int),
    "lrx_det_propose_general": ([ctypes.POINTER(lrx_state), _I, _P, _P, _I, _P, _P, _P, _P], ctypes.c_int),
    "lrx_det_accept_general": ([ctypes.POINTER(lrx_state), _I, _P, _P, _I, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_propose_general": ([ctypes.POINTER(lrx_state), _I, _P, _P, _P, _P], ctypes.c_int),
    "lrx_pf_accept_general": ([ctypes.POINTER(lrx_state), _I, _P, _P, _P, _P], ctypes.c_int),
    "lrx_metropolis": ([ctypes.POINTER(lrx_state), _P, _P, ctypes.c_uint64, ctypes.c_uint64, _I, _P, _P],
                       ctypes.c_int),
    "lrx_hop_commit": ([_I, _I, _I, _I, _P, _P, _P, _P, _P, _P, _P], ctypes.c_int),
    "lrx_autotune_store": ([_I, _I, _I, ctypes.POINTER(lrx_tune)], ctypes.c_int),
    "lrx_autotune_lookup": ([_I, _I, _I, ctypes.POINTER(lrx_tune)], ctypes.c_int),
    "lrx_det_window_noalloc": ([ctypes.POINTER(lrx_window_class), _I, _I, _I, ctypes.c_uint64, ctypes.c_uint64,
                                _I, _P], ctypes.c_int),
    "lrx_window_work_bytes": ([ctypes.POINTER(lrx_window_class), _I, ctypes.POINTER(ctypes.c_size_t)],
                              ctypes.c_int),
    "lrx_det_window": ([ctypes.POINTER(lrx_window_class), _I, _I, _I, ctypes.c_uint64, ctypes.c_uint64, _P,
                        ctypes.c_size_t, _I, _P], ctypes.c_int),
}
for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


class LrxError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lrx_strerror(code)} (code {code})")


def _check(rc, where):
    if rc != LRX_OK:
        raise LrxError(rc, where)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, name, dtype=None, shape=None, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------------------
def lrx_version() -> int:
    return int(_lib.lrx_version())


def lrx_strerror(code: int) -> str:
    return _lib.lrx_strerror(int(code)).decode()


def lrx_state_sizes(kind, dtype, walkers, n, k_max, delay, layout=0):
    """Byte sizes of the state buffers (host only; raises LrxError for bad shapes)."""
    shp = lrx_shape(kind, dtype, walkers, n, k_max, delay, layout)
    out = lrx_sizes()
    _check(_lib.lrx_state_sizes(ctypes.byref(shp), ctypes.byref(out)), "lrx_state_sizes")
    return {f: getattr(out, f) for f, _ in lrx_sizes._fields_}


class State:
    """Device buffers of one walker batch plus the C state (caller-owned memory)."""

    def __init__(self, kind, dtype, walkers, n, k_max=1, delay=0, device="cuda", layout=0):
        code = DTYPE_CODE[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
        self.sizes = lrx_state_sizes(kind, code, walkers, n, k_max, delay, layout)
        self.kind, self.code, self.dtype = kind, code, CODE_DTYPE[code]
        self.walkers, self.n, self.k_max, self.delay, self.layout = walkers, n, k_max, delay, layout
        dev = torch.device(device)
        self.buffers = {}
        for name in ("inv", "fa", "fb", "stash", "logabs", "phase", "flags", "work"):
            nbytes = max(int(self.sizes[name]), 256)
            self.buffers[name] = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.buffers["flags"].zero_()
        ptr = {k: ctypes.c_void_p(v.data_ptr()) for k, v in self.buffers.items()}
        self.c = lrx_state(lrx_shape(kind, code, walkers, n, k_max, delay, layout), 0, 0,
                           ptr["inv"], ptr["fa"], ptr["fb"], ptr["stash"], ptr["logabs"], ptr["phase"],
                           ptr["flags"], ptr["work"])
        _check(_lib.lrx_validate(ctypes.byref(self.c)), "lrx_validate")

    # Typed views of the device state.
    @property
    def inv(self):
        """M0 as stored: [W][n][n], or [W][tiles][64][64] for the packed layout."""
        v = self.buffers["inv"][: self.sizes["inv"]].view(self.dtype)
        if self.layout == LRX_LAYOUT_PACKED:
            return v.view(self.walkers, -1, LRX_PACK_TILE, LRX_PACK_TILE)
        return v.view(self.walkers, self.n, self.n)

    @property
    def logabs(self):
        return self.buffers["logabs"][: self.sizes["logabs"]].view(torch.float64)

    @property
    def phase(self):
        return self.buffers["phase"][: self.sizes["phase"]].view(WIDE[self.code])

    @property
    def flags(self):
        return self.buffers["flags"][: self.sizes["flags"]].view(torch.int32)

    @property
    def slot(self):
        return int(self.c.slot)

    @property
    def wide(self):
        return WIDE[self.code]

    def ptr(self):
        return ctypes.byref(self.c)


def _kvec(st, k, rows, name="rows"):
    _dev(k, "k", torch.int32, (st.walkers,))
    _dev(rows, name, torch.int32, (st.walkers, st.k_max))


# ------------------------------------------------------------------ DET
def lrx_det_init_inverse(st: State, phi, sites, occ, stream=None):
    pocc = _dev(occ, "occ", torch.int32, (st.walkers, st.n), allow_none=True)
    pphi = _dev(phi, "phi", st.wide)
    _check(_lib.lrx_det_init_inverse(st.ptr(), pphi, int(sites), pocc, _stream(stream)), "lrx_det_init_inverse")


def lrx_det_refresh(st: State, phi, sites, occ, report=None, stream=None):
    pocc = _dev(occ, "occ", torch.int32, (st.walkers, st.n), allow_none=True)
    prep = _dev(report, "report", torch.float64, (st.walkers, 2), allow_none=True)
    _check(_lib.lrx_det_refresh(st.ptr(), _dev(phi, "phi", st.wide), int(sites), pocc, prep, _stream(stream)),
           "lrx_det_refresh")


def lrx_det_build_hop(st: State, phi, sites, occ, empty, n_empty, k, elec, slot, u, stream=None):
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(empty, "empty", torch.int32, (st.walkers, n_empty))
    _kvec(st, k, elec, "elec")
    _dev(slot, "slot", torch.int32, (st.walkers, st.k_max))
    _dev(u, "u", st.dtype, (st.walkers, st.k_max, st.n))
    _check(_lib.lrx_det_build_hop(st.ptr(), _dev(phi, "phi", st.wide), int(sites), _dev(occ, "occ"),
                                  _dev(empty, "empty"), int(n_empty), _dev(k, "k"), _dev(elec, "elec"),
                                  _dev(slot, "slot"), _dev(u, "u"), _stream(stream)), "lrx_det_build_hop")


def lrx_det_propose_ratio(st: State, k, rows, u, ratio, stream=None):
    _kvec(st, k, rows)
    _dev(u, "u", st.dtype, (st.walkers, st.k_max, st.n))
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    _check(_lib.lrx_det_propose_ratio(st.ptr(), _dev(k, "k"), _dev(rows, "rows"), _dev(u, "u"),
                                      _dev(ratio, "ratio"), _stream(stream)), "lrx_det_propose_ratio")


def lrx_det_accept_update(st: State, k, rows, u, accept, stream=None):
    _kvec(st, k, rows)
    _dev(u, "u", st.dtype, (st.walkers, st.k_max, st.n))
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _check(_lib.lrx_det_accept_update(st.ptr(), _dev(k, "k"), _dev(rows, "rows"), _dev(u, "u"),
                                      _dev(accept, "accept"), _stream(stream)), "lrx_det_accept_update")


def lrx_det_propose_hop(st: State, phi, sites, occ, empty, n_empty, k, elec, slot, u, ratio, stream=None):
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(empty, "empty", torch.int32, (st.walkers, n_empty))
    _kvec(st, k, elec, "elec")
    _dev(slot, "slot", torch.int32, (st.walkers, st.k_max))
    _dev(u, "u", st.dtype, (st.walkers, st.k_max, st.n))
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    _check(_lib.lrx_det_propose_hop(st.ptr(), _dev(phi, "phi", st.wide), int(sites), _dev(occ, "occ"),
                                    _dev(empty, "empty"), int(n_empty), _dev(k, "k"), _dev(elec, "elec"),
                                    _dev(slot, "slot"), _dev(u, "u"), _dev(ratio, "ratio"), _stream(stream)),
           "lrx_det_propose_hop")


def lrx_det_accept_hop(st: State, k, elec, slot, u, mode, u01, seed, counter, accept, occ, empty, n_empty,
                       stream=None):
    _kvec(st, k, elec, "elec")
    _dev(slot, "slot", torch.int32, (st.walkers, st.k_max))
    _dev(u, "u", st.dtype, (st.walkers, st.k_max, st.n))
    pu = _dev(u01, "u01", torch.float64, (st.walkers,), allow_none=True)
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(empty, "empty", torch.int32, (st.walkers, n_empty))
    _check(_lib.lrx_det_accept_hop(st.ptr(), _dev(k, "k"), _dev(elec, "elec"), _dev(slot, "slot"), _dev(u, "u"),
                                   int(mode), pu, ctypes.c_uint64(seed), ctypes.c_uint64(counter),
                                   _dev(accept, "accept"), _dev(occ, "occ"), _dev(empty, "empty"), int(n_empty),
                                   _stream(stream)), "lrx_det_accept_hop")


def lrx_det_flush_delayed(st: State, stream=None):
    _check(_lib.lrx_det_flush_delayed(st.ptr(), _stream(stream)), "lrx_det_flush_delayed")


# ------------------------------------------------------------------ low-rank log det
def lrx_det_lowrank_fwd(st: State, r, B, C, P, Q, Rinv, logabs, phase, stream=None):
    shp = (st.walkers, st.n, r)
    for t, nm in ((B, "B"), (C, "C"), (P, "P"), (Q, "Q")):
        _dev(t, nm, st.dtype, shp)
    _dev(Rinv, "Rinv", st.dtype, (st.walkers, r, r))
    _dev(logabs, "logabs", torch.float64, (st.walkers,))
    _dev(phase, "phase", st.wide, (st.walkers,))
    _check(_lib.lrx_det_lowrank_fwd(st.ptr(), int(r), _dev(B, "B"), _dev(C, "C"), _dev(P, "P"), _dev(Q, "Q"),
                                    _dev(Rinv, "Rinv"), _dev(logabs, "logabs"), _dev(phase, "phase"),
                                    _stream(stream)), "lrx_det_lowrank_fwd")


def lrx_det_lowrank_work_bytes(st: State, r, sites) -> int:
    out = ctypes.c_size_t()
    _check(_lib.lrx_det_lowrank_work_bytes(ctypes.byref(st.c.shape), int(r), int(sites), ctypes.byref(out)),
           "lrx_det_lowrank_work_bytes")
    return int(out.value)


def lrx_det_lowrank_bwd(st: State, r, occ, sites, P, Q, Rinv, g, dphi, dB, dC, work, stream=None):
    shp = (st.walkers, st.n, r)
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    for t, nm in ((P, "P"), (Q, "Q"), (dB, "dB"), (dC, "dC")):
        _dev(t, nm, st.dtype, shp)
    _dev(Rinv, "Rinv", st.dtype, (st.walkers, r, r))
    _dev(g, "g", st.wide, (st.walkers,))
    _dev(dphi, "dphi", st.dtype, (sites, st.n))
    _dev(work, "work", torch.uint8)
    _check(_lib.lrx_det_lowrank_bwd(st.ptr(), int(r), _dev(occ, "occ"), int(sites), _dev(P, "P"), _dev(Q, "Q"),
                                    _dev(Rinv, "Rinv"), _dev(g, "g"), _dev(dphi, "dphi"), _dev(dB, "dB"),
                                    _dev(dC, "dC"), _dev(work, "work"), ctypes.c_size_t(work.numel()),
                                    _stream(stream)), "lrx_det_lowrank_bwd")


def lrx_pf_lowrank_fwd(st: State, r, U, P, Rinv, logabs, phase, stream=None):
    shp = (st.walkers, st.n, r)
    _dev(U, "U", st.dtype, shp)
    _dev(P, "P", st.dtype, shp)
    _dev(Rinv, "Rinv", st.dtype, (st.walkers, r, r))
    _dev(logabs, "logabs", torch.float64, (st.walkers,))
    _dev(phase, "phase", st.wide, (st.walkers,))
    _check(_lib.lrx_pf_lowrank_fwd(st.ptr(), int(r), _dev(U, "U"), _dev(P, "P"), _dev(Rinv, "Rinv"),
                                   _dev(logabs, "logabs"), _dev(phase, "phase"), _stream(stream)),
           "lrx_pf_lowrank_fwd")


def lrx_pf_lowrank_work_bytes(st: State, r, sites) -> int:
    out = ctypes.c_size_t()
    _check(_lib.lrx_pf_lowrank_work_bytes(ctypes.byref(st.c.shape), int(r), int(sites), ctypes.byref(out)),
           "lrx_pf_lowrank_work_bytes")
    return int(out.value)


def lrx_pf_lowrank_bwd(st: State, r, occ, sites, P, Rinv, g, dF, dU, work, stream=None):
    shp = (st.walkers, st.n, r)
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(P, "P", st.dtype, shp)
    _dev(dU, "dU", st.dtype, shp)
    _dev(Rinv, "Rinv", st.dtype, (st.walkers, r, r))
    _dev(g, "g", st.wide, (st.walkers,))
    _dev(dF, "dF", st.dtype, (sites, sites))
    _dev(work, "work", torch.uint8)
    _check(_lib.lrx_pf_lowrank_bwd(st.ptr(), int(r), _dev(occ, "occ"), int(sites), _dev(P, "P"), _dev(Rinv, "Rinv"),
                                   _dev(g, "g"), _dev(dF, "dF"), _dev(dU, "dU"), _dev(work, "work"),
                                   ctypes.c_size_t(work.numel()), _stream(stream)), "lrx_pf_lowrank_bwd")


def lrx_pf_grad(st: State, g, dA, stream=None):
    _dev(g, "g", st.wide, (st.walkers,))
    _dev(dA, "dA", st.dtype, (st.walkers, st.n, st.n))
    _check(_lib.lrx_pf_grad(st.ptr(), _dev(g, "g"), _dev(dA, "dA"), _stream(stream)), "lrx_pf_grad")


# ------------------------------------------------------------------ PF
def lrx_pf_init_inverse(st: State, f, sites, occ, stream=None):
    pocc = _dev(occ, "occ", torch.int32, (st.walkers, st.n), allow_none=True)
    _check(_lib.lrx_pf_init_inverse(st.ptr(), _dev(f, "f", st.wide), int(sites), pocc, _stream(stream)),
           "lrx_pf_init_inverse")


def lrx_pf_refresh(st: State, f, sites, occ, report=None, stream=None):
    pocc = _dev(occ, "occ", torch.int32, (st.walkers, st.n), allow_none=True)
    prep = _dev(report, "report", torch.float64, (st.walkers, 2), allow_none=True)
    _check(_lib.lrx_pf_refresh(st.ptr(), _dev(f, "f", st.wide), int(sites), pocc, prep, _stream(stream)),
           "lrx_pf_refresh")


def lrx_pf_build_hop(st: State, f, sites, occ, empty, n_empty, k, elec, slot, x, stream=None):
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(empty, "empty", torch.int32, (st.walkers, n_empty))
    _kvec(st, k, elec, "elec")
    _dev(slot, "slot", torch.int32, (st.walkers, st.k_max))
    _dev(x, "x", st.dtype, (st.walkers, st.n))
    _check(_lib.lrx_pf_build_hop(st.ptr(), _dev(f, "f", st.wide), int(sites), _dev(occ, "occ"),
                                 _dev(empty, "empty"), int(n_empty), _dev(k, "k"), _dev(elec, "elec"),
                                 _dev(slot, "slot"), _dev(x, "x"), _stream(stream)), "lrx_pf_build_hop")


def lrx_pf_propose_ratio(st: State, k, cols, x, ratio, stream=None):
    _kvec(st, k, cols, "cols")
    _dev(x, "x", st.dtype, (st.walkers, st.n))
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    _check(_lib.lrx_pf_propose_ratio(st.ptr(), _dev(k, "k"), _dev(cols, "cols"), _dev(x, "x"),
                                     _dev(ratio, "ratio"), _stream(stream)), "lrx_pf_propose_ratio")


def lrx_pf_accept_update(st: State, k, cols, x, accept, stream=None):
    _kvec(st, k, cols, "cols")
    _dev(x, "x", st.dtype, (st.walkers, st.n))
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _check(_lib.lrx_pf_accept_update(st.ptr(), _dev(k, "k"), _dev(cols, "cols"), _dev(x, "x"),
                                     _dev(accept, "accept"), _stream(stream)), "lrx_pf_accept_update")


def lrx_pf_propose_hop(st: State, f, sites, occ, empty, n_empty, k, cols, slot, x, ratio, stream=None):
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(empty, "empty", torch.int32, (st.walkers, n_empty))
    _kvec(st, k, cols, "cols")
    _dev(slot, "slot", torch.int32, (st.walkers, st.k_max))
    _dev(x, "x", st.dtype, (st.walkers, st.n))
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    _check(_lib.lrx_pf_propose_hop(st.ptr(), _dev(f, "f", st.wide), int(sites), _dev(occ, "occ"),
                                   _dev(empty, "empty"), int(n_empty), _dev(k, "k"), _dev(cols, "cols"),
                                   _dev(slot, "slot"), _dev(x, "x"), _dev(ratio, "ratio"), _stream(stream)),
           "lrx_pf_propose_hop")


def lrx_pf_accept_hop(st: State, k, cols, slot, x, mode, u01, seed, counter, accept, occ, empty, n_empty,
                      stream=None):
    _kvec(st, k, cols, "cols")
    _dev(slot, "slot", torch.int32, (st.walkers, st.k_max))
    _dev(x, "x", st.dtype, (st.walkers, st.n))
    pu = _dev(u01, "u01", torch.float64, (st.walkers,), allow_none=True)
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _dev(occ, "occ", torch.int32, (st.walkers, st.n))
    _dev(empty, "empty", torch.int32, (st.walkers, n_empty))
    _check(_lib.lrx_pf_accept_hop(st.ptr(), _dev(k, "k"), _dev(cols, "cols"), _dev(slot, "slot"), _dev(x, "x"),
                                  int(mode), pu, ctypes.c_uint64(seed), ctypes.c_uint64(counter),
                                  _dev(accept, "accept"), _dev(occ, "occ"), _dev(empty, "empty"), int(n_empty),
                                  _stream(stream)), "lrx_pf_accept_hop")


def lrx_pf_flush_delayed(st: State, stream=None):
    _check(_lib.lrx_pf_flush_delayed(st.ptr(), _stream(stream)), "lrx_pf_flush_delayed")


def lrx_pf_read_inverse(st: State, out, stream=None):
    """out: device bulk dtype [W][n][n] <- A^-1 of every walker (any layout, state unchanged)."""
    po = _dev(out, "out", st.dtype, (st.walkers, st.n, st.n))
    _check(_lib.lrx_pf_read_inverse(st.ptr(), po, _stream(stream)), "lrx_pf_read_inverse")


# ------------------------------------------------------------------ chain helpers
def _general_det_args(st, ev, xu, eu, xv):
    kr = 0 if ev is None else int(ev.shape[1])
    kc = 0 if eu is None else int(eu.shape[1])
    pev = _dev(ev, "ev", torch.int32, (st.walkers, kr), allow_none=True) if kr else None
    pxu = _dev(xu, "xu", st.dtype, (st.walkers, kr, st.n), allow_none=True) if kr else None
    peu = _dev(eu, "eu", torch.int32, (st.walkers, kc), allow_none=True) if kc else None
    pxv = _dev(xv, "xv", st.dtype, (st.walkers, kc, st.n), allow_none=True) if kc else None
    return kr, pev, pxu, kc, peu, pxv


def lrx_det_propose_general(st: State, ev, xu, eu, xv, ratio, stream=None):
    """ev: int32 [W][kr] rows, xu [W][kr][n] (or both None); eu: int32 [W][kc] columns,
    xv [W][kc][n] (or both None)."""
    kr, pev, pxu, kc, peu, pxv = _general_det_args(st, ev, xu, eu, xv)
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    _check(_lib.lrx_det_propose_general(st.ptr(), kr, pev, pxu, kc, peu, pxv, _dev(ratio, "ratio"),
                                        _stream(stream)), "lrx_det_propose_general")


def lrx_det_accept_general(st: State, ev, xu, eu, xv, accept, stream=None):
    kr, pev, pxu, kc, peu, pxv = _general_det_args(st, ev, xu, eu, xv)
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _check(_lib.lrx_det_accept_general(st.ptr(), kr, pev, pxu, kc, peu, pxv, _dev(accept, "accept"),
                                       _stream(stream)), "lrx_det_accept_general")


def lrx_pf_propose_general(st: State, cols, x, ratio, stream=None):
    """cols: int32 [W][k]; x: [W][k][n]."""
    k = int(cols.shape[1])
    _dev(cols, "cols", torch.int32, (st.walkers, k))
    _dev(x, "x", st.dtype, (st.walkers, k, st.n))
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    _check(_lib.lrx_pf_propose_general(st.ptr(), k, _dev(cols, "cols"), _dev(x, "x"), _dev(ratio, "ratio"),
                                       _stream(stream)), "lrx_pf_propose_general")


def lrx_pf_accept_general(st: State, cols, x, accept, stream=None):
    k = int(cols.shape[1])
    _dev(cols, "cols", torch.int32, (st.walkers, k))
    _dev(x, "x", st.dtype, (st.walkers, k, st.n))
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _check(_lib.lrx_pf_accept_general(st.ptr(), k, _dev(cols, "cols"), _dev(x, "x"), _dev(accept, "accept"),
                                      _stream(stream)), "lrx_pf_accept_general")


def lrx_metropolis(st: State, ratio, u01, seed, counter, mode, accept, stream=None):
    _dev(ratio, "ratio", st.wide, (st.walkers,))
    pu = _dev(u01, "u01", torch.float64, (st.walkers,), allow_none=True)
    _dev(accept, "accept", torch.uint8, (st.walkers,))
    _check(_lib.lrx_metropolis(st.ptr(), _dev(ratio, "ratio"), pu, ctypes.c_uint64(seed),
                               ctypes.c_uint64(counter), int(mode), _dev(accept, "accept"), _stream(stream)),
           "lrx_metropolis")


def lrx_hop_commit(walkers, n, n_empty, k_max, k, elec, slot, accept, occ, empty, stream=None):
    _dev(k, "k", torch.int32, (walkers,))
    _dev(elec, "elec", torch.int32, (walkers, k_max))
    _dev(slot, "slot", torch.int32, (walkers, k_max))
    _dev(accept, "accept", torch.uint8, (walkers,))
    _dev(occ, "occ", torch.int32, (walkers, n))
    _dev(empty, "empty", torch.int32, (walkers, n_empty))
    _check(_lib.lrx_hop_commit(int(walkers), int(n), int(n_empty), int(k_max), _dev(k, "k"), _dev(elec, "elec"),
                               _dev(slot, "slot"), _dev(accept, "accept"), _dev(occ, "occ"),
                               _dev(empty, "empty"), _stream(stream)), "lrx_hop_commit")


# ------------------------------------------------------------------ uneven window
class WindowClass:
    """Device buffers of one size class for lrx_det_window.

    st: State (DET, FP32/FP64, delay >= 1); table: phi [sites][n] FP64; occ/empty:
    int32 [W][n] / [W][n_empty]; k: int32 [steps][W]; elec/slot: int32
    [steps][W][k_max]; u: bulk [W][k_max][n]; ratio: float64 [steps][W]; accept:
    uint8 [steps][W]; u01: float64 [steps][W] or None.
    """

    def __init__(self, st, table, occ, empty, k, elec, slot, u, ratio, accept, u01=None):
        self.st, self.table, self.occ, self.empty = st, table, occ, empty
        self.k, self.elec, self.slot, self.u, self.ratio, self.accept, self.u01 = k, elec, slot, u, ratio, accept, u01

    def c_struct(self, steps):
        st = self.st
        W, KM, n = st.walkers, st.k_max, st.n
        n_empty = int(self.empty.shape[1])
        _dev(self.table, "table", torch.float64)
        _dev(self.occ, "occ", torch.int32, (W, n))
        _dev(self.empty, "empty", torch.int32, (W, n_empty))
        _dev(self.k, "k", torch.int32, (steps, W))
        _dev(self.elec, "elec", torch.int32, (steps, W, KM))
        _dev(self.slot, "slot", torch.int32, (steps, W, KM))
        _dev(self.u, "u", st.dtype, (W, KM, n))
        _dev(self.ratio, "ratio", torch.float64, (steps, W))
        _dev(self.accept, "accept", torch.uint8, (steps, W))
        pu = _dev(self.u01, "u01", torch.float64, (steps, W), allow_none=True)
        return lrx_window_class(ctypes.pointer(st.c), self.table.data_ptr(), int(self.table.shape[0]), n_empty,
                                self.occ.data_ptr(), self.empty.data_ptr(), self.k.data_ptr(),
                                self.elec.data_ptr(), self.slot.data_ptr(), pu, self.u.data_ptr(),
                                self.ratio.data_ptr(), self.accept.data_ptr())


def _class_array(classes, steps):
    arr = (lrx_window_class * len(classes))()
    for i, c in enumerate(classes):
        arr[i] = c.c_struct(steps) if isinstance(c, WindowClass) else c
    return arr


def lrx_window_work_bytes(classes, steps=1) -> int:
    arr = _class_array(classes, steps)
    out = ctypes.c_size_t()
    _check(_lib.lrx_window_work_bytes(arr, len(classes), ctypes.byref(out)), "lrx_window_work_bytes")
    return int(out.value)


def lrx_det_window(classes, steps, mode, seed, counter, work, grid, stream=None):
    arr = _class_array(classes, steps)
    _dev(work, "work", torch.uint8)
    _check(_lib.lrx_det_window(arr, len(classes), int(steps), int(mode), ctypes.c_uint64(seed),
                               ctypes.c_uint64(counter), _dev(work, "work"), int(work.numel()), int(grid),
                               _stream(stream)), "lrx_det_window")


def lrx_det_window_noalloc(classes, steps, mode, seed, counter, grid, stream=None):
    """lrx_det_window with the library's own counters (no workspace argument)."""
    arr = _class_array(classes, steps)
    _check(_lib.lrx_det_window_noalloc(arr, len(classes), int(steps), int(mode), ctypes.c_uint64(seed),
                                       ctypes.c_uint64(counter), int(grid), _stream(stream)),
           "lrx_det_window_noalloc")


# ------------------------------------------------------------------ tuning table
def lrx_autotune_store(dtype, n, k_max, delay, rows_per_block=0, wgs_per_cu=0, window=1):
    """Register tuned launch parameters of a size class with the library (host only)."""
    code = DTYPE_CODE[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    t = lrx_tune(int(delay), int(rows_per_block), int(wgs_per_cu), int(bool(window)), 0, 0)
    _check(_lib.lrx_autotune_store(code, int(n), int(k_max), ctypes.byref(t)), "lrx_autotune_store")


def lrx_autotune_lookup(dtype, n, k_max):
    """Launch parameters of a size class: the stored entry or the library's byte-model default."""
    code = DTYPE_CODE[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    t = lrx_tune()
    _check(_lib.lrx_autotune_lookup(code, int(n), int(k_max), ctypes.byref(t)), "lrx_autotune_lookup")
    return {"delay": t.delay, "rows_per_block": t.rows_per_block, "wgs_per_cu": t.wgs_per_cu,
            "window": bool(t.window), "tuned": bool(t.tuned)}
