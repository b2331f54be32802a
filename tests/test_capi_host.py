"""The C-ABI library loads, exports every symbol lrx.h declares, and rejects bad
arguments on the host (no GPU needed: every path here returns before any HIP call)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrx.h")

lrx = pytest.importorskip("paper_2602_05255_amd.lrx", reason="liblrx.so not built")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lrx_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("lrx_det_init_inverse", "lrx_det_propose_ratio", "lrx_det_accept_update",
                     "lrx_det_flush_delayed", "lrx_det_refresh", "lrx_pf_init_inverse",
                     "lrx_pf_propose_ratio", "lrx_pf_accept_update", "lrx_pf_flush_delayed",
                     "lrx_pf_refresh"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(lrx.LIB_PATH)
    for name in header_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lrx.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lrx_[a-z0-9_]+)\b", out))
    assert set(header_functions()) <= exported
    # the binding wraps exactly the declared entry points
    assert set(lrx.EXPORTED) == set(header_functions())


def test_version_and_strerror():
    assert lrx.lrx_version() == 2
    assert "flush" in lrx.lrx_strerror(lrx.LRX_ENEEDFLUSH)
    assert lrx.lrx_strerror(999) == "unknown error"


def test_state_sizes_det():
    s = lrx.lrx_state_sizes(lrx.LRX_DET, lrx.LRX_F64, 1024, 256, 4, 16)
    assert s["inv"] == 1024 * 256 * 256 * 8
    assert s["fa"] == 1024 * 16 * 4 * 256 * 8
    assert s["fb"] == 1024 * 256 * 16 * 4 * 8
    assert s["logabs"] == 1024 * 8 and s["phase"] == 1024 * 8 and s["flags"] == 1024 * 4
    assert s["stash_stride"] % 256 == 0 and s["stash"] == 1024 * s["stash_stride"]
    assert s["work"] >= 1024 * 256 * 256 * 8
    c = lrx.lrx_state_sizes(lrx.LRX_DET, lrx.LRX_C64, 2, 32, 1, 0)
    assert c["inv"] == 2 * 32 * 32 * 8 and c["fa"] == 0 and c["phase"] == 2 * 16


def test_state_sizes_pf():
    s = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_C64, 256, 512, 1, 32)
    assert s["fa"] == 256 * 32 * 2 * 512 * 8
    assert s["fb"] == 256 * 32 * 4 * 8
    assert s["work"] >= 256 * 512 * 512 * 16
    g = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_C128, 4, 64, 4, 0)     # general k-row/k-column updates
    assert g["stash_stride"] >= 8 * 64 * 16 + 8 * 8 * 16


@pytest.mark.parametrize("args,code", [
    ((lrx.LRX_DET, lrx.LRX_F64, 0, 8, 1, 0), lrx.LRX_ESHAPE),
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 0, 1, 0), lrx.LRX_ESHAPE),
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 1025, 1, 0), lrx.LRX_ESHAPE),
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 8, 3, 0), lrx.LRX_ESHAPE),
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 8, 16, 0), lrx.LRX_ESHAPE),
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 4, 8, 0), lrx.LRX_ESHAPE),          # k_max > n
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 8, 1, 65), lrx.LRX_ESHAPE),
    ((lrx.LRX_DET, lrx.LRX_F64, 4, 64, 8, 64), lrx.LRX_ESHAPE),        # K * k_max > 256
    ((lrx.LRX_DET, 9, 4, 8, 1, 0), lrx.LRX_EUNSUPPORTED),
    ((5, lrx.LRX_F64, 4, 8, 1, 0), lrx.LRX_EUNSUPPORTED),
    ((lrx.LRX_DET, lrx.LRX_C128, 4, 1024, 8, 0), lrx.LRX_EUNSUPPORTED),  # LDS panel limit
    ((lrx.LRX_PF, lrx.LRX_C64, 4, 7, 1, 0), lrx.LRX_EODD),
    ((lrx.LRX_PF, lrx.LRX_C64, 4, 8, 3, 0), lrx.LRX_EUNSUPPORTED),    # k_max 1, 2 or 4
    ((lrx.LRX_PF, lrx.LRX_C64, 4, 8, 2, 4), lrx.LRX_EUNSUPPORTED),    # general Pfaffian states are plain
    ((lrx.LRX_PF, lrx.LRX_C64, 4, 6, 4, 0), lrx.LRX_ESHAPE),          # 2 k_max > n
])
def test_state_sizes_rejects(args, code):
    with pytest.raises(lrx.LrxError) as e:
        lrx.lrx_state_sizes(*args)
    assert e.value.code == code


def fake_state(kind=lrx.LRX_DET, dtype=lrx.LRX_F64, W=4, n=8, k_max=1, delay=0, slot=0, null=(), layout=0):
    p = {f: ctypes.c_void_p(0x10000 + 0x1000 * i) for i, f in
         enumerate(("inv", "fa", "fb", "stash", "logabs", "phase", "flags", "work"))}
    for f in null:
        p[f] = ctypes.c_void_p(0)
    return lrx.lrx_state(lrx.lrx_shape(kind, dtype, W, n, k_max, delay, layout), slot, 0, p["inv"], p["fa"], p["fb"],
                         p["stash"], p["logabs"], p["phase"], p["flags"], p["work"])


P = ctypes.c_void_p(0x20000)


def test_validate():
    lib = lrx._lib
    assert lib.lrx_validate(ctypes.byref(fake_state())) == lrx.LRX_OK
    assert lib.lrx_validate(None) == lrx.LRX_EINVAL
    for f in ("inv", "stash", "logabs", "phase", "flags", "work"):
        assert lib.lrx_validate(ctypes.byref(fake_state(null=(f,)))) == lrx.LRX_EINVAL
    # slot buffers are only required with a delay
    assert lib.lrx_validate(ctypes.byref(fake_state(null=("fa", "fb")))) == lrx.LRX_OK
    assert lib.lrx_validate(ctypes.byref(fake_state(delay=4, null=("fa",)))) == lrx.LRX_EINVAL
    assert lib.lrx_validate(ctypes.byref(fake_state(delay=4, slot=5))) == lrx.LRX_EINVAL
    assert lib.lrx_validate(ctypes.byref(fake_state(delay=4, slot=-1))) == lrx.LRX_EINVAL


def test_kind_mismatch():
    lib = lrx._lib
    pf = fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64)
    det = fake_state()
    assert lib.lrx_det_propose_ratio(ctypes.byref(pf), P, P, P, P, None) == lrx.LRX_EKIND
    assert lib.lrx_det_flush_delayed(ctypes.byref(pf), None) == lrx.LRX_EKIND
    assert lib.lrx_pf_accept_update(ctypes.byref(det), P, P, P, P, None) == lrx.LRX_EKIND
    assert lib.lrx_pf_accept_hop(ctypes.byref(det), P, P, P, P, lrx.LRX_MH_FORCE, None, 0, 0, P, P, P, 8,
                                 None) == lrx.LRX_EKIND
    assert lib.lrx_pf_init_inverse(ctypes.byref(det), P, 8, P, None) == lrx.LRX_EKIND


def test_null_arguments():
    lib = lrx._lib
    st = fake_state()
    assert lib.lrx_det_propose_ratio(ctypes.byref(st), None, P, P, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_det_propose_ratio(ctypes.byref(st), P, P, None, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_det_accept_update(ctypes.byref(st), P, P, P, None, None) == lrx.LRX_EINVAL
    assert lib.lrx_det_init_inverse(ctypes.byref(st), None, 8, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_det_build_hop(ctypes.byref(st), P, 16, P, None, 8, P, P, P, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_det_build_hop(ctypes.byref(st), P, 4, P, P, 8, P, P, P, P, None) == lrx.LRX_ESHAPE


def test_delay_window_bookkeeping():
    lib = lrx._lib
    full = fake_state(delay=4, slot=4)
    assert lib.lrx_det_propose_ratio(ctypes.byref(full), P, P, P, P, None) == lrx.LRX_ENEEDFLUSH
    assert lib.lrx_det_accept_update(ctypes.byref(full), P, P, P, P, None) == lrx.LRX_ENEEDFLUSH
    pending = fake_state(delay=4, slot=2)
    assert lib.lrx_det_refresh(ctypes.byref(pending), P, 16, P, None, None) == lrx.LRX_ENEEDFLUSH
    pf_full = fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64, delay=2, slot=2)
    assert lib.lrx_pf_accept_update(ctypes.byref(pf_full), P, P, P, P, None) == lrx.LRX_ENEEDFLUSH
    assert lib.lrx_pf_accept_hop(ctypes.byref(pf_full), P, P, P, P, lrx.LRX_MH_FORCE, None, 0, 0, P, P, P, 8,
                                 None) == lrx.LRX_ENEEDFLUSH
    # flushing an empty window is a no-op that never touches the GPU
    empty = fake_state(delay=4, slot=0)
    assert lib.lrx_det_flush_delayed(ctypes.byref(empty), None) == lrx.LRX_OK
    plain = fake_state(delay=0, slot=0)
    assert lib.lrx_det_flush_delayed(ctypes.byref(plain), None) == lrx.LRX_OK


def test_metropolis_and_commit_validation():
    lib = lrx._lib
    st = fake_state()
    assert lib.lrx_metropolis(ctypes.byref(st), P, None, 1, 0, 7, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_metropolis(ctypes.byref(st), P, None, 1, 0, lrx.LRX_MH_UNIFORMS, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_metropolis(ctypes.byref(st), None, P, 1, 0, lrx.LRX_MH_FORCE, P, None) == lrx.LRX_EINVAL
    assert lib.lrx_hop_commit(0, 8, 8, 1, P, P, P, P, P, P, None) == lrx.LRX_ESHAPE
    assert lib.lrx_hop_commit(4, 8, 8, 9, P, P, P, P, P, P, None) == lrx.LRX_ESHAPE
    assert lib.lrx_hop_commit(4, 8, 8, 1, P, P, P, P, None, P, None) == lrx.LRX_EINVAL
    pf = fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64)
    ph = lib.lrx_pf_propose_hop
    assert ph(ctypes.byref(pf), P, 16, P, P, 8, P, P, None, P, P, None) == lrx.LRX_EINVAL
    assert ph(ctypes.byref(pf), P, 4, P, P, 8, P, P, P, P, P, None) == lrx.LRX_ESHAPE      # sites < n
    assert ph(ctypes.byref(st), P, 16, P, P, 8, P, P, P, P, P, None) == lrx.LRX_EKIND
    hop = lib.lrx_pf_accept_hop
    assert hop(ctypes.byref(pf), P, P, P, P, 7, None, 0, 0, P, P, P, 8, None) == lrx.LRX_EINVAL
    assert hop(ctypes.byref(pf), P, P, P, P, lrx.LRX_MH_UNIFORMS, None, 0, 0, P, P, P, 8, None) == lrx.LRX_EINVAL
    assert hop(ctypes.byref(pf), P, P, None, P, lrx.LRX_MH_FORCE, None, 0, 0, P, P, P, 8, None) == lrx.LRX_EINVAL
    assert hop(ctypes.byref(pf), P, P, P, P, lrx.LRX_MH_FORCE, None, 0, 0, P, P, P, 0, None) == lrx.LRX_ESHAPE


def test_pf_refresh_sites_check():
    lib = lrx._lib
    st = fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64, n=8)
    assert lib.lrx_pf_refresh(ctypes.byref(st), P, 4, P, None, None) == lrx.LRX_ESHAPE


def fake_class(st, null=()):
    p = {f: 0x30000 + 0x100 * i for i, f in
         enumerate(("table", "occ", "empty", "k", "elec", "slot", "u01", "u", "ratio", "accept"))}
    for f in null:
        p[f] = 0
    return lrx.lrx_window_class(ctypes.pointer(st), p["table"], 2 * st.shape.n, st.shape.n, p["occ"], p["empty"],
                                p["k"], p["elec"], p["slot"], p["u01"], p["u"], p["ratio"], p["accept"])


def classes_of(*cls):
    arr = (lrx.lrx_window_class * len(cls))()
    for i, c in enumerate(cls):
        arr[i] = c
    return arr


def test_window_work_bytes():
    lib = lrx._lib
    sts = [fake_state(W=3, n=64, k_max=4, delay=4, dtype=lrx.LRX_F32),
           fake_state(W=200, n=256, k_max=4, delay=8, dtype=lrx.LRX_F32)]
    arr = classes_of(*[fake_class(s) for s in sts])
    out = ctypes.c_size_t()
    assert lib.lrx_window_work_bytes(arr, 2, ctypes.byref(out)) == lrx.LRX_OK
    assert out.value == 256           # one work counter, rounded up to 256 bytes
    assert lib.lrx_window_work_bytes(arr, 2, None) == lrx.LRX_EINVAL


def test_window_validation():
    lib = lrx._lib
    P2 = ctypes.c_void_p(0x40000)

    def call(arr, n_cls, steps=4, mode=lrx.LRX_MH_FORCE, work_bytes=4096, grid=8, work=P2):
        return lib.lrx_det_window(arr, n_cls, steps, mode, 1, 0, work, work_bytes, grid, None)

    ok = fake_state(W=4, n=64, k_max=4, delay=4, dtype=lrx.LRX_F32)
    base = fake_class(ok)
    assert lib.lrx_det_window(None, 1, 4, lrx.LRX_MH_FORCE, 1, 0, P2, 4096, 8, None) == lrx.LRX_EINVAL
    assert call(classes_of(base), 0) == lrx.LRX_EINVAL
    assert call(classes_of(*[base] * 9), 9) == lrx.LRX_EINVAL
    assert call(classes_of(base), 1, steps=0) == lrx.LRX_EINVAL
    assert call(classes_of(base), 1, steps=lrx.LRX_MAX_WINDOW_STEPS + 1) == lrx.LRX_EINVAL
    assert call(classes_of(base), 1, grid=0) == lrx.LRX_EINVAL
    assert call(classes_of(base), 1, work_bytes=2) == lrx.LRX_EINVAL        # the counter needs 4 bytes
    assert call(classes_of(base), 1, work=None) == lrx.LRX_EINVAL
    assert call(classes_of(base), 1, mode=7) == lrx.LRX_EINVAL
    assert call(classes_of(fake_class(ok, null=("u01",))), 1, mode=lrx.LRX_MH_UNIFORMS) == lrx.LRX_EINVAL
    for f in ("table", "occ", "empty", "k", "elec", "slot", "u", "ratio", "accept"):
        assert call(classes_of(fake_class(ok, null=(f,))), 1) == lrx.LRX_EINVAL, f
    cplx = fake_state(W=4, n=64, k_max=4, delay=4, dtype=lrx.LRX_C64)
    assert call(classes_of(fake_class(cplx)), 1) == lrx.LRX_EUNSUPPORTED
    plain = fake_state(W=4, n=64, k_max=4, delay=0, dtype=lrx.LRX_F32)
    assert call(classes_of(fake_class(plain)), 1) == lrx.LRX_EUNSUPPORTED
    other_dtype = fake_state(W=4, n=64, k_max=4, delay=4, dtype=lrx.LRX_F64)
    assert call(classes_of(base, fake_class(other_dtype)), 2) == lrx.LRX_EUNSUPPORTED
    other_k = fake_state(W=4, n=64, k_max=2, delay=4, dtype=lrx.LRX_F32)
    assert call(classes_of(base, fake_class(other_k)), 2) == lrx.LRX_EUNSUPPORTED
    pf = fake_state(kind=lrx.LRX_PF, W=4, n=64, k_max=1, delay=4, dtype=lrx.LRX_F32)
    assert call(classes_of(fake_class(pf)), 1) == lrx.LRX_EKIND
    full = fake_state(W=4, n=64, k_max=4, delay=4, slot=4, dtype=lrx.LRX_F32)
    assert call(classes_of(fake_class(full)), 1) == lrx.LRX_ENEEDFLUSH


def test_autotune_table():
    """Byte-model defaults for an unknown size class; a stored entry replaces them."""
    d = lrx.lrx_autotune_lookup(lrx.LRX_F32, 1000, 1)
    assert d == {"delay": 32, "rows_per_block": 0, "wgs_per_cu": 2, "window": False,
                 "tuned": False}                                       # sqrt(2000) = 44.7 -> 32
    assert lrx.lrx_autotune_lookup(lrx.LRX_F64, 128, 1)["delay"] == 16   # the paper's det optimum T = 16
    assert lrx.lrx_autotune_lookup(lrx.LRX_F32, 64, 8)["window"] is True
    lrx.lrx_autotune_store(lrx.LRX_F32, 1000, 1, 8, 256, 3, 0)
    assert lrx.lrx_autotune_lookup(lrx.LRX_F32, 1000, 1) == {"delay": 8, "rows_per_block": 256, "wgs_per_cu": 3,
                                                            "window": False, "tuned": True}
    lrx.lrx_autotune_store(lrx.LRX_F32, 1000, 1, 16, 0, 0, 1)
    assert lrx.lrx_autotune_lookup(lrx.LRX_F32, 1000, 1)["delay"] == 16
    with pytest.raises(lrx.LrxError):
        lrx.lrx_autotune_store(lrx.LRX_F32, 1000, 8, 64, 0, 0)     # K k_max > 256
    with pytest.raises(lrx.LrxError):
        lrx.lrx_autotune_lookup(lrx.LRX_F32, 0, 1)
    with pytest.raises(lrx.LrxError):
        lrx.lrx_autotune_store(lrx.LRX_F32, 64, 1, 4, 8, 0)        # rows per block below 16


def test_layout_sizes_and_checks():
    """Fused and packed Pfaffian layouts: sizes (upper 64 x 64 tiles, one or two pending
    slots, partial dots in the workspace) and the shapes they refuse."""
    W, n, es = 3, 130, 16
    full = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_C128, W, n, 1, 0)
    fused = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_C128, W, n, 1, 0, lrx.LRX_LAYOUT_FUSED)
    packed = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_C128, W, n, 1, 0, lrx.LRX_LAYOUT_PACKED)
    nt = 3                                              # ceil(130 / 64)
    assert fused["inv"] == full["inv"] == W * n * n * es
    assert packed["inv"] == W * nt * (nt + 1) // 2 * 64 * 64 * es
    assert fused["fa"] == W * 2 * 2 * n * es and fused["fb"] == W * 2 * 4 * es
    assert packed["fa"] == W * 1 * 2 * n * es and packed["fb"] == W * 1 * 4 * es
    assert packed["work"] >= W * 6 * 2 * 64 * es
    # at n = 1024 the packed triangle is 136 of 256 tiles
    big = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_F32, 1, 1024, 1, 0, lrx.LRX_LAYOUT_PACKED)
    assert big["inv"] == 136 * 4096 * 4
    pdel = lrx.lrx_state_sizes(lrx.LRX_PF, lrx.LRX_C128, W, n, 1, 4, lrx.LRX_LAYOUT_PACKED)
    assert pdel["inv"] == packed["inv"] and pdel["fa"] == W * 4 * 2 * n * es and pdel["fb"] == W * 4 * 4 * es
    for args in [(lrx.LRX_DET, lrx.LRX_F64, 2, 8, 1, 0, lrx.LRX_LAYOUT_FUSED),      # DET
                 (lrx.LRX_PF, lrx.LRX_C64, 2, 8, 1, 4, lrx.LRX_LAYOUT_FUSED),       # delayed
                 (lrx.LRX_PF, lrx.LRX_C64, 2, 8, 2, 0, lrx.LRX_LAYOUT_PACKED),      # k_max 2
                 (lrx.LRX_PF, lrx.LRX_C64, 2, 8, 1, 0, 3)]:                         # unknown layout
        with pytest.raises(lrx.LrxError) as e:
            lrx.lrx_state_sizes(*args)
        assert e.value.code == lrx.LRX_EUNSUPPORTED, args
    lib = lrx._lib
    st = fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64, layout=lrx.LRX_LAYOUT_PACKED, slot=1)
    assert lib.lrx_validate(ctypes.byref(st)) == lrx.LRX_OK
    assert lib.lrx_validate(ctypes.byref(fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64,
                                                    layout=lrx.LRX_LAYOUT_FUSED, slot=2))) == lrx.LRX_EINVAL
    assert lib.lrx_validate(ctypes.byref(fake_state(kind=lrx.LRX_PF, dtype=lrx.LRX_C64, layout=lrx.LRX_LAYOUT_FUSED,
                                                    null=("fa",)))) == lrx.LRX_EINVAL
    # refresh with a pending update, and the entry points that take full storage only
    assert lib.lrx_pf_refresh(ctypes.byref(st), P, 16, P, None, None) == lrx.LRX_ENEEDFLUSH
    assert lib.lrx_pf_lowrank_fwd(ctypes.byref(st), 2, P, P, P, P, P, None) == lrx.LRX_EUNSUPPORTED
    assert lib.lrx_pf_grad(ctypes.byref(st), P, P, None) == lrx.LRX_EUNSUPPORTED
    assert lib.lrx_pf_propose_general(ctypes.byref(st), 1, P, P, P, None) == lrx.LRX_EUNSUPPORTED
    assert lib.lrx_pf_read_inverse(ctypes.byref(st), None, None) == lrx.LRX_EINVAL
    assert lib.lrx_pf_read_inverse(ctypes.byref(fake_state()), P, None) == lrx.LRX_EKIND
