"""Host logic of bench.py: the counter-profile hash that keys recorded HBM traffic to the
kernel code."""
from __future__ import annotations

import os
import sys

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))

import bench  # noqa: E402


def test_counter_hash_ignores_comments_not_code():
    base = b"int f(int x) {\n    return x + 1;  // one\n}\n"
    doc = b"/* header\n   text */\nint f(int x) {\n\n    return x + 1;  // another remark\n}\n"
    code = b"int f(int x) {\n    return x + 2;  // one\n}\n"
    assert bench.source_code_bytes(base) == bench.source_code_bytes(doc)
    assert bench.source_code_bytes(base) != bench.source_code_bytes(code)


def test_headline_counter_profile_matches_the_sources():
    """The recorded traffic of the headline accept is reported only for the code it was
    measured on: the stored hash must match the current determinant sources."""
    t = bench.counter_traffic("det_accept_kernel_uneven_n64_1024_fp32_counters.md", bench.DET_SOURCES, None,
                              key="n1024_K16_rows64")
    assert t is not None, ("the determinant sources changed since the counters in "
                           "profiles/det_accept_kernel_uneven_n64_1024_fp32_counters.md were taken: "
                           "re-run its FETCH_SIZE / WRITE_SIZE passes")
    assert 4.0e6 < t < 5.0e6
