"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/pat.h declares; host-only entry points work without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1501_03869_amd import pat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdrs = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]
    names = set()
    for h in hdrs:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(pat_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = pat.lib()
    names = declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(pat.EXPORTED) <= set(names)


def test_version_and_error_string():
    assert pat.lib().pat_version() >= 10000
    assert isinstance(pat.lib().pat_last_error(), bytes)


def test_null_context_is_rejected_without_gpu():
    L = pat.lib()
    rc = L.pat_filter(None, None, 1, 4, 0.0, 1e-8, None, None)
    assert rc == pat.PAT_EINVAL
    assert b"context" in L.pat_last_error()
    assert L.pat_ctx_create(0, None) == pat.PAT_EINVAL


def test_tile_order_host_helper():
    nx, ny = 37, 29
    rng = np.random.default_rng(0)
    pix = rng.permutation(nx * ny)[:500].astype(np.int32)
    out = pat.tile_order(nx, ny, pix, 8, 4)
    assert sorted(out.tolist()) == sorted(pix.tolist())
    i, j = out % nx, out // nx
    key = ((j // 4) * ((nx + 7) // 8) + i // 8) * 32 + (j % 4) * 8 + (i % 8)
    assert np.all(np.diff(key) > 0)
    with pytest.raises(pat.PatError):
        pat.tile_order(nx, ny, np.array([nx * ny], np.int32), 8, 4)


def test_scratch_size_is_host_only():
    assert pat.backproject_scratch_bytes(0, 10, 1) == 0
    # several sensor groups at this size: at least two partial images
    b = pat.backproject_scratch_bytes(512, 21336, 1)
    assert b >= 2 * 21336 * 4
    # one sensor group needs no scratch
    assert pat.backproject_scratch_bytes(8, 1 << 20, 1) == 0
