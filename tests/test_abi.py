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


def test_update_eval_validates_before_any_launch():
    # argument errors return before the library touches the GPU
    L = pat.lib()
    assert L.pat_eikonal_update_eval(None, None, -1, 2, None, None) == pat.PAT_EINVAL
    assert b"negative" in L.pat_last_error()
    assert L.pat_eikonal_update_eval(None, None, 4, 4, None, None) == pat.PAT_EINVAL
    assert b"dims" in L.pat_last_error()
    assert L.pat_eikonal_update_eval(None, None, 4, 3, None, None) == pat.PAT_EINVAL
    assert b"null" in L.pat_last_error()
    assert L.pat_eikonal_update_eval(None, None, 0, 2, None, None) == pat.PAT_OK


def _morton(i, j):
    r = 0
    for b in range(16):
        r |= ((i >> b) & 1) << (2 * b) | ((j >> b) & 1) << (2 * b + 1)
    return r


def test_tile_order_host_helper():
    nx, ny = 37, 29
    rng = np.random.default_rng(0)
    pix = rng.permutation(nx * ny)[:500].astype(np.int32)
    out = pat.tile_order(nx, ny, pix, 8, 4)
    assert sorted(out.tolist()) == sorted(pix.tolist())
    i, j = out % nx, out // nx
    tx = (nx + 7) // 8

    def tile(ii, jj):  # serpentine tile rows
        r = jj // 4
        return r * tx + (tx - 1 - ii // 8 if r % 2 else ii // 8)

    key = [(tile(ii, jj) << 32) | _morton(ii % 8, jj % 4) for ii, jj in zip(i.tolist(), j.tolist())]
    assert all(a < b for a, b in zip(key, key[1:]))
    # a full 32x32 tile: every aligned run of 256 pixels is a 16x16 square
    full = np.arange(64 * 64, dtype=np.int32)
    o = pat.tile_order(64, 64, full, 32, 32)
    for r in range(0, 1024, 256):
        blk = o[r:r + 256]
        assert np.ptp(blk % 64) == 15 and np.ptp(blk // 64) == 15
    # consecutive tiles are neighbours: along the order, tile coordinates never jump
    o = pat.tile_order(100, 100, np.arange(100 * 100, dtype=np.int32), 32, 32)
    ti, tj = (o % 100) // 32, (o // 100) // 32
    step = np.abs(np.diff(ti)) + np.abs(np.diff(tj))
    assert step.max() <= 1
    with pytest.raises(pat.PatError):
        pat.tile_order(nx, ny, np.array([nx * ny], np.int32), 8, 4)


def test_tile_order_3d_host_helper():
    nx, ny, nz = 13, 11, 9
    rng = np.random.default_rng(1)
    vox = rng.permutation(nx * ny * nz)[:700].astype(np.int32)
    out = pat.tile_order_3d(nx, ny, nz, vox, 4, 4, 2)
    assert sorted(out.tolist()) == sorted(vox.tolist())
    # every full 4x4x2 tile is one aligned run of 32 compact voxels
    n = 16
    o = pat.tile_order_3d(n, n, n, np.arange(n ** 3, dtype=np.int32), 4, 4, 2)
    for r in range(0, n ** 3, 32):
        blk = o[r:r + 32]
        i, j, l = blk % n, (blk // n) % n, blk // (n * n)
        assert np.ptp(i) == 3 and np.ptp(j) == 3 and np.ptp(l) == 1
    # consecutive tiles are neighbours: along the order, tile coordinates never jump
    ti, tj, tl = (o % n) // 4, ((o // n) % n) // 4, (o // (n * n)) // 2
    step = np.abs(np.diff(ti)) + np.abs(np.diff(tj)) + np.abs(np.diff(tl))
    assert step.max() <= 1
    # inside a tile: Morton order of the local coordinates
    t0 = o[:32]
    loc = [(int(a % n) % 4, int((a // n) % n) % 4, int(a // (n * n)) % 2) for a in t0]
    mort = [sum((((x >> b) & 1) << (3 * b)) | (((y >> b) & 1) << (3 * b + 1)) | (((z >> b) & 1) << (3 * b + 2))
                for b in range(3)) for x, y, z in loc]
    assert mort == sorted(mort)
    with pytest.raises(pat.PatError):
        pat.tile_order_3d(nx, ny, nz, np.array([nx * ny * nz], np.int32), 4, 4, 2)


def test_interleaved_table_size_is_host_only():
    L = pat.lib()
    assert L.pat_table_x4_bytes(0, 10) == 0
    assert L.pat_table_x4_bytes(1, 10) == 160
    assert L.pat_table_x4_bytes(5, 7) == 2 * 7 * 16
    assert L.pat_table_x4_bytes(512, 21336) == 512 * 21336 * 4


def test_scratch_size_is_host_only():
    assert pat.backproject_scratch_bytes(0, 10, 1) == 0
    # several sensor groups at this size: at least two partial images
    b = pat.backproject_scratch_bytes(512, 21336, 1)
    assert b >= 2 * 21336 * 4
    # one sensor group needs no scratch
    assert pat.backproject_scratch_bytes(8, 1 << 20, 1) == 0


# The boundary's named calls (the operations of Sections II-B, II-C and III:
# per-sensor tables, their 16.16 form, the filter, the back projection sum and
# the offline/online frame server) with their parameter types in order.
BOUNDARY = {
    "pat_last_error": ["void"],
    "pat_ctx_create": ["int", "pat_ctx**"],
    "pat_ctx_destroy": ["pat_ctx*"],
    "pat_eikonal_tables": ["pat_ctx*", "const float*", "int", "int", "double", "const double*", "int",
                           "const int32_t*", "int", "float*", "void*"],
    "pat_table_to_fixed": ["pat_ctx*", "const float*", "int", "int", "double", "double", "int", "uint32_t*",
                           "void*"],
    "pat_tile_order": ["int", "int", "const int32_t*", "int", "int", "int", "int32_t*"],
    "pat_filter": ["pat_ctx*", "const float*", "int", "int", "double", "double", "float*", "void*"],
    "pat_backproject": ["pat_ctx*", "const void*", "int", "const void*", "int", "int", "const float*",
                        "const float*", "int", "int", "int", "double", "double", "int", "float*", "void*"],
    "pat_server_create": ["pat_ctx*", "size_t", "pat_server**"],
    "pat_server_add_map": ["pat_server*", "const float*", "int", "int", "double", "const double*", "int",
                           "const int32_t*", "int", "double", "double", "int", "int*"],
    "pat_server_submit": ["pat_server*", "int", "const void*", "int", "float", "int", "uint64_t*"],
    "pat_server_wait": ["pat_server*", "uint64_t", "float*", "int"],
    "pat_server_stats": ["pat_server*", "pat_stats*"],
    "pat_server_remove_map": ["pat_server*", "int"],
    "pat_server_destroy": ["pat_server*"],
}


def _declared_params():
    txt = open(os.path.join(ROOT, "include", "pat.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for m in re.finditer(r"\b(pat_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", txt):
        params = []
        for p in m.group(2).split(","):
            p = " ".join(p.replace("*", " * ").split())
            words = p.split(" ")
            if words != ["void"]:
                words = words[:-1]  # drop the parameter name
            params.append(" ".join(words).replace(" *", "*"))
        out[m.group(1)] = params
    return out


def test_boundary_calls_exported_with_their_signatures():
    L = pat.lib()
    decl = _declared_params()
    for name, params in BOUNDARY.items():
        assert hasattr(L, name), name
        assert decl.get(name) == params, (name, decl.get(name))
