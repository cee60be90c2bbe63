"""Precision study on the 1024^2 workload: every storage variant of the back
projection gathered on the GPU from the oracle's own eikonal table (FP64 heap
fast marching, all 1024 sensors, rounded to float32 seconds) and one
synthetic frame, and checked against the FP64 oracle: on the whole image
(823592 pixels) against the oracle gathering the delays each variant stores,
and on 94 whole 32-pixel tiles (3008 pixels) against the a-priori bounds.

Variants: V0 float32 table + float32 frame; V1 16.16 table + float32 frame;
V2 float32 table + binary16 frame (per-frame scale); V3 16.16 + binary16;
V4 16-bit tile-relative table + binary16 (V4a with a float32 frame).
Each variant is checked two ways: against the oracle gathering exactly the
delays the variant stores (16.16 and 16-bit tables decoded by the oracle's
own encoders) within the FP32 image tolerance, and against the FP64 gather of
the unquantised inputs within its a-priori per-pixel bound."""
import time

import numpy as np
import pytest

from paper_1501_03869_amd import inputs

from error_bounds import f32_decode_quant, fp16_frames, gather_error_bound

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_large_grid_precision_variants(orc):
    from paper_1501_03869_amd import pat
    geo = inputs.config("large")
    geo.pix = pat.tile_order(geo.nx, geo.ny, geo.pix, 32, 32)
    S, P, N, dt = geo.S, geo.P, geo.n_samples, geo.dt
    tiles = np.sort(np.random.default_rng(91).choice(P // 32, 94, replace=False))
    sample = (tiles[:, None] * 32 + np.arange(32)[None, :]).ravel()
    t = time.time()
    T32 = np.empty((S, P), np.float32)
    T64s = np.empty((S, sample.size))
    for s0 in range(0, S, 128):
        chunk = orc.tables(geo.speed, geo.h, geo.sensors[s0:s0 + 128], geo.pix)
        T32[s0:s0 + 128] = chunk
        T64s[s0:s0 + 128] = chunk[:, sample]
        del chunk
    print(f"[precision-1024] oracle tables for {S} sensors in {time.time() - t:.1f} s", flush=True)
    p = inputs.frame_for(geo, T32, 0)
    p64 = p.astype(np.float64)
    scale, h16, p16 = fp16_frames(p[None])
    scale, h16, p16 = float(scale[0]), h16[0], p16[0]
    T32s = T32[:, sample].astype(np.float64)

    ctx = pat.Context(0)
    try:
        Td = dev(T32)
        pd, hd = dev(p), dev(h16)
        sd = torch.tensor([scale], dtype=torch.float32, device="cuda")
        got = {"V0": ctx.backproject(Td, pd, dt, filtered=False),
               "V2": ctx.backproject(Td, hd, dt, filtered=False, frame_scale=sd)}
        q = ctx.table_to_q16(Td, dt, N)
        got["V1"] = ctx.backproject(q, pd, dt, filtered=False)
        got["V3"] = ctx.backproject(q, hd, dt, filtered=False, frame_scale=sd)
        del q
        r16 = ctx.table_to_r16(Td, dt, N)
        got["V4"] = ctx.backproject(r16, hd, dt, filtered=False, frame_scale=sd)
        got["V4a"] = ctx.backproject(r16, pd, dt, filtered=False)
        torch.cuda.synchronize()
        got_full = {k: v.cpu().numpy() for k, v in got.items()}
        got = {k: v[sample] for k, v in got_full.items()}
        del Td, r16
    finally:
        ctx.close()

    # the oracle's references on the sampled pixels
    ref64 = orc.backproject(T64s, p64, dt)          # unrounded FP64 table
    ref = orc.backproject(T32s, p64, dt)             # the float32 table, FP64 arithmetic
    ref16 = orc.backproject(T32s, p16, dt)           # the same on the binary16 frame's values
    b32, b16 = orc.filt(p64, dt), orc.filt(p16, dt)
    q16 = orc.table_to_q16(T32s.astype(np.float32), dt, N)
    off, hdr = orc.table_to_r16(T32s.astype(np.float32), dt, N)
    qr16 = orc.r16_to_q16(off, hdr)
    exact = {"V0": ref, "V2": ref16, "V1": orc.gather_q16(q16, b32), "V3": orc.gather_q16(q16, b16),
             "V4": orc.gather_q16(qr16, b16), "V4a": orc.gather_q16(qr16, b32)}
    k = 16 - (hdr & 0xFFFF).astype(np.int64)                      # per (sensor, tile) shift
    quant_r16 = np.repeat(2.0 ** -(k + 1), 32, axis=1)
    dq = f32_decode_quant(T32s, dt)
    quant = {"V0": dq, "V2": dq, "V1": 2.0 ** -17, "V3": 2.0 ** -17, "V4": quant_r16, "V4a": quant_r16}
    half = {"V0": None, "V1": None, "V4a": None, "V2": scale, "V3": scale, "V4": scale}
    for name in ("V0", "V1", "V2", "V3", "V4", "V4a"):
        g = got[name]
        e_exact = rel_l2(g, exact[name])
        bound = gather_error_bound(T32s, p64, dt, quant[name], half[name])
        err = np.abs(g - ref)
        print(f"[precision-1024] {name}: rel L2 vs FP64 on the unquantised inputs {rel_l2(g, ref):.3e} "
              f"(vs the unrounded FP64 table {rel_l2(g, ref64):.3e}); vs the oracle on the stored delays "
              f"{e_exact:.3e}; bound rel L2 {np.linalg.norm(bound) / np.linalg.norm(ref):.3e}, "
              f"max err/bound {(err / bound).max():.3f}; k median {int(np.median(k))} min {int(k.min())}",
              flush=True)
        assert e_exact <= IMG_TOL, name
        assert np.all(err <= bound), name
    # the V0 image is also within the FP32 target against the unrounded table
    assert rel_l2(got["V0"], ref64) <= IMG_TOL

    # the whole image of every variant against the oracle gathering exactly
    # the delays the variant stores
    t = time.time()
    full = {"V0": orc.gather(T32, b32, dt), "V2": orc.gather(T32, b16, dt)}
    q = orc.table_to_q16(T32, dt, N)
    full["V1"], full["V3"] = orc.gather_q16(q, b32), orc.gather_q16(q, b16)
    del q
    off, hdr = orc.table_to_r16(T32, dt, N)
    qr = orc.r16_to_q16(off, hdr)
    del off, hdr, T32
    full["V4"], full["V4a"] = orc.gather_q16(qr, b16), orc.gather_q16(qr, b32)
    del qr
    print(f"[precision-1024] whole-image oracle references in {time.time() - t:.1f} s", flush=True)
    for name in ("V0", "V1", "V2", "V3", "V4", "V4a"):
        e = rel_l2(got_full[name], full[name])
        print(f"[precision-1024] {name}: whole image ({P} pixels) rel L2 vs the oracle on the stored delays {e:.3e}",
              flush=True)
        assert e <= IMG_TOL, name
