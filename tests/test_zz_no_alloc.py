"""pat_backproject_noalloc: the same kernels as pat_backproject with the gather
scratch taken from the device's fixed array.  Its images must equal
pat_backproject's bit for bit, on two calls in a row (the second with a
smaller input, so stale partial sums or counters of the first would show),
for the shapes that use scratch: the LDS-windowed kernel over several sensor
groups and the batched kernel (and for the split-sensor and wave-window
kernels, which use none); and it must allocate nothing, which a context that
refuses every device allocation shows."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1501_03869_amd import pat  # noqa: E402

DT = 25e-9


def _inputs(seed, S, P, N, F, f16):
    rng = np.random.default_rng(seed)
    # delays over the record and a little beyond both ends (those contribute 0)
    table = ((rng.random((S, P), dtype=np.float32) * (N + 1.0) - 1.0) * DT).astype(np.float32)
    sig = rng.standard_normal((F, S, N)).astype(np.float32)
    dev = torch.device("cuda:0")
    t = torch.from_numpy(table).to(dev)
    if f16:
        s = torch.from_numpy(sig.astype(np.float16)).to(dev)
        scale = torch.from_numpy(rng.uniform(0.5, 2.0, F).astype(np.float32)).to(dev)
    else:
        s = torch.from_numpy(sig).to(dev)
        scale = None
    return t, s, scale


def _both(ctx, t, s, scale, F, filtered=False):
    P = t.shape[1]
    sig = s if F > 1 else s[0]
    ref = ctx.backproject(t, sig, DT, filtered=filtered, frame_scale=scale)
    out = torch.full((F, P) if F > 1 else (P,), float("nan"), dtype=torch.float32, device=t.device)
    ctx.backproject(t, sig, DT, filtered=filtered, frame_scale=scale, out=out, noalloc=True)
    torch.cuda.synchronize()
    return ref, out


# (S, P, N, F, fp16 frames): first call, then a smaller one
CASES = {
    # N < 4: the LDS-windowed kernel, sensors split over several groups
    "windowed": [(512, 21336, 3, 2, False), (200, 5000, 3, 1, False)],
    # several frames with a table above 128 MiB: the batched kernel
    "batched": [(320, 120000, 64, 3, True), (280, 121000, 64, 2, True)],
    # the split-sensor kernel (no scratch) through the same entry point
    "split_sensor": [(512, 21336, 2048, 1, False), (64, 4099, 1024, 1, True)],
    # tables above 128 MiB with at least 131072 columns: the wave-window
    # kernel (no scratch)
    "wave_window": [(256, 140000, 256, 2, True), (260, 135000, 200, 1, False)],
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_noalloc_equals_backproject_on_two_calls(case):
    ctx = pat.Context(0)
    try:
        for i, (S, P, N, F, f16) in enumerate(CASES[case]):
            need = pat.backproject_scratch_bytes(S, P, F)
            if case in ("windowed", "batched"):
                assert need > 0, (case, S, P, F)
            assert need < pat.NOALLOC_SCRATCH_BYTES
            print(f"[noalloc] {case} call {i}: S={S} P={P} N={N} F={F} fp16={f16} scratch<={need}", flush=True)
            t, s, scale = _inputs(100 + i, S, P, N, F, f16)
            ref, out = _both(ctx, t, s, scale, F)
            assert torch.isfinite(ref).all()
            assert torch.equal(ref, out), float((ref - out).abs().max())
    finally:
        ctx.close()


def test_noalloc_rejects_sizes_beyond_the_fixed_scratch():
    # the LDS-windowed kernel (N < 4) over two sensor groups: 2 P F floats
    S, P, N, F = 64, 1000000, 3, 3
    need = pat.backproject_scratch_bytes(S, P, F)
    assert need == 2 * P * F * 4 > pat.NOALLOC_SCRATCH_BYTES
    ctx = pat.Context(0)
    try:
        dev = torch.device("cuda:0")
        t = torch.zeros((S, P), dtype=torch.float32, device=dev)
        s = torch.zeros((F, S, N), dtype=torch.float32, device=dev)
        out = torch.full((F, P), 7.0, dtype=torch.float32, device=dev)
        with pytest.raises(pat.PatError) as e:
            ctx.backproject(t, s, DT, filtered=False, out=out, noalloc=True)
        assert e.value.code == pat.PAT_EINVAL
        assert "fixed scratch" in str(e.value)
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())  # nothing was launched
    finally:
        ctx.close()


def test_noalloc_needs_no_allocation():
    # a context that refuses every device allocation: pat_backproject cannot
    # get its scratch, pat_backproject_noalloc needs none
    S, P, N, F = 512, 21336, 3, 1
    t, s, _ = _inputs(7, S, P, N, F, False)
    good = pat.Context(0)
    try:
        ref = good.backproject(t, s[0], DT, filtered=False)
    finally:
        good.close()
    os.environ["PAT_FAULT_ALLOC_BYTES"] = "1"
    try:
        ctx = pat.Context(0)
    finally:
        del os.environ["PAT_FAULT_ALLOC_BYTES"]
    try:
        with pytest.raises(pat.PatError) as e:
            ctx.backproject(t, s[0], DT, filtered=False)
        assert e.value.code == pat.PAT_ENOMEM
        out = torch.empty((P,), dtype=torch.float32, device=t.device)
        for _ in range(2):
            out.fill_(float("nan"))
            ctx.backproject(t, s[0], DT, filtered=False, out=out, noalloc=True)
            torch.cuda.synchronize()
            assert torch.equal(ref, out)
    finally:
        ctx.close()
