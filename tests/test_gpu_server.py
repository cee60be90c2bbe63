"""Frame server on the GPU: continuous batching of frames of different
geometries, HBM-budget admission, eviction and rebuild, slots, and the rule
that a frame's image is the same alone and in a mix (bitwise)."""
import numpy as np
import pytest

from paper_1501_03869_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

WAIT_MS = 30000


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_03869_amd import pat
    c = pat.Context(0)
    yield c
    c.close()


def _maps():
    tiny = inputs.config("tiny")
    small = inputs.config("small")
    # a ragged variant: a pixel count that is not a multiple of 4 and another sampling
    rag = inputs.Geometry("ragged", small.nx, small.ny, small.h, small.speed, small.sensors[::3], small.pix[:9999],
                          600, 4e-8, 1e-7)
    return [tiny, small, rag]


_tables = {}


def _oracle_tables(orc, geos):
    for g in geos:
        if g.name not in _tables:
            _tables[g.name] = orc.tables(g.speed, g.h, g.sensors, g.pix)
    return [_tables[g.name] for g in geos]


def _frames(geos, tabs, per_map):
    out = []
    for gi, (g, T) in enumerate(zip(geos, tabs)):
        for k in range(per_map):
            nodes, amp = inputs.point_absorbers(7000 + 10 * gi + k, g.nx, g.ny, g.h, count=4,
                                                r_max=0.35 * g.nx * g.h)
            col = np.full(g.nx * g.ny, -1)
            col[g.pix] = np.arange(g.P)
            keep = col[nodes] >= 0
            nodes, amp = nodes[keep], amp[keep]
            p = inputs.npulse_signals(T[:, col[nodes]], amp, inputs.source_distances(g, nodes), g.n_samples, g.dt,
                                      g.t0)
            out.append((gi, p))
    return out


def _server(ctx, **kw):
    from paper_1501_03869_amd import pat
    return pat.Server(ctx, **kw)


def _add_all(srv, geos):
    ids = [srv.add_map(g.speed, g.h, g.sensors, g.pix, g.n_samples, g.dt, g.t0) for g in geos]
    return ids


@pytest.mark.parametrize("variant", ["f32", "q16_f16"])
def test_alone_equals_mix_and_matches_oracle(ctx, orc, variant):
    from paper_1501_03869_amd import pat
    geos = _maps()
    tabs = _oracle_tables(orc, geos)
    frames = _frames(geos, tabs, 3)
    if variant == "f32":
        srv = _server(ctx, max_batch=16)
        enc = [(gi, p, 1.0) for gi, p in frames]
    else:
        srv = _server(ctx, table_fmt=pat.TABLE_Q16, sig_fmt=pat.SIG_F16, max_batch=16)
        enc = []
        for gi, p in frames:
            sc = float(np.abs(p).max() / 2.0 ** 14)
            enc.append((gi, (p / sc).astype(np.float16), sc))
    ids = _add_all(srv, geos)
    # alone: one frame in the system at a time
    alone = []
    for gi, p, sc in enc:
        t = srv.submit(ids[gi], p, sc)
        alone.append(srv.wait(t, ids[gi], timeout_ms=WAIT_MS))
    # mix: everything queued at once, interleaved over the maps, released
    # together so that the geometries share launches
    order = list(range(len(enc)))[::-1]
    srv.reset_stats()
    srv.hold(True)
    tickets = {k: srv.submit(ids[enc[k][0]], enc[k][1], enc[k][2]) for k in order}
    srv.hold(False)
    mixed = {k: srv.wait(tickets[k], ids[enc[k][0]], timeout_ms=WAIT_MS) for k in order}
    st = srv.stats()
    print(f"[server {variant}] batches {st['batches']} mean batch {st['mean_batch_frames']:.2f} "
          f"p50 {st['latency_p50_us']:.0f} us p99 {st['latency_p99_us']:.0f} us", flush=True)
    assert st["batches"] - len(enc) < len(enc)  # the mix really shared launches
    for k in range(len(enc)):
        assert np.array_equal(alone[k], mixed[k]), f"frame {k} differs between alone and mix"
    # accuracy against the FP64 oracle (server tables are its own GPU builds)
    for k, (gi, p) in enumerate(frames):
        g = geos[gi]
        ref = orc.backproject(tabs[gi], p, g.dt, g.t0)
        err = np.linalg.norm(alone[k] - ref) / np.linalg.norm(ref)
        assert err <= (2e-3 if variant == "f32" else 5e-3), (k, err)
    srv.close()


def test_server_image_equals_backproject(ctx, orc):
    # the server splits each frame exactly like a single-frame pat_backproject
    # call, so with the same table the images are bitwise equal
    g = inputs.config("small")
    T = torch.from_numpy(_oracle_tables(orc, [g])[0].astype(np.float32)).cuda()
    srv = _server(ctx)
    mid = srv.add_map(g.speed, g.h, g.sensors, g.pix, g.n_samples, g.dt)
    (_, p), = _frames([g], [_oracle_tables(orc, [g])[0]], 1)
    got = srv.wait(srv.submit(mid, p), mid, timeout_ms=WAIT_MS)
    # rebuild the table the way the server did and gather it directly
    Tg = ctx.eikonal_tables(torch.from_numpy(g.speed).cuda(), g.h, g.sensors, torch.from_numpy(g.pix).cuda())
    direct = ctx.backproject(Tg, torch.from_numpy(p).cuda(), g.dt, filtered=False).cpu().numpy()
    assert np.allclose(got, direct, rtol=1e-5, atol=1e-5 * np.abs(direct).max())
    del T
    srv.close()


def test_admission_eviction_and_rebuild(ctx, orc):
    from paper_1501_03869_amd import pat
    g = inputs.config("small")
    tab = _oracle_tables(orc, [g])[0]
    (_, p), = _frames([g], [tab], 1)
    table_b = g.S * g.P * 4
    # room for one map's table and working memory, not two tables
    srv = _server(ctx, hbm_budget_bytes=int(2.6 * table_b))
    a = srv.add_map(g.speed, g.h, g.sensors, g.pix, g.n_samples, g.dt)
    img_a = srv.wait(srv.submit(a, p), a, timeout_ms=WAIT_MS)
    b = srv.add_map(g.speed, g.h, g.sensors, g.pix, g.n_samples, g.dt)
    img_b = srv.wait(srv.submit(b, p), b, timeout_ms=WAIT_MS)
    st = srv.stats()
    assert st["evictions"] >= 1
    assert srv.map_state(a) == pat.MAP_EVICTED
    # a frame for the evicted map brings its table back
    img_a2 = srv.wait(srv.submit(a, p), a, timeout_ms=WAIT_MS)
    assert np.allclose(img_a2, img_a, rtol=1e-5, atol=1e-5 * np.abs(img_a).max())
    assert np.allclose(img_b, img_a, rtol=1e-5, atol=1e-5 * np.abs(img_a).max())
    assert srv.stats()["builds"] >= 3
    # a map that cannot fit at all is refused
    big = inputs.config("paper")
    with pytest.raises(pat.PatError) as e:
        srv.add_map(big.speed, big.h, big.sensors, big.pix, big.n_samples, big.dt)
    assert e.value.code == pat.PAT_EBUSY
    srv.close()


def test_slots_refuse_and_recover(ctx, orc):
    from paper_1501_03869_amd import pat
    g = inputs.config("tiny")
    tab = _oracle_tables(orc, [g])[0]
    (_, p), = _frames([g], [tab], 1)
    srv = _server(ctx, max_slots=2)
    m = srv.add_map(g.speed, g.h, g.sensors, g.pix, g.n_samples, g.dt)
    t1 = srv.submit(m, p)
    t2 = srv.submit(m, p)
    with pytest.raises(pat.PatError) as e:
        srv.submit(m, p, nonblocking=True)
    assert e.value.code == pat.PAT_EBUSY
    srv.wait(t1, m, timeout_ms=WAIT_MS)
    t3 = srv.submit(m, p, nonblocking=True)
    srv.wait(t2, m, timeout_ms=WAIT_MS)
    srv.wait(t3, m, timeout_ms=WAIT_MS)
    assert srv.stats()["frames_refused"] == 1
    with pytest.raises(pat.PatError) as e:
        srv.wait(t3, m, timeout_ms=10)
    assert e.value.code == pat.PAT_ENOTFOUND
    with pytest.raises(pat.PatError) as e:
        srv.submit(999, p)
    assert e.value.code == pat.PAT_ENOTFOUND
    srv.close()


def test_build_overlaps_frames(ctx, orc):
    # frames keep completing for a resident map while a new map is built
    from paper_1501_03869_amd import pat
    geos = _maps()[:2]
    tabs = _oracle_tables(orc, geos)
    frames = _frames(geos, tabs, 2)
    srv = _server(ctx)
    a = srv.add_map(geos[0].speed, geos[0].h, geos[0].sensors, geos[0].pix, geos[0].n_samples, geos[0].dt)
    first = srv.wait(srv.submit(a, frames[0][1]), a, timeout_ms=WAIT_MS)
    b = srv.add_map(geos[1].speed, geos[1].h, geos[1].sensors, geos[1].pix, geos[1].n_samples, geos[1].dt)
    tick = [srv.submit(a, frames[0][1]) for _ in range(20)]
    tb = srv.submit(b, frames[2][1])
    for t in tick:
        assert np.array_equal(srv.wait(t, a, timeout_ms=WAIT_MS), first)
    img_b = srv.wait(tb, b, timeout_ms=WAIT_MS)
    ref = orc.backproject(tabs[1], frames[2][1], geos[1].dt)
    assert np.linalg.norm(img_b - ref) / np.linalg.norm(ref) < 2e-3
    assert srv.map_state(b) == pat.MAP_READY
    with pytest.raises(pat.PatError):
        srv.remove_map(12345)
    srv.remove_map(a)
    srv.close()


def test_server_3d_map(ctx, orc):
    # a 3-D map in the frame server beside a 2-D one: its table is built by
    # the 3-D eikonal solver on the build stream, and its frames match the
    # single-frame launch on the same (GPU) table and the all-oracle pipeline
    from paper_1501_03869_amd import pat
    g3 = inputs.config3("head3")
    sens = g3.sensors[::4]
    vox = pat.tile_order_3d(g3.nx, g3.ny, g3.nz, g3.pix, 4, 4, 2)
    g = inputs.Geometry3(g3.name, g3.nx, g3.ny, g3.nz, g3.h, g3.speed, sens, vox, g3.n_samples, g3.dt)
    T64 = orc.tables3(g3.speed, g3.h, sens, vox)
    frames = [inputs.frame_for3(g, T64, f) for f in range(3)]
    g2 = inputs.config("small")
    srv = pat.Server(ctx, max_batch=8)
    try:
        m2 = srv.add_map(g2.speed, g2.h, g2.sensors, g2.pix, g2.n_samples, g2.dt)
        m3 = srv.add_map_3d(g3.speed, g3.h, sens, vox, g3.n_samples, g3.dt)
        t2 = srv.submit(m2, inputs.random_signals(5, g2.S, g2.n_samples))
        imgs = [srv.wait(srv.submit(m3, f), m3, timeout_ms=WAIT_MS) for f in frames]
        srv.wait(t2, m2, timeout_ms=WAIT_MS)
        st = srv.stats()
    finally:
        srv.close()
    assert st["builds"] >= 2
    Tg = ctx.eikonal_tables_3d(torch.from_numpy(g3.speed).cuda(), g3.h, sens, torch.from_numpy(vox).cuda())
    for f, img in zip(frames, imgs):
        single = ctx.backproject(Tg, torch.from_numpy(f).cuda(), g3.dt, filtered=False).cpu().numpy()
        ref = orc.backproject(T64, f, g3.dt)
        e1 = float(np.linalg.norm(img - single) / np.linalg.norm(single))
        e2 = float(np.linalg.norm(img - ref) / np.linalg.norm(ref))
        print(f"[server 3d] rel L2 vs single launch {e1:.3e}, vs oracle pipeline {e2:.3e}", flush=True)
        assert e1 <= 1e-5
        assert e2 <= 2e-3


def test_budget_create_and_mixed_signal_formats(ctx, orc):
    # pat_server_create with an HBM budget only; float32 and binary16 frames
    # of two maps submitted together: each launch takes one format, and every
    # image equals the same frame submitted alone, bit for bit
    from paper_1501_03869_amd import pat
    geos = _maps()[:2]
    tabs = _oracle_tables(orc, geos)
    frames = _frames(geos, tabs, 3)
    srv = pat.Server(ctx, hbm_budget_bytes=2 << 30, budget_only=True)
    try:
        ids = _add_all(srv, geos)
        enc = []
        for k, (gi, p) in enumerate(frames):
            if k % 2:
                sc = float(np.abs(p).max() / 2.0 ** 14)
                enc.append((gi, (p / sc).astype(np.float16), sc, pat.SIG_F16))
            else:
                enc.append((gi, p, 1.0, pat.SIG_F32))
        alone = [srv.wait(srv.submit(ids[gi], p, sc, sig_fmt=fmt), ids[gi], timeout_ms=WAIT_MS)
                 for gi, p, sc, fmt in enc]
        srv.reset_stats()
        b0 = srv.stats()["batches"]
        srv.hold(True)
        tickets = [srv.submit(ids[gi], p, sc, sig_fmt=fmt) for gi, p, sc, fmt in enc]
        srv.hold(False)
        mixed = [srv.wait(t, ids[gi], timeout_ms=WAIT_MS) for t, (gi, _, _, _) in zip(tickets, enc)]
        st = srv.stats()
    finally:
        srv.close()
    assert st["bytes_budget"] == 2 << 30
    assert st["batches"] - b0 == 2  # one launch per signal format
    for k, (gi, p) in enumerate(frames):
        assert np.array_equal(alone[k], mixed[k]), k
        ref = orc.backproject(tabs[gi], p, geos[gi].dt, geos[gi].t0)
        err = np.linalg.norm(mixed[k] - ref) / np.linalg.norm(ref)
        assert err <= (2e-3 if k % 2 == 0 else 5e-3), (k, err)
