"""Error paths on the GPU, forced from the host so that every kernel still runs
to completion: the eikonal round cap (PAT_ENOCONV) and device allocation
failures (PAT_ENOMEM) in a context and in the frame server.  After each
failure the context or server must keep working."""
import numpy as np
import pytest

from paper_1501_03869_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

WAIT_MS = 60000


@pytest.fixture(scope="module")
def pat_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_03869_amd import pat
    return pat


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_round_cap_gives_enoconv_and_context_recovers(pat_mod, orc, monkeypatch):
    pat = pat_mod
    g = inputs.config("small")
    ctx = pat.Context(0)
    try:
        speed, pix = _dev(g.speed), _dev(g.pix)
        monkeypatch.setenv("PAT_EIK_ROUND_CAP", "2")
        with pytest.raises(pat.PatError) as e:
            ctx.eikonal_tables(speed, g.h, g.sensors, pix)
        assert e.value.code == pat.PAT_ENOCONV
        g3 = inputs.config3("tiny3")
        with pytest.raises(pat.PatError) as e:
            ctx.eikonal_tables_3d(_dev(g3.speed), g3.h, g3.sensors, _dev(g3.pix))
        assert e.value.code == pat.PAT_ENOCONV
        monkeypatch.delenv("PAT_EIK_ROUND_CAP")
        # the same context then builds the full tables
        T = ctx.eikonal_tables(speed, g.h, g.sensors, pix).cpu().numpy()
        ref = orc.tables(g.speed, g.h, g.sensors, g.pix)
        err = float((np.abs(T - ref) / ref).max())
        print(f"[round cap] rounds {ctx.eikonal_stats()['rounds']}, max rel err after recovery {err:.2e}", flush=True)
        assert ctx.eikonal_stats()["rounds"] > 2
        assert err <= 1e-5
    finally:
        ctx.close()


def test_allocation_failure_in_context(pat_mod, orc, monkeypatch):
    pat = pat_mod
    monkeypatch.setenv("PAT_FAULT_ALLOC_BYTES", str(1 << 20))
    ctx = pat.Context(0)
    monkeypatch.delenv("PAT_FAULT_ALLOC_BYTES")
    try:
        g = inputs.config("small")  # 64 working maps of 128^2: 4 MiB, refused
        with pytest.raises(pat.PatError) as e:
            ctx.eikonal_tables(_dev(g.speed), g.h, g.sensors, _dev(g.pix))
        assert e.value.code == pat.PAT_ENOMEM
        # smaller work still runs on the same context
        t = inputs.config("tiny")
        T = ctx.eikonal_tables(_dev(t.speed), t.h, t.sensors, _dev(t.pix)).cpu().numpy()
        ref = orc.tables(t.speed, t.h, t.sensors, t.pix)
        assert float((np.abs(T - ref) / ref).max()) <= 1e-5
        # a gather that needs partial sums above the threshold is refused; the
        # split-sensor gather (no scratch) still runs
        S, P, N, dt = 512, 70000, 3, 4e-8  # N < 4: the windowed kernel with sensor groups
        need = pat.backproject_scratch_bytes(S, P, 1)
        assert need >= (1 << 20)
        tab = _dev(inputs.random_table(1, S, P, N, dt))
        sig = _dev(inputs.random_signals(2, S, N))
        with pytest.raises(pat.PatError) as e:
            ctx.backproject(tab, sig, dt, filtered=False)
        assert e.value.code == pat.PAT_ENOMEM
        N = 64
        tab = _dev(inputs.random_table(3, S, P, N, dt))
        sig = _dev(inputs.random_signals(4, S, N))
        img = ctx.backproject(tab, sig, dt, filtered=False).cpu().numpy()
        ref = orc.backproject(tab.cpu().numpy().astype(np.float64), sig.cpu().numpy(), dt)
        assert np.linalg.norm(img - ref) / np.linalg.norm(ref) <= 1e-4
    finally:
        ctx.close()


def test_allocation_failure_in_server(pat_mod, orc, monkeypatch):
    # the paper-scale map's 43.6 MB table is refused; its build fails with
    # PAT_ENOMEM while the small map keeps serving frames
    pat = pat_mod
    ctx = pat.Context(0)
    monkeypatch.setenv("PAT_FAULT_ALLOC_BYTES", str(20 << 20))
    srv = pat.Server(ctx, max_batch=8)
    monkeypatch.delenv("PAT_FAULT_ALLOC_BYTES")
    try:
        small, paper = inputs.config("small"), inputs.config("paper")
        tab = orc.tables(small.speed, small.h, small.sensors, small.pix)
        frames = [inputs.frame_for(small, tab, f) for f in range(3)]
        a = srv.add_map(small.speed, small.h, small.sensors, small.pix, small.n_samples, small.dt)
        first = srv.wait(srv.submit(a, frames[0]), a, timeout_ms=WAIT_MS)
        b = srv.add_map(paper.speed, paper.h, paper.sensors, paper.pix, paper.n_samples, paper.dt)
        pb = inputs.random_signals(9, paper.S, paper.n_samples)
        tick_b = None
        try:
            tick_b = srv.submit(b, pb)
        except pat.PatError as err:  # the build may already have failed
            assert err.code == pat.PAT_ENOMEM
        ticks = [srv.submit(a, f) for f in frames]
        if tick_b is not None:
            with pytest.raises(pat.PatError) as e:
                srv.wait(tick_b, b, timeout_ms=WAIT_MS)
            assert e.value.code == pat.PAT_ENOMEM
        assert srv.map_state(b) == pat.MAP_FAILED
        imgs = [srv.wait(t, a, timeout_ms=WAIT_MS) for t in ticks]
        assert np.array_equal(imgs[0], first)
        for f, img in zip(frames, imgs):
            ref = orc.backproject(tab, f, small.dt)
            assert np.linalg.norm(img - ref) / np.linalg.norm(ref) <= 2e-3
        with pytest.raises(pat.PatError) as e:
            srv.submit(b, pb)
        assert e.value.code == pat.PAT_ENOMEM
        # the failed map can be removed and a new map that fits is built
        srv.remove_map(b)
        c = srv.add_map(small.speed, small.h, small.sensors[::2], small.pix, small.n_samples, small.dt)
        img_c = srv.wait(srv.submit(c, frames[1][::2]), c, timeout_ms=WAIT_MS)
        ref_c = orc.backproject(tab[::2], frames[1][::2], small.dt)
        assert np.linalg.norm(img_c - ref_c) / np.linalg.norm(ref_c) <= 2e-3
        st = srv.stats()
        print(f"[server alloc failure] builds {st['builds']} frames {st['frames_done']}", flush=True)
        assert st["builds"] == 2
    finally:
        srv.close()
        ctx.close()
