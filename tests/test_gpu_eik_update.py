"""The travel-time tables' local update, exact in integers, and the tables'
independence of the relaxation schedule.

pat_eikonal_update_eval evaluates the update the 2-D and 3-D solvers apply
(Section II-B, first-order upwind scheme on uint32 fixed-point times).  Its
definition: the largest T with sum_k max(2 (T - n_k) - 1, 0)^2 <= 4 F^2 over
the neighbour minima n_k, that is the first-order root rounded to the nearest
unit.  The checks here:
  - against that definition by a vectorised binary search over T (not the
    kernel's closed forms), exhaustively for small F and on random entries up
    to F = 2^23, the largest slowness the solvers produce;
  - monotone in every neighbour (raising one never lowers the result), the
    property that makes the relaxation's fixed point independent of the order
    of the node updates;
  - within half a unit of the continuous first-order root, evaluated in FP64
    by its textbook closed form over the sorted neighbours;
  - the tables themselves: the same bits whether the sensors are built in one
    call or in chunks (which changes how many maps each launch relaxes and so
    the workgroup schedule), in 2-D and 3-D, and whether the host learns each
    round's size by polling or by synchronising the stream."""
import numpy as np
import pytest

from paper_1501_03869_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

INF = 0xFFFFFFFF


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03869_amd import pat
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pat.Context(0)
    yield c
    c.close()


def gpu_update(nbr, F, dims):
    """nbr int64 [n][3] (uint32 values), F int64 [n] -> int64 [n]."""
    from paper_1501_03869_amd import pat
    nb = torch.from_numpy(np.ascontiguousarray(nbr.astype(np.uint32).view(np.int32))).cuda()
    f = torch.from_numpy(np.ascontiguousarray(F.astype(np.uint32).view(np.int32))).cuda()
    out = pat.eikonal_update_eval(nb, f, dims)
    return out.cpu().numpy().view(np.uint32).astype(np.int64)


def defined_update(nbr, F, dims):
    """Largest T with sum_k max(2 (T - n_k) - 1, 0)^2 <= 4 F^2, held below
    INF; INF when no neighbour is reached.  Binary search over [m, m + F]."""
    n = nbr[:, :dims].astype(np.int64)
    F = F.astype(np.int64)
    reached = n != INF
    m = np.where(reached, n, np.iinfo(np.int64).max).min(axis=1)
    none = ~reached.any(axis=1)
    m = np.where(none, 0, m)
    lim = 4 * F * F

    def G(T):
        x = 2 * (T[:, None] - n) - 1
        return np.where(reached & (x > 0), x * x, 0).sum(axis=1)

    lo, hi = m.copy(), m + F  # G(lo) = 0; G(m + F + 1) > 4 F^2
    while np.any(lo < hi):
        mid = (lo + hi + 1) // 2
        ok = G(mid) <= lim
        lo = np.where(ok, mid, lo)
        hi = np.where(ok, hi, mid - 1)
    return np.where(none, INF, np.minimum(lo, INF - 1))


def continuous_root(nbr, F, dims):
    """The first-order root in FP64 over the sorted neighbours: one-, two-
    or three-axis, whichever exceeds the neighbours it uses.  Solved over the
    offsets from the smallest neighbour, so that FP64 keeps the fraction."""
    out = np.empty(len(F))
    for i in range(len(F)):
        v = sorted(int(x) for x in nbr[i, :dims] if x != INF)
        base = v[0]
        o = [float(x - base) for x in v]
        f = float(F[i])
        T = f
        for k in range(2, len(o) + 1):
            if T <= o[k - 1]:
                break
            s = sum(o[:k])
            q = sum(x * x for x in o[:k])
            T = (s + np.sqrt(s * s - k * (q - f * f))) / k
        out[i] = base + T
    return out


def cases_2d():
    rows = []
    for F in range(0, 201):
        for d in range(0, 2 * F + 3):
            for base in (1000, 2 ** 31 + 12345):
                rows.append((base, base + d, 0, F))
                rows.append((base + d, base, 0, F))
    return np.array(rows, dtype=np.int64)


def cases_3d():
    rng = np.random.default_rng(7)
    rows = []
    for F in range(0, 41):
        for d in range(0, 2 * F + 2):
            for e in range(d, 2 * F + 2):
                v = np.array([5000, 5000 + d, 5000 + e])
                rng.shuffle(v)
                rows.append((*v, F))
    return np.array(rows, dtype=np.int64)


def cases_large(dims, n, seed):
    """Random slowness up to 2^23 with neighbour gaps spread over the three
    regimes and packed near their boundaries."""
    rng = np.random.default_rng(seed)
    F = rng.integers(1, 2 ** 23 + 1, n)
    F[: n // 8] = 2 ** 23 - rng.integers(0, 3, n // 8)
    a = rng.integers(0, 2 ** 31, n)
    d = (rng.random(n) * 2.2 * F).astype(np.int64)
    near = rng.random(n) < 0.3
    d = np.where(near, np.maximum(F - rng.integers(0, 4, n), 0), d)
    e = d + (rng.random(n) * 1.5 * F).astype(np.int64)
    c = a + e if dims == 3 else np.zeros(n, np.int64)
    return np.stack([a, a + d, c, F], axis=1)


def special_cases():
    F = 100
    return np.array([
        (INF, INF, INF, F),          # nothing reached
        (7, INF, INF, F),            # one neighbour: 7 + F
        (INF, 7, INF, F),
        (INF - 3, INF, INF, F),      # held below "not reached"
        (INF - 3, INF - 2, INF, F),
        (5, 5, INF, 0),              # zero slowness
        (5, 5, 5, 0),
        (0, 0, 0, 2 ** 23),          # the largest slowness
        (0, 2 ** 23 - 1, 2 ** 23 - 1, 2 ** 23),
    ], dtype=np.int64)


@pytest.mark.parametrize("dims", [2, 3])
def test_update_matches_its_definition(ctx, dims):
    rows = np.concatenate([cases_2d() if dims == 2 else cases_3d(), cases_large(dims, 200000, 11 + dims),
                           special_cases()])
    nbr, F = rows[:, :3].copy(), rows[:, 3]
    if dims == 2:
        nbr[:, 2] = 0
    got = gpu_update(nbr, F, dims)
    want = defined_update(nbr, F, dims)
    bad = np.flatnonzero(got != want)
    print(f"[eik update] {dims}-D: {len(F)} entries, {len(bad)} differ from the definition", flush=True)
    assert len(bad) == 0, f"first differing entries {rows[bad[:5]].tolist()}: got {got[bad[:5]]}, want {want[bad[:5]]}"


@pytest.mark.parametrize("dims", [2, 3])
def test_update_is_monotone(ctx, dims):
    rows = np.concatenate([cases_2d() if dims == 2 else cases_3d(), cases_large(dims, 100000, 21 + dims)])
    nbr, F = rows[:, :3].copy(), rows[:, 3]
    if dims == 2:
        nbr[:, 2] = 0
    base = gpu_update(nbr, F, dims)
    for k in range(dims):
        up = nbr.copy()
        up[:, k] += 1
        raised = gpu_update(up, F, dims)
        lowered = np.flatnonzero(raised < base)
        print(f"[eik update] {dims}-D, neighbour {k} raised by one: {len(lowered)} results fall", flush=True)
        assert len(lowered) == 0, f"entries {rows[lowered[:5]].tolist()}"


@pytest.mark.parametrize("dims", [2, 3])
def test_update_rounds_the_continuous_root(ctx, dims):
    rows = cases_large(dims, 5000, 31 + dims)
    nbr, F = rows[:, :3].copy(), rows[:, 3]
    if dims == 2:
        nbr[:, 2] = 0
    got = gpu_update(nbr, F, dims).astype(np.float64)
    root = continuous_root(nbr, F, dims)
    # T is an integer within half a unit of the root; the FP64 root of values
    # near 2^31 carries up to about 1e-6 of rounding
    err = np.abs(got - root).max()
    print(f"[eik update] {dims}-D: max |T - root| = {err:.6f} units", flush=True)
    assert err <= 0.5 + 1e-5


def test_update_rejects_bad_arguments(ctx):
    from paper_1501_03869_amd import pat
    nb = torch.zeros((4, 3), dtype=torch.int32, device="cuda")
    f = torch.zeros(4, dtype=torch.int32, device="cuda")
    with pytest.raises(pat.PatError):
        pat.eikonal_update_eval(nb, f, 4)
    assert pat.eikonal_update_eval(nb[:0], f[:0], 2).numel() == 0
    # slowness above 2^23 gives 0
    big = torch.full((4,), 2 ** 23 + 1, dtype=torch.int32, device="cuda")
    assert (pat.eikonal_update_eval(nb, big, 2).cpu() == 0).all()


def _tables(ctx, geo, sensors, pix, is3):
    sp = torch.from_numpy(geo.speed).cuda()
    px = torch.from_numpy(pix).cuda()
    if is3:
        return ctx.eikonal_tables_3d(sp, geo.h, sensors, px).cpu().numpy()
    return ctx.eikonal_tables(sp, geo.h, sensors, px).cpu().numpy()


@pytest.mark.parametrize("name,chunks", [("small", (1, 5, 17)), ("paper", (64, 100)), ("tiny3", (1, 4)),
                                         ("head3", (32, 100))])
def test_tables_same_bits_in_any_chunking(ctx, name, chunks):
    is3 = name in ("tiny3", "head3")
    geo = inputs.config3(name) if is3 else inputs.config(name)
    sensors = geo.sensors if len(geo.sensors) <= 256 else geo.sensors[:256]
    whole = _tables(ctx, geo, sensors, geo.pix, is3)
    again = _tables(ctx, geo, sensors, geo.pix, is3)
    assert np.array_equal(whole.view(np.uint32), again.view(np.uint32))
    for ch in chunks:
        parts = [_tables(ctx, geo, sensors[s:s + ch], geo.pix, is3) for s in range(0, len(sensors), ch)]
        split = np.concatenate(parts, axis=0)
        diff = int((split.view(np.uint32) != whole.view(np.uint32)).sum())
        print(f"[eik tables] {name}: {len(sensors)} sensors in chunks of {ch}: {diff} entries differ", flush=True)
        assert diff == 0


@pytest.mark.parametrize("name", ["paper", "tiny3"])
def test_tables_same_bits_when_rounds_synchronise(ctx, name, monkeypatch):
    """Between relaxation rounds the host polls a pinned word the device
    writes, and synchronises the stream instead when the word is late;
    PAT_EIK_SPIN_MS=0 takes that second path every round.  Both paths, and a
    short spin window, give the same tables (the rounds and visits, which
    follow the schedule, are printed)."""
    is3 = name == "tiny3"
    geo = inputs.config3(name) if is3 else inputs.config(name)
    sensors = geo.sensors if len(geo.sensors) <= 256 else geo.sensors[:256]
    monkeypatch.delenv("PAT_EIK_SPIN_MS", raising=False)
    polled = _tables(ctx, geo, sensors, geo.pix, is3)
    st_polled = ctx.eikonal_stats()
    for spin in ("0", "0.001"):
        monkeypatch.setenv("PAT_EIK_SPIN_MS", spin)
        other = _tables(ctx, geo, sensors, geo.pix, is3)
        st = ctx.eikonal_stats()
        diff = int((other.view(np.uint32) != polled.view(np.uint32)).sum())
        print(f"[eik tables] {name}: spin {spin} ms against polling: {diff} entries differ, rounds "
              f"{st['rounds']} / {st_polled['rounds']}, visits {st['tile_visits']} / {st_polled['tile_visits']}",
              flush=True)
        assert diff == 0
        assert st["rounds"] > 0 and st["tile_visits"] > 0


@pytest.mark.parametrize("name", ["small", "paper", "large"])
def test_tables_satisfy_the_scheme_at_every_node(ctx, name):
    """Every non-frozen ROI node whose four neighbours are ROI nodes, for
    every sensor and at full size: the table value T and the first-order root
    of its final neighbours (FP64, the node's exact slowness h/c) differ by at
    most ulp32(T) + lsb.  The bound follows from the arithmetic: the table
    rounds each time to float32 (half an ulp for T and for each neighbour,
    and the root moves by at most the largest neighbour change), and the
    integer update rounds the root to the nearest unit (half a unit) with the
    slowness rounded to whole units (at most half a unit more, since the
    root's slope in F is at most 1)."""
    geo = inputs.config(name)
    nx, ny, h = geo.nx, geo.ny, geo.h
    pix = geo.pix.astype(np.int64)
    P = len(pix)
    col_of = np.full(nx * ny, -1, np.int64)
    col_of[pix] = np.arange(P)
    i, j = pix % nx, pix // nx
    nb = []
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        nb.append(np.where(ok, col_of[np.clip(jj, 0, ny - 1) * nx + np.clip(ii, 0, nx - 1)], -1))
    inner = np.all(np.stack(nb) >= 0, axis=0)
    cols = np.flatnonzero(inner)
    W, E, Sn, N = (torch.from_numpy(x[inner]).cuda() for x in nb)
    colt = torch.from_numpy(cols).cuda()
    fh = torch.from_numpy(h / geo.speed.reshape(-1).astype(np.float64)[pix[inner]]).cuda()
    xs = torch.from_numpy((i[inner] - (nx - 1) / 2.0) * h).cuda()
    ys = torch.from_numpy((j[inner] - (ny - 1) / 2.0) * h).cuda()
    T = ctx.eikonal_tables(torch.from_numpy(geo.speed).cuda(), h, geo.sensors, torch.from_numpy(geo.pix).cuda())
    lsb = ctx.eikonal_stats()["lsb_seconds"]
    worst, checked = 0.0, 0
    for s0 in range(0, geo.S, 64):
        Tc = T[s0:s0 + 64].double()
        t = Tc[:, colt]
        a = torch.minimum(Tc[:, W], Tc[:, E])
        b = torch.minimum(Tc[:, Sn], Tc[:, N])
        m, d = torch.minimum(a, b), (a - b).abs()
        two = (a + b + torch.sqrt(torch.clamp(2 * fh * fh - d * d, min=0.0))) / 2
        upd = torch.where(d >= fh, m + fh, two)
        ulp = torch.pow(2.0, torch.floor(torch.log2(t)) - 23)
        bound = ulp + lsb + 1e-15 * t
        sens = torch.from_numpy(geo.sensors[s0:s0 + 64]).cuda()
        r = torch.sqrt((xs[None] - sens[:, :1]) ** 2 + (ys[None] - sens[:, 1:]) ** 2)
        live = r > 2.0 * h * (1 + 1e-9)
        ratio = torch.where(live, (t - upd).abs() / bound, torch.zeros_like(t))
        worst = max(worst, float(ratio.max()))
        checked += int(live.sum())
    print(f"[eik tables] {name}: {checked} node values of {geo.S} sensors checked, "
          f"max |T - root| / (ulp32(T) + lsb) = {worst:.3f}", flush=True)
    assert worst <= 1.0


def _root3(a, b, c, fh):
    """First-order root over the three axis minima (FP64 tensors), as the
    textbook sorted form: one-, two- or three-axis."""
    s = torch.stack([a, b, c])
    s, _ = torch.sort(s, dim=0)
    a, b, c = s[0], s[1], s[2]
    t1 = a + fh
    d = b - a
    t2 = (a + b + torch.sqrt(torch.clamp(2 * fh * fh - d * d, min=0.0))) / 2
    sm, sq = a + b + c, a * a + b * b + c * c
    t3 = (sm + torch.sqrt(torch.clamp(sm * sm - 3 * (sq - fh * fh), min=0.0))) / 3
    return torch.where(t1 <= b, t1, torch.where(t2 <= c, t2, t3))


@pytest.mark.parametrize("name", ["tiny3", "head3"])
def test_tables3_satisfy_the_scheme_at_every_node(ctx, name):
    """The 3-D form of the check above: every non-frozen ROI voxel whose six
    neighbours are ROI voxels, every sensor, within ulp32(T) + lsb of the
    root of its final neighbours (the three-axis root is also 1-Lipschitz in
    its neighbours, with slope at most 1 in F)."""
    geo = inputs.config3(name)
    nx, ny, nz, h = geo.nx, geo.ny, geo.nz, geo.h
    vox = geo.pix.astype(np.int64)
    P = len(vox)
    col_of = np.full(nx * ny * nz, -1, np.int64)
    col_of[vox] = np.arange(P)
    i, j, l = vox % nx, (vox // nx) % ny, vox // (nx * ny)
    nb = []
    for di, dj, dl in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        ii, jj, ll = i + di, j + dj, l + dl
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (ll >= 0) & (ll < nz)
        k2 = (np.clip(ll, 0, nz - 1) * ny + np.clip(jj, 0, ny - 1)) * nx + np.clip(ii, 0, nx - 1)
        nb.append(np.where(ok, col_of[k2], -1))
    inner = np.all(np.stack(nb) >= 0, axis=0)
    cols = torch.from_numpy(np.flatnonzero(inner)).cuda()
    nbt = [torch.from_numpy(x[inner]).cuda() for x in nb]
    fh = torch.from_numpy(h / geo.speed.reshape(-1).astype(np.float64)[vox[inner]]).cuda()
    pos = torch.from_numpy(np.stack([(i[inner] - (nx - 1) / 2.0) * h, (j[inner] - (ny - 1) / 2.0) * h,
                                     (l[inner] - (nz - 1) / 2.0) * h], axis=1)).cuda()
    T = ctx.eikonal_tables_3d(torch.from_numpy(geo.speed).cuda(), h, geo.sensors, torch.from_numpy(geo.pix).cuda())
    lsb = ctx.eikonal_stats()["lsb_seconds"]
    worst, checked = 0.0, 0
    for s0 in range(0, geo.S, 32):
        Tc = T[s0:s0 + 32].double()
        t = Tc[:, cols]
        ax = [torch.minimum(Tc[:, nbt[2 * q]], Tc[:, nbt[2 * q + 1]]) for q in range(3)]
        upd = _root3(ax[0], ax[1], ax[2], fh)
        ulp = torch.pow(2.0, torch.floor(torch.log2(t)) - 23)
        bound = ulp + lsb + 1e-15 * t
        sens = torch.from_numpy(geo.sensors[s0:s0 + 32]).cuda()
        r = torch.cdist(sens, pos)
        live = r > 2.0 * h * (1 + 1e-9)
        ratio = torch.where(live, (t - upd).abs() / bound, torch.zeros_like(t))
        worst = max(worst, float(ratio.max()))
        checked += int(live.sum())
    print(f"[eik3 tables] {name}: {checked} voxel values of {geo.S} sensors checked, "
          f"max |T - root| / (ulp32(T) + lsb) = {worst:.3f}", flush=True)
    assert worst <= 1.0


def test_random_media_satisfy_the_scheme_at_every_node(ctx):
    """Random small grids (2 x N strips, sizes across tile edges), speeds
    1000-4000 m/s per node, random sensors and every node in the ROI: every
    non-frozen node, edges included (a missing neighbour counts as +inf),
    is within ulp32(T) + lsb of the root of its final neighbours, and its
    increment over the smaller upwind neighbour lies in [f h / sqrt(2), f h]
    (causality), both up to the same bound."""
    rng = np.random.default_rng(4242)
    worst, worst_c = 0.0, 0.0
    for case in range(16):
        nx, ny = int(rng.integers(2, 41)), int(rng.integers(2, 41))
        if case == 0:
            nx, ny = 2, 37
        if case == 1:
            nx, ny = 40, 2
        h = float(rng.uniform(0.05e-3, 0.5e-3))
        c = rng.uniform(1000, 4000, size=(ny, nx)).astype(np.float32)
        x, y = inputs.node_coords(nx, ny, h)
        S = int(rng.integers(1, 6))
        sens = np.stack([rng.uniform(x[0], x[-1], S), rng.uniform(y[0], y[-1], S)], 1)
        pix = np.arange(nx * ny, dtype=np.int32)
        T = ctx.eikonal_tables(torch.from_numpy(c).cuda(), h, sens, torch.from_numpy(pix).cuda())
        lsb = ctx.eikonal_stats()["lsb_seconds"]
        t = T.double().cpu().numpy().reshape(S, ny, nx)
        pad = np.full((S, ny + 2, nx + 2), np.inf)
        pad[:, 1:-1, 1:-1] = t
        a = np.minimum(pad[:, 1:-1, :-2], pad[:, 1:-1, 2:])
        b = np.minimum(pad[:, :-2, 1:-1], pad[:, 2:, 1:-1])
        fh = h / c.astype(np.float64)
        m, M = np.minimum(a, b), np.maximum(a, b)
        d = M - m
        with np.errstate(invalid="ignore"):
            two = (a + b + np.sqrt(np.maximum(2 * fh * fh - d * d, 0.0))) / 2
        upd = np.where(d >= fh, m + fh, two)
        bound = 2.0 ** (np.floor(np.log2(t)) - 23) + lsb + 1e-15 * t
        r = np.sqrt((x[None, None, :] - sens[:, 0, None, None]) ** 2 + (y[None, :, None] - sens[:, 1, None, None]) ** 2)
        live = r > 2.0 * h * (1 + 1e-9)
        res = np.where(live, np.abs(t - upd) / bound, 0.0)
        inc = t - m
        caus = np.where(live, np.maximum(fh / np.sqrt(2) - inc, inc - fh) / bound, 0.0)
        worst, worst_c = max(worst, float(res.max())), max(worst_c, float(caus.max()))
        assert res.max() <= 1.0, (case, nx, ny)
        assert caus.max() <= 1.0, (case, nx, ny)
    print(f"[eik tables] random media: max |T - root| / bound {worst:.3f}; causality excess / bound {worst_c:.3f}",
          flush=True)


def test_tables_across_internal_chunks(ctx, orc):
    """A 2048^2 grid with 600 sensors: the working maps (16 MB each) exceed the
    8 GiB a build holds at once, so one call relaxes the sensors in two
    chunks (512 + 88).  The tables must be the same bits as two calls of 300
    sensors each, and the first sensor and the last (in the second chunk)
    must match the oracle's fast marching."""
    n, h = 2048, 0.05e-3
    rng = np.random.default_rng(2048)
    # a smooth medium: 1540 m/s with a faster ring between r = 30 and 36 mm
    x = (np.arange(n) - (n - 1) / 2.0) * h
    r = np.hypot(x[None, :], x[:, None])
    speed = np.where((r > 30e-3) & (r < 36e-3), 2600.0, 1540.0).astype(np.float32)
    ang = np.linspace(0, 2 * np.pi, 600, endpoint=False) + rng.uniform(0, 1e-3, 600)
    sensors = np.stack([40e-3 * np.cos(ang), 40e-3 * np.sin(ang)], 1)
    pix = np.arange(0, n * n, 97, dtype=np.int32)
    sp, px = torch.from_numpy(speed).cuda(), torch.from_numpy(pix).cuda()
    whole = ctx.eikonal_tables(sp, h, sensors, px).cpu().numpy()
    parts = np.concatenate([ctx.eikonal_tables(sp, h, sensors[s:s + 300], px).cpu().numpy() for s in (0, 300)])
    diff = int((whole.view(np.uint32) != parts.view(np.uint32)).sum())
    ref = orc.tables(speed, h, sensors[[0, 599]], pix)
    err = float((np.abs(whole[[0, 599]] - ref) / ref).max())
    print(f"[eik tables] 2048^2, 600 sensors in two internal chunks: {diff} entries differ from two calls; "
          f"sensors 0 and 599 against the oracle: max rel err {err:.3e}", flush=True)
    assert diff == 0
    assert err <= 1e-5


def test_tables3_across_internal_chunks(ctx):
    """A 256^3 grid with 150 sensors: the working maps (67 MB each) exceed the
    8 GiB a build holds at once, so one call relaxes the sensors in two
    chunks (128 + 22); the tables must be the same bits as two calls of 75."""
    n, h = 256, 0.5e-3
    x = (np.arange(n) - (n - 1) / 2.0) * h
    r = np.sqrt(x[None, None, :] ** 2 + x[None, :, None] ** 2 + x[:, None, None] ** 2)
    speed = np.where((r > 40e-3) & (r < 48e-3), 2600.0, 1540.0).astype(np.float32)
    rng = np.random.default_rng(256)
    v = rng.standard_normal((150, 3))
    sensors = 55e-3 * v / np.linalg.norm(v, axis=1, keepdims=True)
    vox = np.arange(0, n ** 3, 101, dtype=np.int32)
    sp, vx = torch.from_numpy(speed).cuda(), torch.from_numpy(vox).cuda()
    whole = ctx.eikonal_tables_3d(sp, h, sensors, vx).cpu().numpy()
    parts = np.concatenate([ctx.eikonal_tables_3d(sp, h, sensors[s:s + 75], vx).cpu().numpy() for s in (0, 75)])
    diff = int((whole.view(np.uint32) != parts.view(np.uint32)).sum())
    print(f"[eik3 tables] 256^3, 150 sensors in two internal chunks: {diff} entries differ from two calls", flush=True)
    assert np.all(np.isfinite(whole))
    assert diff == 0
