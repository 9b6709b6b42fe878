"""GPU tile server: every served tile equals the stand-alone call of the same request bit
for bit (the dyadic strip code for dyadic 2D requests, the general kernel otherwise, as the
result reports), alone and in a mixed, continuously arriving stream; samples agree with the
FP64 oracle within 1e-5 * A."""
import threading
import time

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu
F0 = 2.0 ** -12


def _mix(n, seed, non_dyadic=0.0):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        dim = 3 if rng.random() < 0.2 else 2
        smooth = int(rng.integers(1, 3))
        f0 = F0 * 1.37 if rng.random() < non_dyadic else F0  # non-dyadic ladders take the general tiles
        if dim == 2:
            side = int(rng.choice([16, 64, 100, 128, 256, 300]))
            octs = int(rng.integers(4, 13))
            ext = (side, int(rng.choice([side, side // 2 + 3])), 1)
        else:
            side = int(rng.choice([8, 32, 64]))
            octs = int(rng.integers(4, 9))
            ext = (side, side, int(rng.choice([side, 5])))
        org = tuple(int(v) for v in rng.integers(-(1 << 46), 1 << 46, size=dim)) + (0,) * (3 - dim)
        reqs.append(dict(dim=dim, smoothness=smooth, octaves=octs, base_freq=f0, persistence=0.5, lacunarity=2.0,
                         seed=int(rng.integers(0, 1 << 32)), origin=org, extent=ext, user_tag=i))
    return reqs


def _solo(r, kernel):
    """The stand-alone call with the kernel family the server used for the request."""
    nx, ny, nz = r["extent"]
    kw = dict(smoothness=r["smoothness"], octaves=r["octaves"], base_freq=r["base_freq"], seed=r["seed"],
              persistence=r["persistence"], lacunarity=r["lacunarity"])
    if r["dim"] == 2:
        out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
        path = "dyadic" if kernel == ptg.PTG_TUNE_STRIP_2D else "general"
        ptg.fbm_2d(out, x0=r["origin"][0], y0=r["origin"][1], path=path, **kw)
    else:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
        path = "dyadic" if kernel == ptg.PTG_TUNE_STRIP_3D else "general"
        ptg.fbm_3d(out, x0=r["origin"][0], y0=r["origin"][1], z0=r["origin"][2], path=path, **kw)
    torch.cuda.current_stream().synchronize()  # not the device: the server's kernel may be running
    return out


def _fetch(res, r):
    nx, ny, nz = r["extent"]
    t = torch.empty((nz, ny, nx) if r["dim"] == 3 else (ny, nx), dtype=torch.float32, device="cuda")
    ptg.device_copy(t.data_ptr(), res.out_dev, res.bytes)
    return t


def _tile_req(r):
    q = dict(r)
    return ptg.tile_req(dim=q.pop("dim"), origin=q.pop("origin"), extent=q.pop("extent"), user_tag=q.pop("user_tag"),
                        **q)


def test_served_tiles_equal_solo_calls_bit_exact():
    reqs = _mix(40, 1610, non_dyadic=0.3)
    with ptg.Server(1 << 30) as srv:
        tickets = srv.submit([_tile_req(r) for r in reqs])
        for t, r in zip(tickets, reqs):
            res = srv.wait(t, int(60e9))
            assert res.status == ptg.PTG_OK and res.user_tag == r["user_tag"]
            got = _fetch(res, r)
            srv.release(t)
            dyadic = r["base_freq"] == F0  # 3D ladders here end at period >= 32
            want = (ptg.PTG_TUNE_STRIP_2D if dyadic else ptg.PTG_TUNE_GENERAL_2D) if r["dim"] == 2 else (
                ptg.PTG_TUNE_STRIP_3D if dyadic else ptg.PTG_TUNE_GENERAL_3D)
            assert res.kernel == want, (res.kernel, r)
            assert torch.equal(got, _solo(r, res.kernel)), r
        st = srv.stats()
        assert st["completed"] == 40 and st["bytes_peak"] <= (1 << 30)


def _solo_model(r, kernel):
    """The stand-alone call with the request's cell model and the kernel family the server
    used."""
    nx, ny, nz = r["extent"]
    kw = dict(smoothness=r["smoothness"], octaves=r["octaves"], base_freq=r["base_freq"], seed=r["seed"],
              model=r["model"], gradient_weight=r["gradient_weight"])
    if r["dim"] == 2:
        out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
        path = "dyadic" if kernel == ptg.PTG_TUNE_STRIP_2D else "general"
        ptg.fbm_2d(out, x0=r["origin"][0], y0=r["origin"][1], path=path, **kw)
    else:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
        path = "dyadic" if kernel == ptg.PTG_TUNE_STRIP_3D else "general"
        ptg.fbm_3d(out, x0=r["origin"][0], y0=r["origin"][1], z0=r["origin"][2], path=path, **kw)
    torch.cuda.current_stream().synchronize()
    return out


def test_served_cell_models_and_orders_equal_solo_calls_bit_exact():
    """Zero-gradient (2D C1), height-and-gradient (2D C1..C3, 3D C1 / C2 on the strip code and
    C3 on general tiles) and septic gradient cells, on dyadic and non-dyadic ladders, in one
    mix: each served tile equals the stand-alone call of the same kernel family bit for bit,
    and the family is the one a dense call would take."""
    rng = np.random.default_rng(1613)
    cases = [(2, "zero_gradient", 1), (2, "height_gradient", 1), (2, "height_gradient", 2), (2, "height_gradient", 3),
             (2, "gradient", 3), (3, "height_gradient", 1), (3, "height_gradient", 2), (3, "gradient", 3),
             (3, "height_gradient", 3)]
    reqs = []
    for i, (dim, model, sm) in enumerate(cases * 2):
        dyadic = i < len(cases)
        f0 = F0 if dyadic else F0 * 1.37
        if dim == 2:
            ext = (int(rng.choice([100, 256, 300])), int(rng.choice([77, 128, 256])), 1)
            octs = int(rng.integers(4, 10))
        else:
            ext = (int(rng.choice([32, 64])), int(rng.choice([16, 40])), int(rng.choice([16, 33])))
            octs = int(rng.integers(3, 7))
        org = tuple(int(v) for v in rng.integers(-(1 << 44), 1 << 44, size=dim)) + (0,) * (3 - dim)
        reqs.append(dict(dim=dim, smoothness=sm, octaves=octs, base_freq=f0, persistence=0.5, lacunarity=2.0,
                         seed=int(rng.integers(0, 1 << 32)), origin=org, extent=ext, user_tag=i, model=model,
                         gradient_weight=float(rng.choice([0.01, 0.5]))))
    with ptg.Server(1 << 30) as srv:
        tickets = srv.submit([_tile_req(r) for r in reqs])
        for t, r in zip(tickets, reqs):
            res = srv.wait(t, int(60e9))
            assert res.status == ptg.PTG_OK, r
            got = _fetch(res, r)
            srv.release(t)
            shape = (r["extent"][0], r["extent"][1]) if r["dim"] == 2 else r["extent"]
            kw = {k: r[k] for k in ("smoothness", "octaves", "base_freq", "model", "gradient_weight")}
            dense_kind = ptg.tune_query(tuple(reversed(shape)), **kw)[0]
            assert ptg.TUNE_NAMES[res.kernel] == dense_kind, (res.kernel, dense_kind, r)
            assert torch.equal(got, _solo_model(r, res.kernel)), r


def test_wait_any_returns_each_completion_once_in_completion_order():
    """ptg_tiles_wait_any over a mix: every ticket comes back exactly once, completion times
    never decrease, and each output equals the stand-alone call."""
    reqs = _mix(30, 1611, non_dyadic=0.2)
    with ptg.Server(1 << 30) as srv:
        tickets = srv.submit([_tile_req(r) for r in reqs])
        index = {t: i for i, t in enumerate(tickets)}
        seen, last = [], 0
        for _ in reqs:
            t, res = srv.wait_any(int(60e9))
            assert res.status == ptg.PTG_OK and t in index and t not in seen
            assert res.t_done_ns >= last
            last = res.t_done_ns
            r = reqs[index[t]]
            assert res.user_tag == r["user_tag"]
            got = _fetch(res, r)
            srv.release(t)
            assert torch.equal(got, _solo(r, res.kernel)), r
            seen.append(t)
        with pytest.raises(ptg.PtgError) as e:
            srv.wait_any(0)
        assert e.value.code == ptg.PTG_ENOENT


def _overlaps(results):
    """Pairs of requests whose [admission, completion] intervals intersect: both were on the
    device at once."""
    iv = sorted((r.t_admit_ns, r.t_done_ns) for r in results)
    n = 0
    for i in range(len(iv)):
        for j in range(i + 1, len(iv)):
            if iv[j][0] < iv[i][1]:
                n += 1
    return n


def test_alone_and_in_a_continuous_mix_are_identical():
    """Every request of a mixed stream is computed alone first (one at a time on an idle
    server), then the whole stream arrives in bursts while earlier bursts are still running:
    each result in the mix equals its result alone bit for bit, and requests demonstrably
    overlapped on the device (admitted before another one completed)."""
    reqs = _mix(30, 7)
    with ptg.Server(1 << 29) as srv:
        alone = {}
        for r in reqs:
            (t,) = srv.submit([_tile_req(r)])
            alone[r["user_tag"]] = _fetch(srv.wait(t, int(60e9)), r)
            srv.release(t)
        got = {}

        def submitter():
            for b in range(0, len(reqs), 6):  # bursts of 6, 1 ms apart
                ts = srv.submit([_tile_req(r) for r in reqs[b:b + 6]])
                for r, t in zip(reqs[b:b + 6], ts):
                    got[r["user_tag"]] = t
                time.sleep(0.001)

        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        results = []
        for r in reqs:
            res = srv.wait(got[r["user_tag"]], int(60e9))
            assert res.status == ptg.PTG_OK
            assert torch.equal(_fetch(res, r), alone[r["user_tag"]]), r
            results.append(res)
            srv.release(got[r["user_tag"]])
        assert _overlaps(results) > 0
        probe = results[5]
        assert any(o is not probe and o.t_admit_ns < probe.t_done_ns and probe.t_admit_ns < o.t_done_ns
                   for o in results)


def test_largest_stream_requests_served_bit_exact_and_against_oracle():
    """The stream's largest requests -- 2048^2 2D tiles with 12 octaves (C1 and C2) and a
    256^3 3D tile with 8 octaves (C2, 64 MiB) -- submitted together with small ones: each
    equals its stand-alone call bit for bit, samples agree with the FP64 oracle, and the
    requests overlapped on the device."""
    rng = np.random.default_rng(2048)
    big = []
    for i, (dim, smooth, octs, ext) in enumerate([(2, 1, 12, (2048, 2048, 1)), (2, 2, 12, (2048, 2048, 1)),
                                                   (3, 2, 8, (256, 256, 256)), (2, 1, 7, (128, 128, 1)),
                                                   (3, 1, 4, (64, 64, 64)), (2, 2, 9, (512, 512, 1))]):
        org = tuple(int(v) for v in rng.integers(-(1 << 46), 1 << 46, size=dim)) + (0,) * (3 - dim)
        big.append(dict(dim=dim, smoothness=smooth, octaves=octs, base_freq=F0, persistence=0.5, lacunarity=2.0,
                        seed=int(rng.integers(0, 1 << 32)), origin=org, extent=ext, user_tag=i))
    with ptg.Server(1 << 30) as srv:
        tickets = srv.submit([_tile_req(r) for r in big])
        results = []
        for t, r in zip(tickets, big):
            res = srv.wait(t, int(120e9))
            assert res.status == ptg.PTG_OK
            got = _fetch(res, r)
            results.append(res)
            srv.release(t)
            assert torch.equal(got, _solo(r, res.kernel)), r
            g = got.cpu().numpy().astype(np.float64)
            A = sum(0.5 ** o for o in range(r["octaves"]))
            k = 400
            if r["dim"] == 2:
                i, j = rng.integers(0, r["extent"][0], k), rng.integers(0, r["extent"][1], k)
                ref = O.fbm_points_2d(r["smoothness"], r["octaves"], 0.5, 2.0, F0, r["seed"], r["origin"][0] + i,
                                      r["origin"][1] + j)
                assert np.max(np.abs(g[j, i] - ref)) <= 1e-5 * A, r
            else:
                i, j, l = (rng.integers(0, r["extent"][a], k) for a in range(3))
                ref = O.fbm_points_3d(r["smoothness"], r["octaves"], 0.5, 2.0, F0, r["seed"], r["origin"][0] + i,
                                      r["origin"][1] + j, r["origin"][2] + l)
                assert np.max(np.abs(g[l, j, i] - ref)) <= 1e-5 * A, r
        assert _overlaps(results) > 0


def _drain(srv, tickets, reqs, timeout_s=60.0):
    """Take completions in whatever order they come and release each at once: with a small
    budget, completed outputs hold arena bytes until released, so waiting in submission
    order could keep a request that later ones passed from ever being admitted."""
    left = dict(zip(tickets, reqs))
    t_end = time.time() + timeout_s
    while left:
        assert time.time() < t_end, f"{len(left)} requests still pending"
        for t in list(left):
            try:
                res = srv.wait(t, 1_000_000)
            except ptg.PtgError as e:
                if e.code == ptg.PTG_ETIMEDOUT:
                    continue
                raise
            r = left.pop(t)
            assert torch.equal(_fetch(res, r), _solo(r, res.kernel)), r
            srv.release(t)


def test_kernel_relaunches_after_idle_and_small_budget_admission():
    reqs = _mix(12, 3)
    biggest = max(r["extent"][0] * r["extent"][1] * r["extent"][2] * 4 for r in reqs)
    with ptg.Server(biggest + 4096) as srv:  # room for about one request at a time
        _drain(srv, srv.submit([_tile_req(r) for r in reqs[:6]]), reqs[:6])
        time.sleep(0.1)  # the persistent kernel is parked after 5 ms with nothing in flight
        _drain(srv, srv.submit([_tile_req(r) for r in reqs[6:]]), reqs[6:])
        st = srv.stats()
        assert st["kernel_launches"] >= 2 and st["bytes_peak"] <= biggest + 4096


def _lat_mix(n, seed):
    """General 2D requests over a few seeds and overlapping windows, so lattice blocks are
    shared between requests; one far from the origin (negative block indices)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        side = int(rng.choice([64, 100, 160, 256]))
        reqs.append(dict(dim=2, smoothness=int(rng.integers(1, 3)), octaves=int(rng.integers(3, 8)),
                         base_freq=float(rng.choice([0.0031, 0.0077, 0.013])), persistence=0.5, lacunarity=2.0,
                         seed=int(rng.choice([7, 8, 9])), origin=(int(rng.integers(-600, 600)),
                                                                  int(rng.integers(-600, 600)), 0),
                         extent=(side, side // 2 + 7, 1), user_tag=i))
    reqs.append(dict(dim=2, smoothness=2, octaves=7, base_freq=0.0077, persistence=0.5, lacunarity=2.0, seed=7,
                     origin=(-(1 << 45) + 17, (1 << 44) + 5, 0), extent=(130, 70, 1), user_tag=n))
    return reqs


@pytest.mark.parametrize("budget", [1 << 30, 3 << 20])
def test_lattice_cache_tiles_equal_solo_calls_bit_exact(budget):
    """With the lattice cache the general 2D tiles read their node gradients from blocks
    that the persistent kernel filled (shared by requests of one seed; evicted and refilled
    under the small budget): every tile equals the stand-alone general call bit for bit."""
    reqs = _lat_mix(40, 31)
    with ptg.Server(budget, lattice_cache=1) as srv:
        _drain(srv, srv.submit([_tile_req(r) for r in reqs[:20]]), reqs[:20])
        _drain(srv, srv.submit([_tile_req(r) for r in reqs[20:]]), reqs[20:])  # blocks resident from the first half
        st = srv.stats()
        assert st["lat_hits"] > 0 and st["lat_misses"] > 0 and st["completed"] == len(reqs)
        assert st["bytes_peak"] <= budget
        if budget < (1 << 24):
            assert st["lat_evictions"] > 0


def test_lattice_cached_samples_match_oracle():
    r = dict(dim=2, smoothness=1, octaves=7, base_freq=0.0093, persistence=0.5, lacunarity=2.0, seed=4242,
             origin=(-(1 << 43) - 29, (1 << 42) + 3, 0), extent=(190, 120, 1), user_tag=1)
    with ptg.Server(1 << 26, lattice_cache=1) as srv:
        g = []
        for _ in range(2):  # filled, then found resident
            (t,) = srv.submit([_tile_req(r)])
            g.append(_fetch(srv.wait(t, int(60e9)), r).cpu().numpy().astype(np.float64))
            srv.release(t)
        st = srv.stats()
        assert st["lat_misses"] > 0 and st["lat_hits"] == st["lat_misses"]
    assert np.array_equal(g[0], g[1])
    rng = np.random.default_rng(1)
    i = rng.integers(0, 190, 500)
    j = rng.integers(0, 120, 500)
    ref = O.fbm_points_2d(1, 7, 0.5, 2.0, 0.0093, 4242, r["origin"][0] + i, r["origin"][1] + j)
    assert np.max(np.abs(g[0][j, i] - ref)) <= 1e-5 * sum(0.5 ** o for o in range(7))


def test_served_samples_match_oracle():
    r = dict(dim=2, smoothness=2, octaves=12, base_freq=F0, persistence=0.5, lacunarity=2.0, seed=99,
             origin=((1 << 40) + 17, -(1 << 41) - 3, 0), extent=(200, 150, 1), user_tag=1)
    with ptg.Server(1 << 24) as srv:
        (t,) = srv.submit([_tile_req(r)])
        g = _fetch(srv.wait(t, int(60e9)), r).cpu().numpy().astype(np.float64)
        srv.release(t)
    rng = np.random.default_rng(0)
    i = rng.integers(0, 200, 500)
    j = rng.integers(0, 150, 500)
    ref = O.fbm_points_2d(2, 12, 0.5, 2.0, F0, 99, r["origin"][0] + i, r["origin"][1] + j)
    assert np.max(np.abs(g[j, i] - ref)) <= 1e-5 * sum(0.5 ** o for o in range(12))


def _plain_stream_matches_solo_calls(modes):
    import ctypes
    import os
    lg = ctypes.CDLL(os.path.join(os.path.dirname(ptg.LIB_PATH), "libptg_loadgen.so"))
    p64 = ctypes.POINTER(ctypes.c_int64)
    lg.ptg_lg_plain.argtypes = [ctypes.POINTER(ptg.TileReq), p64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_int32, ctypes.c_int32, p64, p64]
    reqs = _mix(24, 11)
    n = len(reqs)
    tr = (ptg.TileReq * n)(*[_tile_req(r) for r in reqs])
    sizes = [r["extent"][0] * r["extent"][1] * r["extent"][2] * 4 for r in reqs]
    offs, o = [], 0
    for b in sizes:
        offs.append(o)
        o += (b + 255) & ~255
    arena = torch.zeros(o, dtype=torch.uint8, device="cuda")
    for mode in modes:
        arena.zero_()
        torch.cuda.synchronize()
        arr = np.ascontiguousarray(np.arange(n) * 100_000, dtype=np.int64)
        done = np.zeros(n, dtype=np.int64)
        st = np.zeros(3, dtype=np.int64)
        rc = lg.ptg_lg_plain(tr, arr.ctypes.data_as(p64), n, arena.data_ptr(), o, mode, 8, done.ctypes.data_as(p64),
                             st.ctypes.data_as(p64))
        assert rc == ptg.PTG_OK, (mode, rc)
        if mode == 2:  # solo: per-request kernel times
            assert np.all(done > 0) and st[0] == n
        else:
            assert np.all(done >= arr) and 1 <= st[0] <= n
        for r, off, b in zip(reqs, offs, sizes):
            got = arena[off:off + b].view(torch.float32)
            want = _solo_auto(r).reshape(-1)
            assert torch.equal(got, want), (mode, r)


def test_plain_stream_direct_and_solo_write_what_solo_calls_write():
    """The benchmark's plain per-tile stream (native driver; direct launches at the arrival
    times, and the solo pass that times each request alone) leaves each request's output at
    its arena offset equal to the same ptg_fbm_* call made on its own."""
    _plain_stream_matches_solo_calls((0, 2))


@pytest.mark.skip(reason="the stream driver's graph mode is switched off: an open-loop stream of one-request "
                         "graphs updated in place ended the process with a segmentation fault of unknown cause")
def test_plain_stream_graph_batched_writes_what_solo_calls_write():
    _plain_stream_matches_solo_calls((1,))


def _solo_auto(r):
    nx, ny, nz = r["extent"]
    kw = dict(smoothness=r["smoothness"], octaves=r["octaves"], base_freq=r["base_freq"], seed=r["seed"],
              persistence=r["persistence"], lacunarity=r["lacunarity"])
    if r["dim"] == 2:
        out = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
        ptg.fbm_2d(out, x0=r["origin"][0], y0=r["origin"][1], **kw)
    else:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device="cuda")
        ptg.fbm_3d(out, x0=r["origin"][0], y0=r["origin"][1], z0=r["origin"][2], **kw)
    torch.cuda.current_stream().synchronize()
    return out
