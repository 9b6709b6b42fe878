"""Tile-shape autotuner on the GPU: every candidate shape of a kernel class writes the same
field bit for bit (the shape changes the schedule, not the arithmetic), the tuner records a
candidate and leaves the field in the output, and a server with tuned or fixed 2D tile
heights serves tiles equal to the stand-alone general-kernel call."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(autouse=True)
def _clean_table():
    ptg.tune_reset()
    yield
    ptg.tune_reset()


def _field2(shape, x0, y0, **kw):
    out = torch.empty(shape, dtype=torch.float32, device=DEV)
    ptg.fbm_2d(out, x0=x0, y0=y0, **kw)
    torch.cuda.current_stream().synchronize()
    return out


def _field3(shape, x0, y0, z0, **kw):
    out = torch.empty(shape, dtype=torch.float32, device=DEV)
    ptg.fbm_3d(out, x0=x0, y0=y0, z0=z0, **kw)
    torch.cuda.current_stream().synchronize()
    return out


@pytest.mark.parametrize("smooth", [1, 2])
def test_general_2d_tile_heights_are_bit_identical(smooth):
    kw = dict(smoothness=smooth, octaves=7, persistence=0.6, lacunarity=2.1, base_freq=0.0071, seed=3)
    shape, x0, y0 = (150, 131), -77, 2 ** 35 + 13
    assert ptg.tune_query(shape, **kw)[0] == "general_2d"
    fields = {}
    for th in (16, 32, 64, 128):
        ptg.tune_set(shape, th, **kw)
        assert ptg.tune_query(shape, **kw) == ("general_2d", th)
        fields[th] = _field2(shape, x0, y0, **kw)
    assert all(torch.equal(fields[th], fields[64]) for th in (16, 32, 128))
    ref = O.fbm_2d(smooth, 7, 0.6, 2.1, 0.0071, 3, x0, y0, shape[1], shape[0])
    amp = sum(0.6 ** o for o in range(7))
    assert np.max(np.abs(fields[16].cpu().numpy().astype(np.float64) - ref)) <= 1e-5 * amp


@pytest.mark.parametrize("smooth", [1, 2])
def test_strip_kernel_waves_are_bit_identical(smooth):
    kw = dict(smoothness=smooth, octaves=8, base_freq=2.0 ** -10, seed=9)
    shape = (300, 333)
    assert ptg.tune_query(shape, **kw)[0] == "strip_2d"
    fields = [None] * 5
    for w in (1, 2, 4):
        ptg.tune_set(shape, w, **kw)
        fields[w] = _field2(shape, -5, 70, **kw)
    assert torch.equal(fields[1], fields[4]) and torch.equal(fields[2], fields[4])
    kw3 = dict(smoothness=smooth, octaves=6, base_freq=1 / 64, seed=9)
    shape3 = (13, 19, 130)
    assert ptg.tune_query(shape3, **kw3)[0] == "strip_3d"
    vols = [None] * 5
    for w in (1, 2, 4):
        ptg.tune_set(shape3, w, **kw3)
        vols[w] = _field3(shape3, 3, -11, 7, **kw3)
    assert torch.equal(vols[1], vols[4]) and torch.equal(vols[2], vols[4])


@pytest.mark.parametrize("kw,kind", [
    (dict(octaves=6, base_freq=0.011, seed=4), "general_2d"),
    (dict(octaves=8, base_freq=2.0 ** -9, seed=4), "strip_2d"),
])
def test_tune_records_a_candidate_and_writes_the_field(kw, kind):
    shape = (512, 512)
    out = torch.empty(shape, dtype=torch.float32, device=DEV)
    r = ptg.tune_2d(out, reps=3, **kw)
    torch.cuda.current_stream().synchronize()
    assert r["kernel"] == kind and r["value"] in r["candidates"]
    assert len(r["candidates"]) == (4 if kind == "general_2d" else 3)  # tile heights / waves per workgroup
    assert all(us > 0 for us in r["candidates"].values())
    assert ptg.tune_query(shape, **kw) == (kind, r["value"])
    assert torch.equal(out, _field2(shape, 0, 0, **kw))


def test_tune_3d_and_untunable_classes():
    vol = torch.empty((16, 16, 128), dtype=torch.float32, device=DEV)
    r = ptg.tune_3d(vol, reps=2, smoothness=2, octaves=6, base_freq=1 / 64)
    assert r["kernel"] == "strip_3d" and r["value"] in (1, 2, 4)
    r = ptg.tune_3d(vol, reps=2, smoothness=1, octaves=4, base_freq=0.03)
    torch.cuda.current_stream().synchronize()
    assert r["kernel"] == "general_3d" and r["value"] == 0 and len(r["candidates"]) == 1


def _served_equals_solo(srv):
    # non-dyadic ladders: the server computes them as general tiles of the tuned height
    reqs = [dict(smoothness=m, octaves=o, base_freq=3e-4, seed=s, origin=(x, y, 0), extent=(nx, ny, 1))
            for m, o, s, x, y, nx, ny in [(1, 9, 5, -1000, 2 ** 40, 200, 130), (2, 12, 6, 77, -3, 64, 17),
                                          (1, 4, 7, 2 ** 45, 5, 130, 300), (2, 6, 8, 0, 0, 16, 16)]]
    tickets = srv.submit([ptg.tile_req(dim=2, **r) for r in reqs])
    for t, r in zip(tickets, reqs):
        res = srv.wait(t, int(60e9))
        assert res.status == ptg.PTG_OK and res.kernel == ptg.PTG_TUNE_GENERAL_2D
        nx, ny, _ = r["extent"]
        got = torch.empty((ny, nx), dtype=torch.float32, device=DEV)
        ptg.device_copy(got.data_ptr(), res.out_dev, res.bytes)
        srv.release(t)
        solo = _field2((ny, nx), r["origin"][0], r["origin"][1], smoothness=r["smoothness"], octaves=r["octaves"],
                       base_freq=r["base_freq"], seed=r["seed"], path="general")
        assert torch.equal(got, solo), r


def test_server_with_fixed_and_tuned_tile_heights_serves_exact_tiles():
    with ptg.Server(1 << 28, tile_h=16) as srv:
        assert srv.stats()["tile_h"] == [16, 16]
        _served_equals_solo(srv)
    with ptg.Server(1 << 28, autotune=1) as srv:
        th = srv.stats()["tile_h"]
        assert all(v in (16, 32, 64) for v in th)
        _served_equals_solo(srv)


def test_tuned_table_saved_and_loaded_on_this_device(tmp_path):
    """A table tuned here is written with this device's architecture name and CU count and
    loads back in full."""
    out = torch.empty((256, 300), dtype=torch.float32, device="cuda")
    r = ptg.tune_2d(out, octaves=4, base_freq=0.013)
    path = tmp_path / "t.txt"
    ptg.tune_save(path)
    head = path.read_text().splitlines()[0].split()
    assert head[2].startswith("gfx") and int(head[3]) > 0
    ptg.tune_reset()
    assert ptg.tune_load(path) >= 1
    assert ptg.tune_query((256, 300), octaves=4, base_freq=0.013)[1] == r["value"]
