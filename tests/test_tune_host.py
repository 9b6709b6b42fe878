"""Tile-shape autotuner, host side: which kernel class a call runs, the recorded shapes,
and the validation of shapes and server settings (no GPU: queries never launch)."""
import ctypes

import pytest

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402


@pytest.fixture(autouse=True)
def _clean_table():
    ptg.tune_reset()
    yield
    ptg.tune_reset()


@pytest.mark.parametrize("shape,kw,expect", [
    ((8192, 8192), dict(octaves=8, base_freq=16 / 8192), ("strip_2d", 4)),            # dyadic ladder to period 4
    ((256, 300), dict(octaves=4, base_freq=0.013), ("general_2d", 64)),               # any base frequency
    ((256, 256), dict(octaves=4, base_freq=1 / 32, path="general"), ("general_2d", 64)),
    ((512, 512, 512), dict(smoothness=2, octaves=6, base_freq=8 / 512), ("strip_3d", 4)),
    ((100, 100, 40), dict(smoothness=2, octaves=6, base_freq=0.02), ("general_3d", 0)),
    ((40, 6, 5), dict(octaves=2, base_freq=0.5), ("general_3d", 0)),                   # ladder from period 2
    ((2048, 2048), dict(octaves=4, base_freq=1 / 64, form=1, out_dtype=1), ("strip_2d", 4)),  # FP16 matrix-core form
    ((2048, 2048), dict(octaves=4, base_freq=1 / 64, form=2, out_dtype=1, basis=2), ("strip_2d", 4)),
])
def test_query_reports_the_kernel_class(shape, kw, expect):
    assert ptg.tune_query(shape, **kw) == expect


def test_set_query_reset_roundtrip():
    kw = dict(octaves=4, base_freq=0.013)
    for v in (16, 32, 64, 128):
        ptg.tune_set((256, 300), v, **kw)
        assert ptg.tune_query((256, 300), **kw) == ("general_2d", v)
    # another class (size class of 2^20 samples) is untouched
    assert ptg.tune_query((1024, 1024), **kw) == ("general_2d", 128)  # untuned: 128 rows for tall fields
    # C2 is a class of its own
    assert ptg.tune_query((256, 300), smoothness=2, **kw) == ("general_2d", 64)
    ptg.tune_set((8192, 8192), 2, octaves=8, base_freq=16 / 8192)
    assert ptg.tune_query((8192, 8192), octaves=8, base_freq=16 / 8192) == ("strip_2d", 2)
    ptg.tune_reset()
    assert ptg.tune_query((256, 300), **kw) == ("general_2d", 64)
    assert ptg.tune_query((8192, 8192), octaves=8, base_freq=16 / 8192) == ("strip_2d", 4)


@pytest.mark.parametrize("shape,kw,value", [
    ((256, 300), dict(octaves=4, base_freq=0.013), 8),            # not a tile height
    ((256, 300), dict(octaves=4, base_freq=0.013), 4),            # a waves count, not a tile height
    ((8192, 8192), dict(octaves=8, base_freq=16 / 8192), 3),      # not a waves count
    ((100, 100, 40), dict(smoothness=2, octaves=6, base_freq=0.02), 64),  # general 3D: nothing to tune
    ((2048, 2048), dict(octaves=4, base_freq=1 / 64, form=1, out_dtype=1), 3),
])
def test_set_rejects_shapes_that_are_not_candidates(shape, kw, value):
    with pytest.raises(ptg.PtgError):
        ptg.tune_set(shape, value, **kw)


def test_query_validates_parameters():
    with pytest.raises(ptg.PtgError):
        ptg.tune_query((0, 16), octaves=4)
    with pytest.raises(ptg.PtgError):
        ptg.tune_query((16, 16), octaves=0)
    with pytest.raises(ptg.PtgError):
        ptg.tune_query((16, 16), base_freq=-1.0)


def test_server_cfg_tile_settings_validation():
    L = ptg.lib()
    h = ctypes.c_void_p()
    bad = [dict(tile_h=8), dict(tile_h=128), dict(autotune=2)]
    for kw in bad:
        cfg = ptg.ServerCfg(1 << 20, 1024, 0, 0, ptg.PTG_EXEC_HOST, 0, 0, kw.get("autotune", 0), kw.get("tile_h", 0))
        assert L.ptg_server_create(ctypes.byref(cfg), ctypes.byref(h)) == ptg.PTG_EINVAL
    with ptg.Server(1 << 20, executor=ptg.PTG_EXEC_HOST, tile_h=32) as s:
        assert s.stats()["tile_h"] == [32, 32]
    with ptg.Server(1 << 20, executor=ptg.PTG_EXEC_HOST) as s:
        assert s.stats()["tile_h"] == [64, 64]


def test_server_tile_height_sets_the_tile_count():
    """A non-dyadic 2D request of 128 x 100 samples is 2 x 2 general tiles of 64 x 64, or
    2 x 7 of 64 x 16; a dyadic one is world-aligned 64 x 64 strips (3 x 3 at this origin)
    whatever the tile height, computed by the strip code."""
    for th, tiles in ((64, 4), (32, 8), (16, 14)):
        with ptg.Server(1 << 22, executor=ptg.PTG_EXEC_HOST, fake_tile_ns=1000, tile_h=th) as s:
            (t,) = s.submit([ptg.tile_req(dim=2, extent=(128, 100, 1), octaves=4, base_freq=3e-4)])
            res = s.wait(t, 10_000_000_000)
            assert s.stats()["tiles_done"] == tiles and res.kernel == ptg.PTG_TUNE_GENERAL_2D
            (t,) = s.submit([ptg.tile_req(dim=2, origin=(-7, 30, 0), extent=(128, 100, 1), octaves=4,
                                          base_freq=2.0 ** -12)])
            res = s.wait(t, 10_000_000_000)
            assert s.stats()["tiles_done"] == tiles + 9 and res.kernel == ptg.PTG_TUNE_STRIP_2D
            (t,) = s.submit([ptg.tile_req(dim=3, extent=(64, 8, 8), octaves=4, base_freq=2.0 ** -12)])
            assert s.wait(t, 10_000_000_000).kernel == ptg.PTG_TUNE_STRIP_3D  # periods 4096..512
            (t,) = s.submit([ptg.tile_req(dim=3, extent=(64, 8, 8), octaves=4, base_freq=1 / 16)])
            assert s.wait(t, 10_000_000_000).kernel == ptg.PTG_TUNE_STRIP_3D  # periods 16..2
            (t,) = s.submit([ptg.tile_req(dim=3, extent=(64, 8, 8), octaves=4, base_freq=3e-4)])
            assert s.wait(t, 10_000_000_000).kernel == ptg.PTG_TUNE_GENERAL_3D  # not dyadic


def test_save_load_roundtrip_keyed_by_device(tmp_path):
    """A saved table loads back on the same device (on a host without a GPU the key is
    "none"); a table written for another device is skipped; malformed tables and missing
    files are errors, and nothing of a bad table is taken."""
    kw2 = dict(octaves=4, base_freq=0.013)
    kw3 = dict(smoothness=2, octaves=6, base_freq=8 / 512)
    ptg.tune_set((256, 300), 32, **kw2)
    ptg.tune_set((512, 512, 512), 2, **kw3)
    path = tmp_path / "table.txt"
    ptg.tune_save(path)
    head = path.read_text().splitlines()[0].split()
    assert head[:2] == ["ptg_tune", "1"] and len(head) == 4
    ptg.tune_reset()
    assert ptg.tune_query((256, 300), **kw2) == ("general_2d", 64)
    assert ptg.tune_load(path) == 2
    assert ptg.tune_query((256, 300), **kw2) == ("general_2d", 32)
    assert ptg.tune_query((512, 512, 512), **kw3) == ("strip_3d", 2)

    ptg.tune_reset()
    lines = path.read_text().splitlines()
    other = tmp_path / "other.txt"
    other.write_text("\n".join(["ptg_tune 1 gfx000 7"] + lines[1:]) + "\n")
    assert ptg.tune_load(other) == 0
    assert ptg.tune_query((256, 300), **kw2) == ("general_2d", 64)

    bad = tmp_path / "bad.txt"
    bad.write_text("\n".join(lines[:1] + ["1 1 0 17 3 48"]) + "\n")  # 48 rows is no candidate
    with pytest.raises(ptg.PtgError) as e:
        ptg.tune_load(bad)
    assert e.value.code == ptg.PTG_EINVAL
    junk = tmp_path / "junk.txt"
    junk.write_text("not a table\n")
    with pytest.raises(ptg.PtgError) as e:
        ptg.tune_load(junk)
    assert e.value.code == ptg.PTG_EINVAL
    with pytest.raises(ptg.PtgError) as e:
        ptg.tune_load(tmp_path / "missing.txt")
    assert e.value.code == ptg.PTG_ENOENT
    assert ptg.tune_query((256, 300), **kw2) == ("general_2d", 64)
