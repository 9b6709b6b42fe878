"""The C-ABI library loads, exports every function include/ptg.h declares, and
rejects bad arguments on the host before any launch (CPU only: no compute call)."""
import ctypes

import pytest

import paper_1610_03525_amd as ptg


def test_library_exports_every_declared_symbol():
    L = ptg.lib()
    names = ptg.declared_symbols()
    assert "ptg_fbm_2d" in names and "ptg_fbm_3d" in names and "ptg_lattice_2d" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/ptg.h but not exported"
    assert ptg.version().startswith("ptg")


def test_params_layout_matches_header():
    # the binding's struct mirrors ptg_params: 4 int32, 3 double, uint32 + 4 int32, double
    assert ptg.Params.model.offset == 4 * 4 + 3 * 8 + 4 * 4
    assert ptg.Params.gradient_weight.offset == 64 and ctypes.sizeof(ptg.Params) == 72
    p = ptg.Params()
    ptg.lib().ptg_params_default(ctypes.byref(p))
    assert (p.dim, p.smoothness, p.octaves, p.persistence, p.lacunarity, p.seed) == (2, 1, 8, 0.5, 2.0, 1)
    assert p.model == ptg.PTG_MODEL_GRADIENT and p.gradient_weight == 0.01


def test_model_validation():
    """The zero-gradient model (Sec. 3.3) is 2D C1 plain form only, the height-and-gradient
    model plain form (2D or 3D) with a finite weight; neither is served."""
    L = ptg.lib()
    ok = ptg.params(model="zero_gradient", base_freq=1 / 64, octaves=3)
    assert ptg.lib().ptg_tune_query_2d(ctypes.byref(ok), 64, 64, ctypes.byref(ctypes.c_int32()),
                                       ctypes.byref(ctypes.c_int32())) == ptg.PTG_OK
    for kw in (dict(model=5), dict(model=-1), dict(model="zero_gradient", smoothness=2),
               dict(model="perlin", smoothness=3), dict(model="perlin", path="dyadic"), dict(model="simplex", smoothness=2),
               dict(model="zero_gradient", form="mfma_f16"), dict(model="height_gradient", form="mfma_bf16"),
               dict(model="height_gradient", gradient_weight=float("inf")),
               dict(model="height_gradient", gradient_weight=float("nan"))):
        p = ptg.params(base_freq=1 / 64, octaves=3, **kw)
        assert L.ptg_fbm_2d(ctypes.byref(p), 0, 0, 16, 16, ctypes.c_void_p(1 << 20), 16, None) == ptg.PTG_EINVAL
    # septic cells: the 2D strip and general kernels (no matrix-core form, not served);
    # orders 4..6 the general kernels only; 7 is rejected
    for kw in (dict(smoothness=3, form="mfma_f16"), dict(smoothness=4, path="dyadic"), dict(smoothness=7),
               dict(smoothness=0)):
        p = ptg.params(base_freq=1 / 64, octaves=3, **kw)
        assert L.ptg_fbm_2d(ctypes.byref(p), 0, 0, 16, 16, ctypes.c_void_p(1 << 20), 16, None) == ptg.PTG_EINVAL
    p = ptg.params(base_freq=1 / 64, octaves=3, smoothness=4)
    assert L.ptg_fbm_2d_grad(ctypes.byref(p), 0, 0, 16, 16, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 21),
                             ctypes.c_void_p(1 << 22), 16, None) == ptg.PTG_EINVAL
    assert ptg.tune_query((64, 64), smoothness=3, octaves=3, base_freq=1 / 64)[0] == "strip_2d"
    assert ptg.tune_query((64, 64), smoothness=5, octaves=3, base_freq=1 / 64) == ("general_2d", 64)
    assert ptg.tune_query((64, 64, 64), smoothness=3, octaves=3, base_freq=1 / 16) == ("general_3d", 0)
    p3 = ptg.params(dim=3, base_freq=1 / 64, octaves=3, smoothness=3, path="dyadic")
    assert L.ptg_fbm_3d(ctypes.byref(p3), 0, 0, 0, 8, 8, 8, ctypes.c_void_p(1 << 20), None) == ptg.PTG_EINVAL
    p3 = ptg.params(dim=3, model="zero_gradient", base_freq=1 / 64, octaves=3)
    assert L.ptg_fbm_3d(ctypes.byref(p3), 0, 0, 0, 8, 8, 8, ctypes.c_void_p(1 << 20), None) == ptg.PTG_EINVAL
    p3 = ptg.params(dim=3, model="height_gradient", base_freq=1 / 64, octaves=3, form="mfma_f16")
    assert L.ptg_fbm_3d(ctypes.byref(p3), 0, 0, 0, 8, 8, 8, ctypes.c_void_p(1 << 20), None) == ptg.PTG_EINVAL
    for sm in (1, 2, 3):  # 3D heights and gradients: the 3D strip kernel (C1, C2) or the general one
        want = ("strip_3d" if sm < 3 else "general_3d")
        assert ptg.tune_query((64, 64, 64), model="height_gradient", smoothness=sm, base_freq=1 / 64,
                              octaves=5)[0] == want
    ok2 = ptg.params(model="height_gradient", smoothness=2, base_freq=1 / 64, octaves=3, gradient_weight=-0.3)
    assert ptg.lib().ptg_tune_query_2d(ctypes.byref(ok2), 64, 64, ctypes.byref(ctypes.c_int32()),
                                       ctypes.byref(ctypes.c_int32())) == ptg.PTG_OK
    assert L.ptg_heights_2d(1, -1, 0, 0, 4, 4, ctypes.c_void_p(1), None) == ptg.PTG_EINVAL
    assert L.ptg_heights_2d(1, 0, 0, 0, 4, 4, None, None) == ptg.PTG_EINVAL
    assert L.ptg_heights_2d(1, 0, 0, 0, 0, 4, None, None) == ptg.PTG_OK  # empty box
    # the server takes the three polynomial cell models at C1..C3 (zero-gradient: 2D C1);
    # the comparison paths, orders above 3, other forms and FP16 output are rejected
    with ptg.Server(1 << 20, executor=ptg.PTG_EXEC_HOST) as s:
        ok = [ptg.tile_req(dim=2, extent=(64, 64, 1), octaves=3, base_freq=1 / 64, model="zero_gradient"),
              ptg.tile_req(dim=2, extent=(64, 64, 1), octaves=3, base_freq=1 / 64, model="height_gradient",
                           smoothness=2),
              ptg.tile_req(dim=3, extent=(16, 16, 16), octaves=3, base_freq=1 / 16, model="height_gradient"),
              ptg.tile_req(dim=2, extent=(64, 64, 1), octaves=3, base_freq=1 / 64, smoothness=3)]
        for t in s.submit(ok):
            s.wait(t, int(5e9))
            s.release(t)
        for kw in (dict(model="perlin"), dict(model="simplex"), dict(smoothness=4), dict(form="mfma_f16", out_dtype=1),
                   dict(out_dtype=1)):
            with pytest.raises(ptg.PtgError) as e:
                s.submit([ptg.tile_req(dim=2, extent=(64, 64, 1), octaves=3, base_freq=1 / 64, **kw)])
            assert e.value.code == ptg.PTG_EINVAL, kw
        with pytest.raises(ptg.PtgError) as e:
            s.submit([ptg.tile_req(dim=3, extent=(16, 16, 16), octaves=3, base_freq=1 / 16, model="zero_gradient")])
        assert e.value.code == ptg.PTG_EINVAL


def _fbm2(p, x0=0, y0=0, nx=16, ny=16, out=1 << 20, pitch=16):
    return ptg.lib().ptg_fbm_2d(ctypes.byref(p), x0, y0, nx, ny, ctypes.c_void_p(out), pitch, None)


@pytest.mark.parametrize("field,value", [
    ("dim", 3), ("smoothness", 0), ("smoothness", 7), ("octaves", 0), ("octaves", 17), ("out_dtype", 5),
    ("persistence", 0.0), ("persistence", float("nan")), ("lacunarity", -2.0), ("base_freq", 0.0),
    ("base_freq", float("inf")), ("form", 9), ("basis", 7), ("path", 3), ("path", -1),
])
def test_rejects_bad_params(field, value):
    p = ptg.params()
    setattr(p, field, value)
    assert _fbm2(p) == ptg.PTG_EINVAL
    assert ptg.last_error() != ""


def test_rejects_lattice_finer_than_samples():
    p = ptg.params(base_freq=1 / 4, octaves=4)  # octave 3: 2 cells per sample
    assert _fbm2(p) == ptg.PTG_EINVAL
    assert "frequency" in ptg.last_error()
    p = ptg.params(base_freq=1 / 8, octaves=4)  # finest 1 cell per sample: allowed
    # (not launched here: a NULL output with an empty field is a no-op)
    assert _fbm2(p, nx=0, out=0) == ptg.PTG_OK


def test_rejects_bad_extents():
    p = ptg.params()
    assert _fbm2(p, nx=-1) == ptg.PTG_EINVAL
    assert _fbm2(p, x0=1 << 52) == ptg.PTG_EINVAL
    assert _fbm2(p, x0=(1 << 52) - 10, nx=16) == ptg.PTG_EINVAL
    assert _fbm2(p, y0=-(1 << 52)) == ptg.PTG_EINVAL
    assert _fbm2(p, pitch=8) == ptg.PTG_EINVAL
    assert _fbm2(p, out=0) == ptg.PTG_EINVAL
    # empty fields are accepted without touching the device
    assert _fbm2(p, nx=0, out=0) == ptg.PTG_OK
    assert _fbm2(p, ny=0, out=0) == ptg.PTG_OK


def test_rejects_mfma_outside_2d_c1():
    p = ptg.params(smoothness=2, form="mfma_f16")
    assert _fbm2(p) == ptg.PTG_EINVAL
    p = ptg.params(dim=3, form="mfma_f16")
    assert ptg.lib().ptg_fbm_3d(ctypes.byref(p), 0, 0, 0, 8, 8, 8, ctypes.c_void_p(1 << 20), None) == ptg.PTG_EINVAL


def test_3d_and_stage_validation():
    L = ptg.lib()
    p = ptg.params(dim=3, base_freq=1 / 8, octaves=3)
    assert L.ptg_fbm_3d(ctypes.byref(p), 0, 0, 0, 8, 8, -1, ctypes.c_void_p(1 << 20), None) == ptg.PTG_EINVAL
    assert L.ptg_fbm_3d(ctypes.byref(p), 0, 0, 0, 8, 8, 0, None, None) == ptg.PTG_OK
    p2 = ptg.params(dim=2)
    assert L.ptg_fbm_3d(ctypes.byref(p2), 0, 0, 0, 8, 8, 8, ctypes.c_void_p(1 << 20), None) == ptg.PTG_EINVAL
    assert L.ptg_coords(0.0, 2.0, 4, 0, 16, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == ptg.PTG_EINVAL
    assert L.ptg_coords(0.5, 2.0, 0, 0, 16, ctypes.c_void_p(1), ctypes.c_void_p(1), None) == ptg.PTG_EINVAL
    assert L.ptg_lattice_2d(1, -1, 0, 0, 4, 4, ctypes.c_void_p(1), None, None) == ptg.PTG_EINVAL
    assert L.ptg_lattice_2d(1, 0, 0, 0, 4, 4, None, None, None) == ptg.PTG_EINVAL
    assert L.ptg_lattice_3d(1, 0, 0, 0, 0, 4, -4, 4, ctypes.c_void_p(1), None, None, None) == ptg.PTG_EINVAL
    assert L.ptg_cells_2d(1, ctypes.c_void_p(1), 1, 4, 1.0, ctypes.c_void_p(1), None) == ptg.PTG_EINVAL
    assert L.ptg_cells_2d(3, ctypes.c_void_p(1), 4, 4, 1.0, ctypes.c_void_p(1), None) == ptg.PTG_EINVAL
    assert L.ptg_cells_3d(1, None, 4, 4, 4, 1.0, ctypes.c_void_p(1), None) == ptg.PTG_EINVAL


def test_declared_symbols_parser():
    names = ptg.declared_symbols()
    assert "ptg_last_error" in names and "ptg_params_default" in names
    assert all(n.startswith("ptg_") for n in names)
