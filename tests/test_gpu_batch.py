"""HIP-graph batches (ptg_batch): a batch of dense-field calls launched as one graph equals
the direct calls bit for bit, on its first launch (instantiation) and on every later launch
of the same shape with new origins, seeds and outputs (arguments updated in place), with
eager work and synchronisations between the replays."""
import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"

# the kernels a batch can hold: 2D strip (dyadic), 2D general, 2D FP16 output, the FP16
# matrix-core form, 3D strip, 3D general, zero-gradient model
CALLS = [
    (2, (192, 130), dict(smoothness=1, octaves=8, base_freq=1 / 256)),
    (2, (100, 77), dict(smoothness=2, octaves=5, base_freq=0.013, lacunarity=1.9)),
    (2, (128, 64), dict(smoothness=2, octaves=6, base_freq=1 / 64, out="f16")),
    (2, (256, 96), dict(smoothness=1, octaves=9, base_freq=1 / 512, form="mfma_f16", basis="centred", out="f16")),
    (3, (64, 24, 16), dict(smoothness=2, octaves=5, base_freq=1 / 64)),
    (3, (40, 9, 7), dict(smoothness=1, octaves=4, base_freq=0.021, lacunarity=2.3)),
    (2, (96, 80), dict(smoothness=1, octaves=6, base_freq=1 / 32, model="zero_gradient")),
]


def _alloc(dim, shape, kw):
    dt = torch.float16 if kw.get("out") == "f16" else torch.float32
    return torch.empty(tuple(reversed(shape)), dtype=dt, device=DEV)


def _kw(kw, seed):
    k = {a: b for a, b in kw.items() if a != "out"}
    k["seed"] = seed
    return k


def _origins(rng, dim):
    return [int(v) for v in rng.integers(-(1 << 40), 1 << 40, size=dim)]


def _direct(dim, out, org, kw):
    ref = torch.empty_like(out)
    if dim == 2:
        ptg.fbm_2d(ref, x0=org[0], y0=org[1], **kw)
    else:
        ptg.fbm_3d(ref, x0=org[0], y0=org[1], z0=org[2], **kw)
    return ref


def _fill(b, rng, outs):
    plan = []
    for (dim, shape, kw), out in zip(CALLS, outs):
        org = _origins(rng, dim)
        k = _kw(kw, int(rng.integers(0, 1 << 32)))
        if dim == 2:
            b.add_2d(out, x0=org[0], y0=org[1], **k)
        else:
            b.add_3d(out, x0=org[0], y0=org[1], z0=org[2], **k)
        plan.append((dim, out, org, k))
    return plan


def _check(plan):
    torch.cuda.synchronize()
    for dim, out, org, k in plan:
        assert torch.equal(out, _direct(dim, out, org, k)), (dim, tuple(out.shape), k)


def test_batch_equals_direct_calls_and_reuses_its_graph():
    rng = np.random.default_rng(5)
    with ptg.Batch(16) as b:
        outs = [_alloc(*c) for c in CALLS]
        plan = _fill(b, rng, outs)
        assert b.stats()["pending"] == len(CALLS)
        b.launch()
        _check(plan)
        st = b.stats()
        assert st["instantiations"] == 1 and st["launches"] == 1 and st["nodes"] == len(CALLS)
        for rep in range(3):  # same shape: new origins, seeds and output buffers
            outs = [_alloc(*c) for c in CALLS]
            plan = _fill(b, rng, outs)
            b.launch()
            torch.ones(1000, device=DEV).sum().item()  # eager work and a sync between replays
            _check(plan)
        st = b.stats()
        assert st["instantiations"] == 1 and st["updates"] == 3 and st["launches"] == 4


def test_batch_launches_in_flight_use_separate_instances():
    """Six launches of one shape queued back to back (no synchronisation between them): at
    most four instances exist, no instance is updated while a launch of it may run, and every
    launch's outputs equal the direct calls."""
    rng = np.random.default_rng(6)
    plans = []
    with ptg.Batch(16) as b:
        for _ in range(6):
            outs = [_alloc(*c) for c in CALLS]
            plans.append(_fill(b, rng, outs))
            b.launch()
        st = b.stats()
        assert 1 <= st["instantiations"] <= 4 and st["instances"] <= 4
        assert st["instantiations"] + st["updates"] == 6
        for plan in plans:
            _check(plan)


def test_batch_shapes_and_samples_against_oracle():
    rng = np.random.default_rng(7)
    with ptg.Batch(4) as b:
        out1 = torch.empty((70, 90), dtype=torch.float32, device=DEV)
        b.add_2d(out1, x0=-(1 << 33) - 5, y0=1 << 20, smoothness=1, octaves=6, base_freq=1 / 64, seed=3)
        b.launch()
        out2 = torch.empty((40, 50), dtype=torch.float32, device=DEV)
        b.add_2d(out2, x0=17, y0=-9, smoothness=1, octaves=6, base_freq=1 / 64, seed=4)
        b.launch()  # the same kernel over another grid: the instance is updated in place
        st = b.stats()
        assert st["instantiations"] == 1 and st["updates"] == 1
        torch.cuda.synchronize()
        ref = O.fbm_2d(1, 6, 0.5, 2.0, 1 / 64, 3, -(1 << 33) - 5, 1 << 20, 90, 70)
        assert np.max(np.abs(out1.cpu().numpy() - ref)) <= 1e-5 * sum(0.5 ** o for o in range(6))
        ref = O.fbm_2d(1, 6, 0.5, 2.0, 1 / 64, 4, 17, -9, 50, 40)
        assert np.max(np.abs(out2.cpu().numpy() - ref)) <= 1e-5 * sum(0.5 ** o for o in range(6))


def test_batch_rejects_and_empty_launch():
    with ptg.Batch(2) as b:
        out = torch.empty((8, 8), dtype=torch.float32, device=DEV)
        with pytest.raises(ptg.PtgError):
            b.add_2d(out, base_freq=2.0, octaves=2)  # frequency above one cell per sample
        b.launch()  # nothing recorded: no-op
        b.add_2d(out, base_freq=1 / 8, octaves=2)
        b.add_2d(out, base_freq=1 / 8, octaves=2, seed=2)
        with pytest.raises(ptg.PtgError):
            b.add_2d(out, base_freq=1 / 8, octaves=2)  # full
        b.clear()
        assert b.stats()["pending"] == 0 and b.stats()["launches"] == 0
