"""GPU parity over whole benchmark fields, element by element against the FP64 oracle.

* 2D 8192 x 8192, 8 octaves, base lattice 16 x 16, C1, FP32 (the throughput workload):
  every sample within 1e-5 * A (A = sum_o p^o), compared in row bands.
* 3D 512^3, 6 octaves, base lattice 8^3, C2 quintic, FP32: every sample within 1e-5 * A,
  compared in z-slabs.
* 2D 16384 x 16384, 10 octaves, base lattice 32 x 32, world offset (2^24 - 3) * 512,
  -(2^24 - 5) * 512 samples (2^24 cells at period 512): the plain FP32 form within
  1e-5 * A everywhere, and the FP16 / BF16 matrix-core forms (monomial and centred bases,
  FP16 output) with their max and RMS error over all 268 M samples stated and held to
  bounds of twice the values measured on MI355X.

The oracle runs on every host core (OpenMP); each test prints its progress per band.  When
the environment variable PTG_RECORD names a directory, the measured errors are written
there as JSON."""
import json
import os
import time

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
import paper_1610_03525_amd as ptg  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _A(p, n):
    return sum(p ** o for o in range(n))


def _record(name, data):
    d = os.environ.get("PTG_RECORD")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name), "w") as fh:
            json.dump(data, fh, indent=1)


def test_fbm2d_8192_8oct_every_sample():
    n, f0 = 8192, 16 / 8192
    kw = dict(smoothness=1, octaves=8, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=1)
    out = torch.empty((n, n), dtype=torch.float32, device=DEV)
    ptg.fbm_2d(out, x0=0, y0=0, **kw)
    torch.cuda.synchronize()
    tol = 1e-5 * _A(0.5, 8)
    worst, t0 = 0.0, time.time()
    band = 1024
    for y0 in range(0, n, band):
        g = out[y0:y0 + band].cpu().numpy().astype(np.float64)
        ref = O.fbm_2d(1, 8, 0.5, 2.0, f0, 1, 0, y0, n, band)
        worst = max(worst, float(np.max(np.abs(g - ref))))
        print(f"[8192^2] rows {y0}..{y0 + band - 1}: max|err| so far {worst:.3e} ({time.time() - t0:.1f} s)",
              flush=True)
    _record("fullfield_2d_8192.json", {"max_abs_err": worst, "A": _A(0.5, 8), "max_over_A": worst / _A(0.5, 8)})
    assert worst <= tol, worst


def test_fbm3d_512_6oct_c2_every_sample():
    n, f0 = 512, 8 / 512
    kw = dict(smoothness=2, octaves=6, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=1)
    out = torch.empty((n, n, n), dtype=torch.float32, device=DEV)
    ptg.fbm_3d(out, x0=0, y0=0, z0=0, **kw)
    torch.cuda.synchronize()
    tol = 1e-5 * _A(0.5, 6)
    worst, t0 = 0.0, time.time()
    slab = 32
    for z0 in range(0, n, slab):
        g = out[z0:z0 + slab].cpu().numpy().astype(np.float64)
        ref = O.fbm_3d(2, 6, 0.5, 2.0, f0, 1, 0, 0, z0, n, n, slab)
        worst = max(worst, float(np.max(np.abs(g - ref))))
        print(f"[512^3 C2] slices {z0}..{z0 + slab - 1}: max|err| so far {worst:.3e} ({time.time() - t0:.1f} s)",
              flush=True)
    _record("fullfield_3d_512_c2.json", {"max_abs_err": worst, "A": _A(0.5, 6), "max_over_A": worst / _A(0.5, 6)})
    assert worst <= tol, worst


# Precision form on the 16384^2 field: bounds on max|err| / A and RMS / A, twice the values
# measured over the whole field on MI355X (profiles/precision_form_errors.md).
PREC_BOUNDS = {
    ("mfma_f16", "monomial"): (2.1e-4, 3.0e-5),   # measured 1.03e-4, 1.48e-5
    ("mfma_f16", "centred"): (1.4e-4, 2.9e-5),    # measured 6.98e-5, 1.44e-5
    ("mfma_f16", "hermite"): (1.4e-4, 2.9e-5),    # measured 7.02e-5, 1.44e-5
    ("mfma_bf16", "monomial"): (1.2e-3, 7.8e-5),  # measured 5.89e-4, 3.88e-5
    ("mfma_bf16", "centred"): (2.7e-4, 3.2e-5),   # measured 1.35e-4, 1.58e-5
    ("mfma_bf16", "hermite"): (2.6e-4, 3.2e-5),   # measured 1.27e-4, 1.59e-5
}
X4, Y4 = (2 ** 24 - 3) * 512, -(2 ** 24 - 5) * 512


def test_fbm2d_16384_10oct_precision_forms_every_sample():
    n, f0, octs = 16384, 32 / 16384, 10
    A = _A(0.5, octs)
    base = dict(smoothness=1, octaves=octs, persistence=0.5, lacunarity=2.0, base_freq=f0, seed=1)
    plain = torch.empty((n, n), dtype=torch.float32, device=DEV)
    ptg.fbm_2d(plain, x0=X4, y0=Y4, **base)
    # the plain FP32 arithmetic with FP16 output: the output rounding floor of every FP16 form
    forms = {("plain", "fp16_out"): torch.empty((n, n), dtype=torch.float16, device=DEV)}
    ptg.fbm_2d(forms[("plain", "fp16_out")], x0=X4, y0=Y4, **base)
    for key in PREC_BOUNDS:
        t = torch.empty((n, n), dtype=torch.float16, device=DEV)
        ptg.fbm_2d(t, x0=X4, y0=Y4, form=key[0], basis=key[1], **base)
        forms[key] = t
    torch.cuda.synchronize()
    acc = {k: [0.0, 0.0] for k in forms}  # max |err|, sum err^2
    worst_plain, t0 = 0.0, time.time()
    band = 512
    for y0 in range(0, n, band):
        ref = O.fbm_2d(1, octs, 0.5, 2.0, f0, 1, X4, Y4 + y0, n, band)
        g = plain[y0:y0 + band].cpu().numpy().astype(np.float64)
        worst_plain = max(worst_plain, float(np.max(np.abs(g - ref))))
        for k, t in forms.items():
            e = np.abs(t[y0:y0 + band].cpu().numpy().astype(np.float64) - ref)
            acc[k][0] = max(acc[k][0], float(e.max()))
            acc[k][1] += float(np.sum(e * e))
        if (y0 // band) % 8 == 7:
            print(f"[16384^2] rows ..{y0 + band - 1}: plain {worst_plain:.3e}, "
                  + ", ".join(f"{a}/{b} {v[0] / A:.2e}" for (a, b), v in acc.items())
                  + f" ({time.time() - t0:.1f} s)", flush=True)
    res = {"plain_fp32": {"max_abs_err": worst_plain, "max_over_A": worst_plain / A}, "A": A, "samples": n * n}
    for (form, basis), (mx, s2) in acc.items():
        rms = float(np.sqrt(s2 / (n * n)))
        res[f"{form}/{basis}"] = {"max_over_A": mx / A, "rms_over_A": rms / A}
        print(f"[16384^2] {form}/{basis}: max/A {mx / A:.3e}  rms/A {rms / A:.3e}", flush=True)
    _record("fullfield_2d_16384_precision.json", res)
    assert worst_plain <= 1e-5 * A, worst_plain
    # FP16 output: round to nearest even, relative error <= 2^-11 of |H| <= A / 2
    assert res["plain/fp16_out"]["max_over_A"] <= 2.0 ** -11 / 2 + 1e-5, res["plain/fp16_out"]
    for key, (bmax, brms) in PREC_BOUNDS.items():
        assert res[f"{key[0]}/{key[1]}"]["max_over_A"] <= bmax, (key, res[f"{key[0]}/{key[1]}"])
        assert res[f"{key[0]}/{key[1]}"]["rms_over_A"] <= brms, (key, res[f"{key[0]}/{key[1]}"])
