"""Benchmark: octave-samples/s of the dense fBm path on one MI355X.

Workload (the throughput configuration): 2D fBm heightmap 8192 x 8192, 8 octaves, base
lattice 16 x 16 cells (base frequency 16/8192), lacunarity 2, persistence 0.5, C1 cubic
cells, unit gradients from the stated lattice hash, FP32 output, seed 1, origin (0, 0).
A step is one ptg_fbm_2d call: coordinate step, lattice hash, per-cell coefficients,
evaluation and octave accumulation for the whole field.  Inputs are parameters only;
the output buffer is allocated before the timed region.

Prints ONE JSON line (rank 0).  Extra fields: the measured pure-store write roofline,
per-kernel event timing, the FP64 CPU oracle timed on the host cores, and "serving": the
terrain-tile stream (Poisson arrivals of uneven 2D/3D requests) through the tile server
against the plain per-tile path, direct and hipGraph-batched: capacity in tiles/s and
p50/p99 latency at 0.5, 0.8 and 0.95 of the plain path's capacity.
"""
import argparse
import ctypes
import faulthandler
import json
import os
import sys
import time

faulthandler.enable()  # a crash in native code prints the Python stack of the phase it hit

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX = NY = 8192
OCTAVES = 8
BASE_FREQ = 16 / 8192
PERSISTENCE = 0.5
LACUNARITY = 2.0
SEED = 1
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fbm2d_strip_2d_8192x8192_8oct_c1.traffic.json")


def progress(msg):
    """One line per finished phase on stderr (the JSON record alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
    or None when the kernel's sources (the files listed, hashed in order) have changed
    since they were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        h = hashlib.sha256()
        for src in t["sources"]:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != t["sources_sha256"]:
            return None
        return t["traffic_bytes"]
    except (OSError, KeyError, ValueError, TypeError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall-time budget of the oracle sample")
    ap.add_argument("--path", default="auto", choices=["auto", "general", "dyadic"])
    ap.add_argument("--serve-requests", type=int, default=5000, help="tile-stream length (0: skip serving)")
    ap.add_argument("--no-other-configs", action="store_true", help="skip the 3D, precision-form and small fields")
    ap.add_argument("--profile-calibration", action="store_true",
                    help="also run a plain torch fill and copy of the field size (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(each GPU would compute its own row band independently).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1610_03525_amd as ptg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    out = torch.empty((NY, NX), dtype=torch.float32, device=dev)
    p = ptg.params(dim=2, smoothness=1, octaves=OCTAVES, persistence=PERSISTENCE, lacunarity=LACUNARITY,
                   base_freq=BASE_FREQ, seed=SEED, path=args.path)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    ptr = out.data_ptr()

    def step():
        ptg.fbm_2d_raw(p, 0, 0, NX, NY, ptr, NX, sh)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: exactly `steps` steps, bracketed by device synchronisation; one pair of
    # HIP events on the launch stream brackets the same back-to-back launches (the GPU
    # never waits for the host), giving the kernel's average duration in the timed region
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_avg_ms = e0.elapsed_time(e1) / args.steps
    # per-launch spread (each launch bracketed by its own events; includes launch gaps)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    kms = sorted(a.elapsed_time(b) for a, b in evs)
    k_med_ms = kms[len(kms) // 2]

    # measured write roofline: a plain fill of the same 256 MiB buffer
    fill_evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for _ in range(3):
        out.fill_(1.0)
    for a, b in fill_evs:
        a.record(stream)
        out.fill_(1.0)
        b.record(stream)
    torch.cuda.synchronize()
    fill_ms = sorted(a.elapsed_time(b) for a, b in fill_evs)[len(fill_evs) // 2]
    if args.profile_calibration:
        src = torch.empty_like(out).fill_(2.0)
        for _ in range(5):
            out.copy_(src)
        torch.cuda.synchronize()
        del src

    # the other kernel choices on the same field, for context (event-timed, 10 launches)
    paths = {}
    for name in ("general", "dyadic"):
        q = ptg.params(dim=2, smoothness=1, octaves=OCTAVES, persistence=PERSISTENCE, lacunarity=LACUNARITY,
                       base_freq=BASE_FREQ, seed=SEED, path=name)
        ptg.fbm_2d_raw(q, 0, 0, NX, NY, ptr, NX, sh)
        a2, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a2.record(stream)
        for _ in range(10):
            ptg.fbm_2d_raw(q, 0, 0, NX, NY, ptr, NX, sh)
        b2.record(stream)
        torch.cuda.synchronize()
        paths[name] = a2.elapsed_time(b2) / 10

    samples = NX * NY
    osamp = samples * OCTAVES
    ms_per_step = wall * 1e3 / args.steps
    value = osamp * args.steps / wall
    out_bytes = samples * 4
    achieved_gbs = out_bytes / (k_avg_ms * 1e-3) / 1e9
    fill_gbs = out_bytes / (fill_ms * 1e-3) / 1e9

    # sanity: the field is finite and within the total amplitude bound of 2D C1 cells
    step()
    torch.cuda.synchronize()
    amax = float(out.abs().max())
    total_amp = sum(PERSISTENCE ** o for o in range(OCTAVES))
    if not (amax == amax and amax <= 0.5 * total_amp):
        print(f"field out of bounds: max|H| = {amax}", file=sys.stderr)
        sys.exit(1)

    progress(f"headline field: {k_avg_ms * 1e3:.1f} us per launch (back to back), {ms_per_step * 1e3:.1f} us per step")
    others = None if args.no_other_configs else other_configs(torch, ptg, stream)
    progress("other configurations done")
    stages = None if args.no_other_configs else stage_kernels(torch, ptg, stream)
    progress("stage kernels done")
    serving = run_serving(args.serve_requests) if args.serve_requests > 0 else None
    progress("serving done")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)
        progress("oracle timing done")

    rec = {
        "metric": "octave-samples/s at 8192^2 8-octave 2D",
        "value": value,
        "unit": "octave-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (lattice hashed from seed 1; no dataset)",
        "config": {
            "workload": "2D fBm heightmap 8192x8192, 8 octaves, base lattice 16x16, lacunarity 2, "
                        "persistence 0.5, C1 cubic cells, FP32 output, seed 1, origin (0,0)",
            "nx": NX, "ny": NY, "octaves": OCTAVES, "base_freq": BASE_FREQ, "smoothness": 1,
            "form": "plain", "path": args.path,
        },
        "kernel_choice_avg_ms": paths,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic() if args.path in ("auto", "dyadic") else None,
            "kernel": "k_fbm2d_strip (one launch per step)" if args.path != "general" else "k_fbm2d_general",
            "kernel_avg_ms": k_avg_ms,
            "kernel_median_ms_single_launch": k_med_ms,
            "algorithmic_bytes_per_launch": out_bytes,
        },
        "write_roofline_measured": {
            "kernel": "torch fill_ of the same 256 MiB buffer",
            "median_ms": fill_ms,
            "GB/s": fill_gbs,
            "frac_of_peak": fill_gbs / HBM_PEAK_GBS,
            "path_frac_of_measured": achieved_gbs / fill_gbs,
        },
        "cpu_baseline": cpu,
        "other_configs": others,
        "stage_kernels": stages,
        "serving": serving,
    }
    print(json.dumps(rec), flush=True)


# ---- the other benchmark fields ---------------------------------------------------------
def _time_launches(torch, stream, fn, n=10):
    """Average time of n back-to-back launches, after one warm-up launch and a short idle
    period (the previous configuration's heavy launches leave the clock lowered for a while;
    every configuration starts from the same state)."""
    fn()
    torch.cuda.synchronize()
    time.sleep(0.3)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(n):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / n


def other_configs(torch, ptg, stream):
    """3D 512^3 6-octave C2 volume; 16384^2 10-octave field at a world offset of 2^24 cells
    through the plain FP32 path and the FP16 / BF16 matrix-core form (their errors against
    the FP64 oracle are measured by the GPU tests); the zero-gradient model on the 8192^2
    8-octave field (dyadic and general ladders) and the height-and-gradient model on it (C1,
    C2); 256^2 4-octave field (launch-bound)."""
    res = {}
    sh = stream.cuda_stream
    # 3D 512^3, 6 octaves, base lattice 8^3, C2
    vol = torch.empty((512, 512, 512), dtype=torch.float32, device="cuda")
    p3 = ptg.params(dim=3, smoothness=2, octaves=6, base_freq=8 / 512, seed=1)
    ms = _time_launches(torch, stream, lambda: ptg.fbm_3d_raw(p3, 0, 0, 0, 512, 512, 512, vol.data_ptr(), sh), 5)
    n3 = 512 ** 3
    res["3d_512_6oct_c2"] = {"workload": "3D fBm 512^3, 6 octaves, base lattice 8^3, C2 quintic, FP32, seed 1",
                             "kernel": "k_fbm3d_strip", "ms": ms, "octave_samples_s": n3 * 6 / (ms * 1e-3),
                             "hbm_frac": n3 * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    hg3 = {}
    for sm in (1, 2):  # D3M1N3 / D3M2N5 with node heights and w-weighted gradients
        q3 = ptg.params(dim=3, smoothness=sm, octaves=6, base_freq=8 / 512, seed=1, model="height_gradient",
                        gradient_weight=0.01)
        ms3 = _time_launches(torch, stream, lambda: ptg.fbm_3d_raw(q3, 0, 0, 0, 512, 512, 512, vol.data_ptr(), sh), 5)
        hg3[f"C{sm}"] = {"ms": ms3, "octave_samples_s": n3 * 6 / (ms3 * 1e-3),
                         "hbm_frac": n3 * 4 / (ms3 * 1e-3) / 1e9 / HBM_PEAK_GBS}
    res["3d_512_6oct_height_gradient"] = {
        "workload": "3D fBm 512^3, 6 octaves, base lattice 8^3, node heights and gradients (weight 0.01), FP32, "
                    "seed 1, 3D strip kernel", "smoothness": hg3}
    del vol
    progress(f"3D 512^3 C2: {ms * 1e3:.1f} us; heights and gradients C1 {hg3['C1']['ms'] * 1e3:.1f} us, "
             f"C2 {hg3['C2']['ms'] * 1e3:.1f} us")
    # 16384^2, 10 octaves, base lattice 32^2, offset (2^24 - 3) * 512, -(2^24 - 5) * 512
    n, f0 = 16384, 32 / 16384
    x0, y0 = (2 ** 24 - 3) * 512, -(2 ** 24 - 5) * 512
    forms = {}
    for form, basis, dt in (("plain", "monomial", torch.float32), ("plain", "monomial", torch.float16),
                            ("mfma_f16", "monomial", torch.float16), ("mfma_f16", "centred", torch.float16),
                            ("mfma_f16", "hermite", torch.float16), ("mfma_bf16", "monomial", torch.float16),
                            ("mfma_bf16", "centred", torch.float16), ("mfma_bf16", "hermite", torch.float16)):
        out = torch.empty((n, n), dtype=dt, device="cuda")
        q = ptg.params(smoothness=1, octaves=10, base_freq=f0, seed=1, form=form, basis=basis,
                       out_dtype=ptg.PTG_F16 if dt == torch.float16 else ptg.PTG_F32)
        ms = _time_launches(torch, stream, lambda: ptg.fbm_2d_raw(q, x0, y0, n, n, out.data_ptr(), n, sh), 5)
        name = f"{form}/{basis}" if form != "plain" else ("plain_fp32" if dt == torch.float32 else "plain_fp16_out")
        progress(f"16384^2 10-octave {name}: {ms * 1e3:.1f} us")
        forms[name] = {
            "ms": ms, "octave_samples_s": n * n * 10 / (ms * 1e-3),
            "hbm_frac": n * n * out.element_size() / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del out
    res["2d_16384_10oct_offset"] = {
        "workload": "2D fBm 16384^2, 10 octaves, base lattice 32^2, world offset (2^24-3)*512, -(2^24-5)*512 "
                    "samples, C1; FP16 output for the matrix-core forms, FP32 for the plain path",
        "forms": forms}
    # the zero-gradient model (Sec. 3.3) on the headline field: 8192^2, 8 octaves, base lattice 16^2
    zf = torch.empty((8192, 8192), dtype=torch.float32, device="cuda")
    zg = {}
    for name, f0z, lac in (("dyadic (strip kernel)", 16 / 8192, 2.0), ("base 0.0031, lacunarity 2.1 (general)",
                                                                      0.0031, 2.1)):
        q = ptg.params(smoothness=1, octaves=8, base_freq=f0z, lacunarity=lac, seed=1, model="zero_gradient")
        ms = _time_launches(torch, stream, lambda: ptg.fbm_2d_raw(q, 0, 0, 8192, 8192, zf.data_ptr(), 8192, sh), 10)
        zg[name] = {"ms": ms, "octave_samples_s": 8192 * 8192 * 8 / (ms * 1e-3),
                    "hbm_frac": 8192 * 8192 * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    progress("zero-gradient model done")
    res["2d_8192_8oct_zero_gradient"] = {
        "workload": "zero-gradient D2M1N3 (random node heights, zero corner gradients), 8192^2, 8 octaves, "
                    "persistence 0.5, FP32, seed 1",
        "ladders": zg}
    # heights and w-weighted gradients (tensor Hermite), same field, C1 and C2, w = 0.01
    hg = {}
    for m in (1, 2):
        q = ptg.params(smoothness=m, octaves=8, base_freq=16 / 8192, seed=1, model="height_gradient",
                       gradient_weight=0.01)
        ms = _time_launches(torch, stream, lambda: ptg.fbm_2d_raw(q, 0, 0, 8192, 8192, zf.data_ptr(), 8192, sh), 10)
        hg[f"C{m}"] = {"ms": ms, "octave_samples_s": 8192 * 8192 * 8 / (ms * 1e-3),
                       "hbm_frac": 8192 * 8192 * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    q = ptg.params(smoothness=3, octaves=8, base_freq=16 / 8192, seed=1)
    ms = _time_launches(torch, stream, lambda: ptg.fbm_2d_raw(q, 0, 0, 8192, 8192, zf.data_ptr(), 8192, sh), 5)
    res["2d_8192_8oct_c3"] = {"workload": "septic (C3) cells, gradient model, 8192^2, 8 octaves, base lattice 16^2, "
                                          "FP32, seed 1 (strip kernel)",
                              "ms": ms, "octave_samples_s": 8192 * 8192 * 8 / (ms * 1e-3),
                              "hbm_frac": 8192 * 8192 * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    progress("height-gradient and septic done")
    gx, gy = torch.empty_like(zf), torch.empty_like(zf)
    q = ptg.params(smoothness=1, octaves=8, base_freq=16 / 8192, seed=1)
    ms = _time_launches(torch, stream, lambda: ptg.lib().ptg_fbm_2d_grad(
        ctypes.byref(q), 0, 0, 8192, 8192, zf.data_ptr(), gx.data_ptr(), gy.data_ptr(), 8192, sh), 5)
    res["2d_8192_8oct_gradient_output"] = {
        "workload": "H, dH/dX, dH/dY of the 8192^2 8-octave C1 field (three FP32 outputs; one strip-kernel launch)",
        "ms": ms, "octave_samples_s": 8192 * 8192 * 8 / (ms * 1e-3),
        "hbm_frac": 3 * 8192 * 8192 * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    del gx, gy
    res["2d_8192_8oct_height_gradient"] = {
        "workload": "heights and gradients (weight 0.01) in tensor Hermite cells, 8192^2, 8 octaves, base lattice "
                    "16^2, FP32, seed 1, strip kernel",
        "smoothness": hg}
    # comparison paths at the same field's parameters: Perlin's noise (S3 and S5 fades) on the
    # general kernel, the simplex-lattice noise on its own kernel, and the polynomial cells
    # on the general kernel (the same tile machinery as Perlin) and the strip kernel
    cmp = {}
    for name, kw in (("polynomial_c1_strip", dict(smoothness=1)),
                     ("polynomial_c1_general", dict(smoothness=1, path="general")),
                     ("perlin_s3_general", dict(model="perlin", smoothness=1)),
                     ("perlin_s5_general", dict(model="perlin", smoothness=2)),
                     ("simplex_lattice", dict(model="simplex"))):
        q = ptg.params(octaves=8, base_freq=16 / 8192, seed=1, **kw)
        ms = _time_launches(torch, stream, lambda: ptg.fbm_2d_raw(q, 0, 0, 8192, 8192, zf.data_ptr(), 8192, sh), 5)
        cmp[name] = {"ms": ms, "octave_samples_s": 8192 * 8192 * 8 / (ms * 1e-3),
                     "hbm_frac": 8192 * 8192 * 4 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        progress(f"comparison path {name}: {ms * 1e3:.1f} us")
    res["2d_8192_8oct_comparison_paths"] = {
        "workload": "8192^2, 8 octaves, base lattice 16^2, persistence 0.5, FP32, seed 1: Perlin's gradient noise "
                    "(Sec. 3.2) and simplex-lattice gradient noise (standing for the paper's OpenSimplex) on the "
                    "same hashed unit gradients, next to the polynomial C1 cells",
        "paths": cmp}
    del zf
    # 256^2, 4 octaves, base lattice 8^2
    small = torch.empty((256, 256), dtype=torch.float32, device="cuda")
    q = ptg.params(smoothness=1, octaves=4, base_freq=8 / 256, seed=1)
    ms = _time_launches(torch, stream, lambda: ptg.fbm_2d_raw(q, 0, 0, 256, 256, small.data_ptr(), 256, sh), 20)
    res["2d_256_4oct"] = {"workload": "2D fBm 256^2, 4 octaves, base lattice 8^2, C1, FP32", "ms": ms,
                          "octave_samples_s": 256 * 256 * 4 / (ms * 1e-3)}
    return res


def stage_kernels(torch, ptg, stream):
    """The stand-alone stage kernels against the HBM roofline: a1 coordinate step, K1
    lattice hash (2D keys + gradients, 2D node heights, 3D keys + second words +
    gradients), K2 per-cell coefficients (2D, 3D; cubic and quintic).  Algorithmic bytes =
    what the call must write plus what it must read (K2 reads the node gradients once)."""
    res = {}
    sh = stream.cuda_stream
    lib = ptg.lib()

    def rec(name, workload, kernel, call, wbytes, rbytes, n=10):
        def fn():
            rc = call()
            if rc != 0:
                raise RuntimeError(f"{name}: status {rc}: {lib.ptg_last_error().decode()}")
        ms = _time_launches(torch, stream, fn, n)
        progress(f"stage kernel {name}: {ms * 1e3:.1f} us")
        gbs = (wbytes + rbytes) / (ms * 1e-3) / 1e9
        res[name] = {"workload": workload, "kernel": kernel, "us": ms * 1e3, "bytes_written": wbytes,
                     "bytes_read": rbytes, "GB_s": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}

    n = 1 << 23
    cells = torch.empty((8, n), dtype=torch.int64, device="cuda")
    frac = torch.empty((8, n), dtype=torch.float32, device="cuda")
    rec("coords_8M_8oct", "a1: 2^23 samples x 8 octaves (cell int64 + fraction FP32)", "k_coords",
        lambda: lib.ptg_coords(2.0 ** -9, 2.0, 8, -(2 ** 40), n, cells.data_ptr(), frac.data_ptr(), sh),
        8 * n * 12, 0)
    del cells, frac
    nx = ny = 8192
    keys = torch.empty((ny, nx), dtype=torch.int32, device="cuda")
    grad = torch.empty((2, ny, nx), dtype=torch.float32, device="cuda")
    rec("lattice2d_8192x8192", "K1 2D: 8192^2 nodes, keys + unit gradients (12 B per node)", "k_lattice2d",
        lambda: lib.ptg_lattice_2d(1, 3, -(2 ** 33), 2 ** 20, nx, ny, keys.data_ptr(), grad.data_ptr(), sh),
        nx * ny * 12, 0)
    rec("heights2d_8192x8192", "K1 2D node heights (zero-gradient model): 8192^2 nodes (4 B per node)",
        "k_heights2d", lambda: lib.ptg_heights_2d(1, 3, 0, 0, nx, ny, grad.data_ptr(), sh), nx * ny * 4, 0)
    del keys, grad
    m = 256
    keys = torch.empty((m, m, m), dtype=torch.int32, device="cuda")
    sec = torch.empty((m, m, m), dtype=torch.int32, device="cuda")
    grad = torch.empty((3, m, m, m), dtype=torch.float32, device="cuda")
    rec("lattice3d_256cubed", "K1 3D: 256^3 nodes, keys + second words + unit gradients (20 B per node)",
        "k_lattice3d",
        lambda: lib.ptg_lattice_3d(1, 2, 0, -(2 ** 30), 7, m, m, m, keys.data_ptr(), sec.data_ptr(),
                                   grad.data_ptr(), sh), m ** 3 * 20, 0)
    del keys, sec, grad
    for smooth, nn in ((1, 4097), (2, 2049)):
        n1 = 2 * smooth + 2
        grad = torch.empty((2, nn, nn), dtype=torch.float32, device="cuda")
        lib.ptg_lattice_2d(1, 0, 0, 0, nn, nn, None, grad.data_ptr(), sh)
        coeff = torch.empty(((nn - 1) ** 2 * n1 * n1,), dtype=torch.float32, device="cuda")
        rec(f"cells2d_c{smooth}_{nn}", f"K2 2D C{smooth}: {nn}^2 nodes -> {(nn - 1)}^2 cells x {n1 * n1} "
            "FP32 coefficients", f"k_cells2d<{smooth}>",
            lambda: lib.ptg_cells_2d(smooth, grad.data_ptr(), nn, nn, ctypes.c_float(0.5), coeff.data_ptr(), sh),
            (nn - 1) ** 2 * n1 * n1 * 4, nn * nn * 8)
        del grad, coeff
    for smooth, nn in ((1, 129), (2, 65)):
        n1 = 2 * smooth + 2
        grad = torch.empty((3, nn, nn, nn), dtype=torch.float32, device="cuda")
        lib.ptg_lattice_3d(1, 0, 0, 0, 0, nn, nn, nn, None, None, grad.data_ptr(), sh)
        coeff = torch.empty(((nn - 1) ** 3 * n1 ** 3,), dtype=torch.float32, device="cuda")
        rec(f"cells3d_c{smooth}_{nn}", f"K2 3D C{smooth}: {nn}^3 nodes -> {(nn - 1)}^3 cells x {n1 ** 3} "
            "FP32 coefficients", f"k_cells3d<{smooth}>",
            lambda: lib.ptg_cells_3d(smooth, grad.data_ptr(), nn, nn, nn, ctypes.c_float(1.0), coeff.data_ptr(), sh),
            (nn - 1) ** 3 * n1 ** 3 * 4, nn ** 3 * 12)
        del grad, coeff
    return res


# ---- tile stream -------------------------------------------------------------------
SERVE_F0 = 2.0 ** -12  # world-fixed base frequency so that tiles stitch (4096 samples per cell)


def tile_stream(n, seed=1610):
    """Requests of the serving workload: 90% 2D tiles of side in {128..2048} with 4..12
    octaves, 10% 3D tiles of side in {64, 128, 256} with 4..8 octaves; C1/C2 50/50; int64
    world origins in [-2^46, 2^46); random 32-bit seeds."""
    import numpy as np

    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        if rng.random() < 0.9:
            dim, side, octs = 2, int(rng.choice([128, 256, 512, 1024, 2048])), int(rng.integers(4, 13))
            ext = (side, side, 1)
        else:
            dim, side, octs = 3, int(rng.choice([64, 128, 256])), int(rng.integers(4, 9))
            ext = (side, side, side)
        smooth = int(rng.integers(1, 3))
        org = [int(v) for v in rng.integers(-(1 << 46), 1 << 46, size=3)]
        if dim == 2:
            org[2] = 0
        out.append(dict(dim=dim, smoothness=smooth, octaves=octs, seed=int(rng.integers(0, 1 << 32)),
                        origin=org, extent=ext))
    return out


def run_serving(n):
    """The tile stream through the server and through the plain per-tile path (one
    ptg_fbm_* call per request; auto kernel choice), driven by the native open-loop
    generator: capacity (all requests at t = 0) and Poisson arrivals at 0.5, 0.8, 0.95 of
    the plain path's capacity.  Latency = host-visible completion - arrival; p50/p99 over
    the steady state (the first 10% of requests dropped)."""
    import ctypes

    import numpy as np
    import torch

    import paper_1610_03525_amd as ptg

    lg = ctypes.CDLL(os.path.join(os.path.dirname(ptg.LIB_PATH), "libptg_loadgen.so"))
    p64 = ctypes.POINTER(ctypes.c_int64)
    lg.ptg_lg_served.argtypes = [ctypes.c_void_p, ctypes.POINTER(ptg.TileReq), p64, ctypes.c_int32, p64, p64,
                                 ctypes.c_int32]
    lg.ptg_lg_plain.argtypes = [ctypes.POINTER(ptg.TileReq), p64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.c_int32, ctypes.c_int32, p64, p64]
    reqs = tile_stream(n)
    treq = (ptg.TileReq * n)()
    for i, r in enumerate(reqs):
        treq[i] = ptg.tile_req(dim=r["dim"], origin=r["origin"], extent=r["extent"], user_tag=i,
                               smoothness=r["smoothness"], octaves=r["octaves"], base_freq=SERVE_F0, seed=r["seed"])
    osamp = sum(r["extent"][0] * r["extent"][1] * r["extent"][2] * r["octaves"] for r in reqs)
    arena_bytes = 4 << 30
    arena = torch.empty(arena_bytes, dtype=torch.uint8, device="cuda")

    def i64(x):
        return np.ascontiguousarray(x, dtype=np.int64)

    def ptr(a):
        return a.ctypes.data_as(p64)

    def summary(arr, done):
        lat = (done - arr) / 1e6
        k = n // 10
        span = (done.max() - arr[0]) / 1e9
        return {"p50_ms": round(float(np.percentile(lat[k:], 50)), 4),
                "p99_ms": round(float(np.percentile(lat[k:], 99)), 4),
                "tiles_s": round(n / span, 1), "octave_samples_s": osamp / span}

    def plain(arr, mode):
        arr, done, st = i64(arr), i64(np.zeros(n)), i64(np.zeros(3))
        rc = lg.ptg_lg_plain(treq, ptr(arr), n, arena.data_ptr(), arena_bytes, mode, 64, ptr(done), ptr(st))
        if rc != 0:
            raise RuntimeError(f"plain stream failed ({rc}): {ptg.last_error()}")
        out = summary(arr, done)
        progress(f"plain stream (mode {mode}): {out}")
        out["launch_units"] = int(st[0])
        return out

    def served(arr, budget):
        arr, done, adm = i64(arr), i64(np.zeros(n)), i64(np.zeros(n))
        with ptg.Server(budget) as srv:
            rc = lg.ptg_lg_served(srv.h, treq, ptr(arr), n, ptr(done), ptr(adm), 0)
            if rc != 0:
                raise RuntimeError(f"served stream failed ({rc}): {ptg.last_error()}")
            st = srv.stats()
        out = summary(arr, done)
        progress(f"served stream (budget {budget >> 20} MiB): {out}")
        out["admit_wait_p99_ms"] = round(float(np.percentile((adm - arr)[n // 10:] / 1e6, 99)), 4)
        out["kernel_launches"] = st["kernel_launches"]
        out["bytes_peak"] = st["bytes_peak"]
        return out

    def solo():
        arr, done, st = i64(np.zeros(n)), i64(np.zeros(n)), i64(np.zeros(3))
        rc = lg.ptg_lg_plain(treq, ptr(arr), n, arena.data_ptr(), arena_bytes, 2, 1, ptr(done), ptr(st))
        if rc != 0:
            raise RuntimeError(f"solo pass failed ({rc}): {ptg.last_error()}")
        total = done.sum() / 1e9
        out = {"kernel_s_sum": round(float(total), 6), "tiles_s_bound": round(n / total, 1),
               "octave_samples_s_bound": osamp / total,
               "kernel_ms_p50": round(float(np.percentile(done / 1e6, 50)), 4)}
        progress(f"solo kernels: {out}")
        return out

    zero = np.zeros(n)
    bound = solo()
    # the 4 GiB budget holds an eighth of the stream's 31 GiB of outputs (admission waits for
    # releases); 64 GiB holds all of it (an MI355X has 288 GB)
    cap = {"plain": plain(zero, 0), "served": served(zero, 4 << 30), "served_64GiB": served(zero, 64 << 30)}
    for v in cap.values():
        v["frac_of_solo_bound"] = round(v["tiles_s"] / bound["tiles_s_bound"], 4)
    rate = cap["plain"]["tiles_s"]
    gaps = np.random.default_rng(1611).exponential(1.0, size=n)
    loads = []
    for f in (0.5, 0.8, 0.95):
        arr = np.cumsum(gaps) / (f * rate) * 1e9
        arr -= arr[0]
        loads.append({"load": f, "rate_req_s": round(f * rate, 1), "plain": plain(arr, 0),
                      "served": served(arr, 4 << 30)})
    arr = np.cumsum(gaps) / (0.8 * rate) * 1e9
    arr -= arr[0]
    budgets = {f"{b}GiB": served(arr, b << 30) for b in (1, 16)}
    budgets["4GiB"] = loads[1]["served"]
    del arena
    lat = run_lattice_cache(lg, ptg, max(200, n // 4))
    return {
        "lattice_cache": lat,
        "workload": "terrain-tile stream: 90% 2D tiles side in {128,256,512,1024,2048}, octaves 4..12; "
                    "10% 3D tiles side in {64,128,256}, octaves 4..8; C1/C2 50/50; base frequency 2^-12, "
                    "lacunarity 2, persistence 0.5; random int64 origins and seeds; FP32 output; seed 1610",
        "requests": n,
        "octave_samples": osamp,
        "plain_path": "one ptg_fbm_2d/3d call per request on one stream (auto kernel choice)",
        "plain_graph": "not run: the stream driver's graph mode (arrived requests as one ptg_batch graph, "
                       "updated in place when a batch shape recurs) is switched off after a segmentation fault "
                       "of unknown cause in an open-loop stream",
        "served_path": "ptg_tiles_submit into one persistent kernel (dyadic 2D / 3D requests on the strip "
                       "code, the rest on general tiles), HBM budget 4 GiB (capacity also at 64 GiB: every "
                       "output of the stream resident); completions taken in request order and released at once",
        "solo_bound": bound,
        "solo_bound_note": "each request's kernels timed alone between two events (plain path, auto kernel "
                           "choice), one after the other; the sum is the GPU time the stream needs without "
                           "overlap between requests",
        "capacity": cap,
        "open_loop": loads,
        "served_budget_at_0.8": budgets,
    }


def lattice_streams(n, seed=1612):
    """Two general-tile streams (base frequency 0.0031: not a dyadic ladder), C1/C2 50/50,
    8 octaves, 256 x 256 requests: "world", one seed and a viewer panning over a 2048 x
    2048 neighbourhood in steps of 64 samples (neighbouring requests overlap); and
    "independent", a fresh seed and random origin per request (nothing to share)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    world, indep = [], []
    x = y = 0
    for i in range(n):
        x = int(np.clip(x + 64 * rng.integers(-1, 2), 0, 1792))
        y = int(np.clip(y + 64 * rng.integers(-1, 2), 0, 1792))
        sm = 1 + i % 2
        world.append(dict(origin=(x, y, 0), seed=77, smoothness=sm))
        indep.append(dict(origin=tuple(int(v) for v in rng.integers(-(1 << 40), 1 << 40, 2)) + (0,),
                          seed=int(rng.integers(0, 1 << 32)), smoothness=sm))
    return world, indep


def run_lattice_cache(lg, ptg, n):
    """Capacity of the served general-tile streams (all n requests at t = 0, budget 4 GiB):
    hashing every node ("hash", the default), with the lattice cache starting empty
    ("cache_cold") and with the same stream again on the same server ("cache_warm": every
    block resident).  Requests/s and block hits and misses; "hash" is the better of two
    passes (the first includes the persistent kernel's launch)."""
    import numpy as np

    p64 = ctypes.POINTER(ctypes.c_int64)
    out = {"requests": n, "extent": [256, 256], "octaves": 8, "base_freq": 0.0031}

    def one(srv, treq):
        arr = np.zeros(n, dtype=np.int64)
        done, adm = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
        rc = lg.ptg_lg_served(srv.h, treq, arr.ctypes.data_as(p64), n, done.ctypes.data_as(p64),
                              adm.ctypes.data_as(p64), 0)
        if rc != 0:
            raise RuntimeError(f"lattice-cache stream failed ({rc}): {ptg.last_error()}")
        span = (done.max() - arr[0]) / 1e9
        st = srv.stats()
        return {"requests_s": round(n / span, 1), "octave_samples_s": n * 256 * 256 * 8 / span,
                "lat_hits": st["lat_hits"], "lat_misses": st["lat_misses"], "lat_blocks": st["lat_blocks"]}

    for name, stream in zip(("world", "independent"), lattice_streams(n)):
        treq = (ptg.TileReq * n)()
        for i, r in enumerate(stream):
            treq[i] = ptg.tile_req(dim=2, origin=r["origin"], extent=(256, 256, 1), user_tag=i,
                                   smoothness=r["smoothness"], octaves=8, base_freq=0.0031, seed=r["seed"])
        res = {}
        with ptg.Server(4 << 30) as srv:
            a, b = one(srv, treq), one(srv, treq)
            res["hash"] = a if a["requests_s"] > b["requests_s"] else b
        with ptg.Server(4 << 30, lattice_cache=1) as srv:
            res["cache_cold"] = one(srv, treq)
            warm = one(srv, treq)
            warm["lat_hits"] -= res["cache_cold"]["lat_hits"]
            warm["lat_misses"] -= res["cache_cold"]["lat_misses"]
            res["cache_warm"] = warm
        progress(f"lattice cache, {name} stream done")
        res["warm_over_hash"] = round(res["cache_warm"]["requests_s"] / res["hash"]["requests_s"], 3)
        out[name] = res
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(fn, unit_samples, octaves, total_units, budget_s):
    """Call fn(i) for units i = 0, 1, ... (row bands / z-slabs) until the budget is spent or
    the workload is done; octave-samples/s and what was covered."""
    done = 0
    t0 = time.perf_counter()
    while done < total_units and (done == 0 or time.perf_counter() - t0 < budget_s):
        fn(done)
        done += 1
    dt = time.perf_counter() - t0
    return done * unit_samples * octaves / dt, done, dt


def cpu_baseline(budget_s):
    """FP64 oracle on the host cores: row bands of the headline field until the time budget
    is spent (rate in octave-samples/s = the reported value), then every configuration of
    the benchmark on all cores and on one core, each over a bounded sample (whole field for
    the 256^2 one, row bands / z-slabs of the others)."""
    import numpy as np  # noqa: F401

    import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    band = 64
    rate, bands, dt = _oracle_rate(
        lambda i: O.fbm_2d(1, OCTAVES, PERSISTENCE, LACUNARITY, BASE_FREQ, SEED, 0, i * band, NX, band,
                           nthreads=threads), NX * band, OCTAVES, NY // band, budget_s)
    rows = bands * band
    # every configuration, all cores and one core
    x4, y4 = (2 ** 24 - 3) * 512, -(2 ** 24 - 5) * 512
    cfgs = {
        "2d_256_4oct_c1": (lambda i, t: O.fbm_2d(1, 4, 0.5, 2.0, 8 / 256, 1, 0, 0, 256, 256, nthreads=t),
                           256 * 256, 4, 400, "the whole 256^2 field, repeated"),
        "2d_8192_8oct_c1": (lambda i, t: O.fbm_2d(1, 8, 0.5, 2.0, 16 / 8192, 1, 0, 16 * i, 8192, 16, nthreads=t),
                            8192 * 16, 8, 512, "16-row bands of the 8192^2 field"),
        "3d_512_6oct_c2": (lambda i, t: O.fbm_3d(2, 6, 0.5, 2.0, 8 / 512, 1, 0, 0, i, 512, 512, 1, nthreads=t),
                           512 * 512, 6, 512, "z-slices of the 512^3 volume"),
        "2d_16384_10oct_c1_offset": (lambda i, t: O.fbm_2d(1, 10, 0.5, 2.0, 32 / 16384, 1, x4, y4 + 8 * i, 16384, 8,
                                                           nthreads=t),
                                     16384 * 8, 10, 2048, "8-row bands of the 16384^2 field at the 2^24-cell offset"),
    }
    per = {}
    for name, (fn, unit, octs, total, what) in cfgs.items():
        entry = {"sample": what}
        for label, t, b in (("all_cores", threads, 2.0), ("one_core", 1, 1.0)):
            r, n, d = _oracle_rate(lambda i, t=t: fn(i, t), unit, octs, total, b)
            entry[label] = {"octave_samples_s": r, "units": n, "seconds": round(d, 2)}
        entry["core_speedup"] = entry["all_cores"]["octave_samples_s"] / entry["one_core"]["octave_samples_s"]
        per[name] = entry
        progress(f"oracle {name}: {entry['all_cores']['octave_samples_s']:.3e} octave-samples/s on {threads} cores, "
                 f"{entry['one_core']['octave_samples_s']:.3e} on one")
    return {
        "value": rate,
        "unit": "octave-samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"rows 0..{rows - 1} of the 8192x8192 8-octave field ({rows * NX} samples, {dt:.1f} s wall)",
        "nproc": os.cpu_count(),
        "cpu_model": _cpu_model(),
        "per_config": per,
    }


if __name__ == "__main__":
    main()
