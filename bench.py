"""Benchmark: octave-samples/s of the dense fBm path on one MI355X.

Workload (the throughput configuration): 2D fBm heightmap 8192 x 8192, 8 octaves, base
lattice 16 x 16 cells (base frequency 16/8192), lacunarity 2, persistence 0.5, C1 cubic
cells, unit gradients from the stated lattice hash, FP32 output, seed 1, origin (0, 0).
A step is one ptg_fbm_2d call: coordinate step, lattice hash, per-cell coefficients,
evaluation and octave accumulation for the whole field.  Inputs are parameters only;
the output buffer is allocated before the timed region.

Prints ONE JSON line (rank 0).  Extra fields: the measured pure-store write roofline,
per-kernel event timing, and the FP64 CPU oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

NX = NY = 8192
OCTAVES = 8
BASE_FREQ = 16 / 8192
PERSISTENCE = 0.5
LACUNARITY = 2.0
SEED = 1
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fbm2d_dyadic_2d_8192x8192_8oct_c1.traffic.json")


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs,
    or None when the kernel source has changed since they were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
        with open(os.path.join(ROOT, t["source"]), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != t["source_sha256"]:
                return None
        return t["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall-time budget of the oracle sample")
    ap.add_argument("--path", default="auto", choices=["auto", "general", "dyadic"])
    ap.add_argument("--profile-calibration", action="store_true",
                    help="also run a plain torch fill and copy of the field size (counter calibration)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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

    # timed region: exactly `steps` steps, bracketed by device synchronisation
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # per-launch kernel duration with HIP events on the launch stream
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize()
    kms = sorted(a.elapsed_time(b) for a, b in evs)
    k_avg_ms = sum(kms) / len(kms)
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
        e2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
        for a, b in e2:
            a.record(stream)
            ptg.fbm_2d_raw(q, 0, 0, NX, NY, ptr, NX, sh)
            b.record(stream)
        torch.cuda.synchronize()
        paths[name] = sorted(a.elapsed_time(b) for a, b in e2)[5]

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

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_seconds)

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
        "kernel_choice_median_ms": paths,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": measured_traffic() if args.path in ("auto", "dyadic") else None,
            "kernel": "k_fbm2d_dyadic (one launch per step)" if args.path != "general" else "k_fbm2d_general",
            "kernel_avg_ms": k_avg_ms,
            "kernel_median_ms": k_med_ms,
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
    }
    print(json.dumps(rec), flush=True)


def cpu_baseline(budget_s):
    """FP64 oracle on the host cores: row bands of the same field until the time budget
    is spent (or the field is done); rate in octave-samples/s."""
    import numpy as np  # noqa: F401

    import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    band = 64
    rows = 0
    t0 = time.perf_counter()
    while rows < NY and time.perf_counter() - t0 < budget_s:
        O.fbm_2d(1, OCTAVES, PERSISTENCE, LACUNARITY, BASE_FREQ, SEED, 0, rows, NX, band, nthreads=threads)
        rows += band
    dt = time.perf_counter() - t0
    return {
        "value": rows * NX * OCTAVES / dt,
        "unit": "octave-samples/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"rows 0..{rows - 1} of the 8192x8192 8-octave field ({rows * NX} samples, {dt:.1f} s wall)",
    }


if __name__ == "__main__":
    main()
