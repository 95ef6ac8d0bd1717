"""Benchmark of the colour-gradient LBM hot path on one MI355X.

Workload (default): the translating-droplet case -- 256^3 periodic box, red
droplet of radius 32 moving with u = 0.05 along x in a blue carrier, density
ratio 10, equal dynamic viscosities, shear rate 1.6 and bulk rate 1.0,
sigma = 0.005, beta = 0.7, +-1e-6 counter noise on the populations, FP32
storage and arithmetic.  A step is one full time update of every node
(pull-streaming, moments, interface stencils, collision, recolouring).

Prints ONE JSON line: MLUPS of the timed steps, the roofline of the dominant
kernel (algorithmic bytes per launch / average launch time from HIP events
recorded on the launch stream during the timed region), and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per node of each kernel (FP32): what it must read and write
KERNEL_BYTES = {
    "pull": 54 * 4 + 11 * 4,          # 54 populations in, 11 local moments out
    "interface": (2 + 3) * 4 + 9 * 4,  # rho_r, rho_b, j in; n, F, Q out
    "collide": 20 * 4 + 54 * 4,        # moments + interface fields in, 54 populations out
    "fused": 11 * 4 + 54 * 4,          # local moments in, 54 populations out
}
STEP_BYTES = 2 * 54 * 4               # whole step: every population read once, written once


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256, help="box edge (default 256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--variant", type=int, default=-1,
                    help="fused launch geometry (default: autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy (counter calibration)")
    return ap.parse_args()


COUNTERS = os.path.join(ROOT, "profiles", "k_fused_translating_droplet_256_hbm_counters.md")
SOURCES = ("paper_2309_07801_amd/csrc/kernels.hpp", "paper_2309_07801_amd/csrc/lattice.hpp",
           "paper_2309_07801_amd/csrc/cglbm.hip")


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (already scaled by the copy-kernel
    calibration), or None if the summary is missing or the kernel sources
    changed since the counters were taken."""
    import hashlib
    import re
    if not os.path.exists(COUNTERS):
        return None
    text = open(COUNTERS).read()
    m = re.search(r"source_sha256: ([0-9a-f]{64})", text)
    h = hashlib.sha256()
    for f in SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if not m or m.group(1) != h.hexdigest():
        return None
    for line in text.splitlines():
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 6 and cells[0] == kernel:
            return float(cells[4])
    return None


def copy_probe():
    """A plain copy kernel of known size: 2 GiB read, 2 GiB written, 5 times."""
    import torch
    n = 2 ** 29
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 5}))


def cpu_baseline(w, seconds):
    """FP64 oracle on a 64^3 window of the same workload (centred on the
    droplet's leading edge, noise keyed by the full box), stepped until about
    `seconds` of CPU work has elapsed."""
    import oracle as O
    box = w.box
    n = 64
    c = [int(v) for v in w.centres[0]]
    off = (c[0] + int(w.radii[0]) - n // 2, c[1] - n // 2, c[2] - n // 2)
    sl = [np.arange(o, o + n) % N for o, N in zip(off, (box.nx, box.ny, box.nz))]
    idx = np.ix_(sl[2], sl[1], sl[0])
    rr = w.rho_r[idx].astype(np.float64)
    rb = w.rho_b[idx].astype(np.float64)
    u = np.stack([w.u[a][idx] for a in range(3)]).astype(np.float64)
    P = O.Params(nx=n, ny=n, nz=n, rho0_r=box.rho0_r, rho0_b=box.rho0_b, alpha_r=box.alpha_r,
                 alpha_b=box.alpha_b, nu_r=box.nu_r, nu_b=box.nu_b, sigma=box.sigma,
                 beta=box.beta, omega=(1.0, 1.0, box.omega_bulk) + (1.0,) * 8)
    f = O.init_window(P, rr, rb, u, (box.nx, box.ny, box.nz), off, seed=w.seed, amp=w.noise)
    steps, t0 = 0, time.perf_counter()
    while True:
        O.step(P, f, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    return {"value": n ** 3 * steps / el / 1e6, "unit": "MLUPS", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": "%d steps of a 64^3 window of the %dx%dx%d workload (FP64, plain "
                      "definitions), %.1f s" % (steps, box.nx, box.ny, box.nz, el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2309_07801_amd as pkg
    import workloads as WL

    if args.copy_probe:
        copy_probe()
        return
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.size
    w = WL.translating_droplet(n=n, R=32.0 * n / 256.0)
    box = w.box
    sim = pkg.Simulation([pkg.box_params_of(box)], [w.rho_r], [w.rho_b], [w.u], seed=w.seed,
                         noise=w.noise)
    fluid = box.fluid_nodes()
    d0 = sim.reduce()[0]
    sim.step(2)
    if args.variant >= 0:
        sim.set_variant(args.variant)
        tune_ms = []
    else:
        tune_ms = sim.autotune(reps=5)
    variant = pkg.variant_info(sim.variant())
    sim.step(args.warmup)
    torch.cuda.synchronize()

    sim.profile_begin(4 * args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_end()
    dt = t1 - t0
    mlups = fluid * args.steps / dt / 1e6

    d1 = sim.reduce()[0]
    kern = {}
    for k, (ms, cnt) in prof.items():
        if cnt:
            avg = ms / cnt / 1e3
            kern[k] = {"avg_ms": avg * 1e3, "gbs": KERNEL_BYTES[k] * fluid / avg / 1e9,
                       "share": ms / 1e3 / dt}
    dom = max(kern, key=lambda k: kern[k]["share"])
    achieved = kern[dom]["gbs"]
    if dom == "fused":
        kname = "k_fused<%d, %d, %d, %d, false, f32>" % (variant["tx"], variant["ty"], variant["zc"],
                                                        variant["min_waves"])
    else:
        kname = "k_%s<f32>" % dom
    traffic = measured_traffic(kname) if n == 256 else None
    line = {
        "metric": "MLUPS and % HBM roofline, FP32 vs FP16-storage vs batched, at fixed error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "translating droplet %d^3 periodic, density ratio 10, R=%g, "
                               "u=0.05, FP32 storage" % (n, w.radii[0]),
                   "nodes": fluid, "storage": "fp32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_unit": "bytes per launch",
                     "algorithmic_bytes": KERNEL_BYTES[dom] * fluid, "kernel": kname,
                     "bytes_per_node": KERNEL_BYTES[dom]},
        "step_roofline_frac": round(mlups * 1e6 * STEP_BYTES / (HBM_PEAK_GBS * 1e9), 4),
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kern.items()},
        "fused_variant": variant,
        "autotune_ms": [round(m, 4) for m in tune_ms],
        "mass_drift": [float((d1[0] - d0[0]) / d0[0]), float((d1[1] - d0[1]) / d0[1])],
        "nonfinite": int(d1[12]),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
