"""Benchmark of the colour-gradient LBM hot path on one MI355X.

Default workload: the translating-droplet case -- 256^3 periodic box, red
droplet of radius 32 moving with u = 0.05 along x in a blue carrier, density
ratio 10, equal dynamic viscosities, shear rate 1.6 and bulk rate 1.0,
sigma = 0.005, beta = 0.7, +-1e-6 counter noise on the populations, FP32
storage and arithmetic.  A step is one full time update of every node
(pull-streaming, moments, interface stencils, collision, recolouring).  The
FP32 lines run the compact schedule (the state between the steps of a call
held as each node's 17-value post-collision state); `--schedule 0` runs the
population schedule.

Prints ONE JSON line: MLUPS of the timed steps, the roofline of the dominant
kernel (against HBM: algorithmic bytes per launch / average launch time from
HIP events recorded on the launch stream during the timed region; against
the FP32 vector issue rate: the committed SQ_INSTS_VALU count per launch x 64
lanes / the same time; reported against the closer ceiling) and the FP64 CPU
oracle timed on a bounded sample of the same workload.  `forms` reports, on
the same workload and step counts, the FP16/BF16-shifted and mass-exact FP32
storage (with their difference to the FP32 run as a proxy error), the
96-box batched workload, the 32^3 static droplet, the Rayleigh-Taylor case
at the paper's size (Models D and A), the translating droplet's
deformation per equilibrium model, the two-dimensional model of App. A on a
4096^2 droplet field (d2q9; d2q9_fp16 and d2q9_bf16 with 16-bit shifted
storage), the main workload in the in-place layout (inplace) and Table II's
surface tensions (table2).  The timed region
launches every kernel directly (HIP events around each launch); after it,
`graph_mlups` times the same update as replays of the captured two-step
graph that cglbm_step uses by default.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402  (seeded inputs; numpy only)

HBM_PEAK_GBS = 8000.0
GRAPH_STEPS = 500   # steps of the graph-replay run after the timed region
STORAGES = {"fp32": 0, "fp16": 1, "bf16": 2, "fp32x": 3, "fp32p": 4}
DTYPE = {"fp32": "f32", "fp16": "f16 storage, f32 arithmetic", "bf16": "bf16 storage, f32 arithmetic",
         "fp32x": "f32", "fp32p": "f32"}


def kernel_bytes(storage: str):
    """Algorithmic bytes per node of each kernel: what it must read and write."""
    if storage in ("fp32", "fp32p"):
        pops, aux_rho = 54 * 4, 0
    else:
        s = 4 if storage == "fp32x" else 2
        pops, aux_rho = 52 * s + 2 * 8, 2 * 8      # moving populations + FP64 rest
    return {
        "pull": pops + 11 * 4 + aux_rho,           # populations in, 11 local moments out
        "interface": (2 + 3) * 4 + 9 * 4,          # rho_r, rho_b, j in; n, F, Q out
        "collide": 20 * 4 + aux_rho + pops,        # moments + interface fields in, populations out
        "fused": 11 * 4 + aux_rho + pops,          # local moments in, populations out
    }


# D2Q9 step kernel (one launch per step): the stored populations read and
# written once per node (9 colour pairs of 2 x float; mass-exact formats: 8
# pairs and the two FP64 rest populations); every moment and interface field
# stays on chip.
def d2q9_bytes(storage: str) -> int:
    if storage in ("fp32", "fp32p"):
        return 2 * 9 * 8
    return 2 * (8 * (8 if storage == "fp32x" else 4) + 2 * 8)


# Compact schedule (FP32, periodic boxes): per node the pull reads the 17
# floats of the compact post-collision state and writes the 11 moments; the
# fused kernel reads the moments and writes the compact state; once per
# call the emission reads the compact state and stores the populations.
COMPACT_BYTES = {"pull": 17 * 4 + 11 * 4, "fused": 11 * 4 + 17 * 4, "collide": 17 * 4 + 54 * 4}

# storage format of the D2Q9 step kernel's template argument
SNAMES = {"fp32": "StoreF32P", "fp32p": "StoreF32P", "fp16": "StoreF16", "bf16": "StoreBF16",
          "fp32x": "StoreF32X"}


def step_bytes(storage: str) -> int:
    """The whole step's algorithmic bytes: every population read and written
    once, 2 * 54 * (bytes per stored population)."""
    return 2 * 54 * (2 if storage in ("fp16", "bf16") else 4)


COUNTERS = os.path.join(ROOT, "profiles", "step_kernels_translating_droplet_256_counters.md")
# FP32 vector issue peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# lane operations per second, unpacked (the 157.3 TFLOP/s figure counts an
# FMA as two operations and packed FP32 as two lanes)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
SOURCES = ("paper_2309_07801_amd/csrc/kernels.hpp", "paper_2309_07801_amd/csrc/lattice.hpp")


def _counter_rows():
    """Table rows of the committed rocprofv3 counter summary, or None if it
    is missing or the kernel sources changed since it was taken."""
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
    return [[c.strip() for c in line.strip().strip("|").split("|")] for line in text.splitlines()]


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` (FETCH_SIZE / WRITE_SIZE, scaled by
    the copy-kernel calibration), or None."""
    for cells in _counter_rows() or []:
        if len(cells) == 6 and cells[0] == kernel:
            return float(cells[4])
    return None


def measured_valu(kernel: str):
    """VALU wave64 instructions per dispatch of `kernel` (SQ_INSTS_VALU), or
    None."""
    for cells in _counter_rows() or []:
        if len(cells) == 4 and cells[0] == kernel:
            return float(cells[2])
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256, help="box edge (default 256)")
    ap.add_argument("--storage", default="fp32", choices=sorted(STORAGES))
    ap.add_argument("--forms", default="fp16,bf16,fp32x,batched,inplace,small,rti,galilean,d2q9,"
                    "d2q9_fp16,d2q9_bf16,table2",
                    help="extra forms on the same workload ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--schedule", type=int, default=None, choices=(0, 1, 2),
                    help="step schedule (default: the autotuner's choice)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="fused launch geometry (default: autotune)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy (counter calibration)")
    return ap.parse_args()


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


def run_form(workloads, storage, steps, warmup, variant=-1, keep_fields=False,
             lattice="d3q27", inplace=False, schedule=None):
    """Initialise, autotune, time `steps` steps; return throughput, per-kernel
    event timings and (optionally) the final fields of box 0."""
    import torch
    import paper_2309_07801_amd as pkg
    sim = pkg.Simulation([pkg.box_params_of(w.box) for w in workloads],
                         [w.rho_r for w in workloads], [w.rho_b for w in workloads],
                         [w.u for w in workloads], seed=workloads[0].seed,
                         noise=workloads[0].noise, storage=STORAGES[storage], lattice=lattice,
                         inplace=inplace)
    fluid = sum(w.box.fluid_nodes() for w in workloads)
    d0 = sim.reduce()
    sim.step(2)
    if variant >= 0:
        sim.set_variant(variant)
        tune_ms = []
    else:
        tune_ms = sim.autotune(reps=5)
    var = pkg.variant_info(sim.variant(), lattice)
    cvar = sim.compact_variant() if lattice == "d3q27" else None
    if schedule is not None:
        sim.set_schedule(schedule)  # loads the geometry the autotuner chose for it
        var = pkg.variant_info(sim.variant(), lattice)
    sim.step(max(warmup - 2, 0))  # also captures the step graph
    torch.cuda.synchronize()
    # timed region: direct launches with HIP events around every kernel
    sim.profile_begin(4 * steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile_end()
    dt = t1 - t0
    # the same update as replays of the captured two-step graph
    ngraph = min(steps, GRAPH_STEPS)
    t2 = time.perf_counter()
    sim.step(ngraph)
    torch.cuda.synchronize()
    graph_mlups = fluid * ngraph / (time.perf_counter() - t2) / 1e6
    d1 = sim.reduce()
    if lattice != "d3q27":
        kb = {"fused": d2q9_bytes(storage)}
    elif sim.schedule() == 2:
        kb = COMPACT_BYTES
    else:
        kb = kernel_bytes(storage)
    kern = {}
    for k, (ms, cnt) in prof.items():
        if cnt:
            avg = ms / cnt / 1e3
            kern[k] = {"avg_ms": avg * 1e3, "gbs": kb[k] * fluid / avg / 1e9, "share": ms / 1e3 / dt}
    m0 = d0[:, :2].sum(axis=0)
    m1 = d1[:, :2].sum(axis=0)
    out = {"mlups": fluid * steps / dt / 1e6, "ms_per_step": dt / steps * 1e3, "dt": dt,
           "graph_mlups": graph_mlups,
           "fluid": fluid, "kernels": kern, "variant": var, "autotune_ms": tune_ms,
           "schedule": ("fused", "three kernels", "compact")[sim.schedule()],
           "mass_drift": [float((m1[0] - m0[0]) / m0[0]), float((m1[1] - m0[1]) / m0[1])],
           "nonfinite": int(d1[:, 12].sum()), "steps": steps,
           "pop_buffer_bytes": sim.pop_a.numel() * (1 if inplace else 2), "compact_variant": cvar}
    if keep_fields:
        out["fields"] = {k: v.cpu().numpy() for k, v in
                         sim.moments(0, ("rho_r", "rho_b", "phi", "ux", "uy", "uz")).items()}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def d2q9_form(steps, warmup, storage="fp32"):
    """The two-dimensional model of App. A: throughput on a 4096^2 field of
    256 droplets (density ratio 10, carried at U = 0.05)."""
    w = WL.droplets_2d()
    r = run_form([w], storage, steps, warmup, lattice="d2q9")
    k = r["kernels"]["fused"]
    out = {"workload": "4096^2 periodic, 16 x 16 droplets R=48, density ratio 10, U=0.05, %s"
                       % storage.upper(),
           "nodes": r["fluid"], "steps": steps, "mlups": round(r["mlups"], 1),
           "graph_mlups": round(r["graph_mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
           "kernel": {"name": "k2_step<%s, %d, %d, 256, false>"
                              % (SNAMES[storage], r["variant"]["tx"], r["variant"]["ty"]),
                      "avg_ms": round(k["avg_ms"], 4), "gbs": round(k["gbs"], 1),
                      "algorithmic_bytes_per_node": d2q9_bytes(storage),
                      "frac": round(k["gbs"] / HBM_PEAK_GBS, 4)},
           "autotune_ms": [round(m, 4) for m in r["autotune_ms"]],
           "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"]}
    return out


def table2_form():
    """Table II's stationary droplets in two dimensions (eight 100^2 boxes in
    one batch, 20000 steps): the surface tension from Laplace's law
    (Eq. 68), sigma_cal = R_eff (p_in - p_out), and its error."""
    import paper_2309_07801_amd as pkg
    out = {}
    cases = ((1, 0.012), (1, 0.072), (1, 0.24), (2, 0.112), (10, 0.132), (30, 0.1116),
             (100, 0.10), (1000, 0.10))
    ws = [WL.stationary_droplet_2d(gamma=float(g), sigma=s) for g, s in cases]
    sim = pkg.Simulation([pkg.box_params_of(x.box) for x in ws], [x.rho_r for x in ws],
                         [x.rho_b for x in ws], [x.u for x in ws], lattice="d2q9")
    sim.step(ws[0].steps)
    d = sim.reduce(centres=[x.centres[0] for x in ws])
    sim.close()
    out["cases"] = [{"gamma": g, "sigma_th": s,
                        "sigma_cal": round(float(d[k, 7] * (d[k, 5] - d[k, 6])), 6),
                        "E_percent": round(float(abs(d[k, 7] * (d[k, 5] - d[k, 6]) - s) / s * 100), 3)}
                       for k, (g, s) in enumerate(cases)]
    return out


def rti_form(W=128, T_list=(1.0, 2.0, 3.0, 4.0)):
    """Single-mode Rayleigh-Taylor instability at the paper's size (W = 128,
    W x W x 4W, At = 0.5, Re = 1024), Models D and A: interface heights / W
    of the spike (x = y = 0), bubble (x = y = W/2) and saddle (x = 0,
    y = W/2) columns at T = t (g/W)^(1/2), and the throughput of the run."""
    import torch
    import paper_2309_07801_amd as pkg
    out = {"workload": "Rayleigh-Taylor %dx%dx%d, At 0.5, Re 1024, walls at z" % (W, W, 4 * W)}
    for model in (3, 0):
        w = WL.rayleigh_taylor(W=W, model=model)
        tu = np.sqrt(W / -w.box.gravity[2])
        sim = pkg.Simulation([pkg.box_params_of(w.box)], [w.rho_r], [w.rho_b], [w.u])
        sim.autotune(reps=2)
        sim.set_schedule(2)  # the compact schedule (walls, every equilibrium family)
        hist, done, t_run = [], 0, 0.0
        for T in T_list:
            n = int(round(T * tu))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step(n - done)
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t0
            done = n
            phi = sim.moments(0, ("phi",))["phi"].cpu().numpy()
            hist.append([T] + [round(WL.interface_height(phi, x, y) / W, 4)
                               for x, y in ((0, 0), (W // 2, W // 2), (0, W // 2))])
        d = sim.reduce()
        out["model_" + "ABCD"[model]] = {
            "mlups": round(w.box.fluid_nodes() * done / t_run / 1e6, 1), "steps": done,
            "schedule": ("fused", "three kernels", "compact")[sim.schedule()],
            "T_spike_bubble_saddle": hist, "nonfinite": int(d[0, 12])}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    return out


def galilean_form(steps=20000):
    """A droplet carried by a uniform flow U = 0.05 through a periodic
    64x48x48 box (density ratio 3, mu_r = mu_b = 0.075, sigma 4.4e-3,
    R = 12): deformation (l_max - l_min)/(l_max + l_min) of the inertia
    tensor of the red region after `steps` steps, per equilibrium model."""
    import dataclasses
    import paper_2309_07801_amd as pkg
    n, R, U, mu = (64, 48, 48), 12.0, 0.05, 0.075
    c = tuple((v - 1) / 2.0 for v in n)
    out = {"workload": "translating droplet 64x48x48, U 0.05, density ratio 3", "steps": steps}
    for model, q, label in ((0, 1, "A"), (1, 1, "B"), (2, 1, "C"), (3, 1, "D"), (3, 0, "D_without_Q")):
        box = dataclasses.replace(WL.two_phase_box(n, 3.0, 3.0, 1.0, 4.4e-3, 0.7), nu_r=mu / 3.0,
                                  nu_b=mu, model=model, use_q=q)
        rr, rb, u = WL.droplet_fields(box, [c], [R], u_carrier=(U, 0.0, 0.0))
        sim = pkg.Simulation([pkg.box_params_of(box)], [rr], [rb], [u])
        sim.step(steps)
        phi = sim.moments(0, ("phi",))["phi"].double().cpu().numpy()
        out[label] = round(deformation(phi), 4)
        sim.close()
    return out


def deformation(phi):
    """(l_max - l_min)/(l_max + l_min) of the inertia tensor of the red region
    (weights (1 + phi)/2) about its periodic centroid."""
    wgt = np.clip((1.0 + phi) / 2.0, 0.0, 1.0)
    coords = []
    for a, n in zip((2, 1, 0), (phi.shape[2], phi.shape[1], phi.shape[0])):
        shape = [1, 1, 1]
        shape[a] = n
        ang = 2.0 * np.pi * np.arange(n) / n
        cen = (np.arctan2((wgt * np.sin(ang).reshape(shape)).sum(),
                          (wgt * np.cos(ang).reshape(shape)).sum()) % (2.0 * np.pi)) * n / (2.0 * np.pi)
        d = (np.arange(n) - cen + n / 2.0) % n - n / 2.0
        coords.append(d.reshape(shape))
    M = np.array([[(wgt * ci * cj).sum() for cj in coords] for ci in coords])
    ev = np.linalg.eigvalsh(M)
    return float((ev[-1] - ev[0]) / (ev[-1] + ev[0]))


def proxy_errors(g, ref, u_ref):
    """Difference of a run to the FP32 run after the same steps (the survey's
    proxy for full-size runs the oracle cannot afford)."""
    rho_g, rho_f = g["rho_r"] + g["rho_b"], ref["rho_r"] + ref["rho_b"]
    du = np.sqrt((g["ux"] - ref["ux"]) ** 2 + (g["uy"] - ref["uy"]) ** 2 + (g["uz"] - ref["uz"]) ** 2)
    return {"e_rho": float((np.abs(rho_g - rho_f) / rho_f).max()),
            "e_u": float(du.max() / u_ref), "e_phi": float(np.abs(g["phi"] - ref["phi"]).max()),
            "e_rho_l2": float(np.sqrt((((rho_g - rho_f) / rho_f) ** 2).mean())),
            "e_u_l2": float(np.sqrt((du ** 2).mean()) / u_ref)}


def main():
    T0 = time.perf_counter()
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe:
        copy_probe()
        return
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.size
    w = WL.translating_droplet(n=n, R=32.0 * n / 256.0)
    forms_req = [f for f in args.forms.split(",") if f]
    sched = args.schedule
    if sched is None and args.storage in ("fp32", "fp32p"):
        sched = 2  # the compact schedule serves this periodic FP32 workload
    main_r = run_form([w], args.storage, args.steps, args.warmup, args.variant,
                      keep_fields=any(f in STORAGES for f in forms_req), schedule=sched)
    fluid = main_r["fluid"]
    kern = {k: v for k, v in main_r["kernels"].items() if k != "collide" or main_r["schedule"] != "compact"}
    dom = max(kern, key=lambda k: kern[k]["share"])
    var = main_r["variant"]
    compact = main_r["schedule"] == "compact"
    geo = (var["tx"], var["ty"], var["zc"], var["min_waves"])
    if compact:
        cv = main_r["compact_variant"]
        kname = {"pull": "k_cpull<%d, %d, %d, false, f32, false>" % (cv["tx"], cv["ty"], cv["zc"]),
                 "fused": "k_fused<%d, %d, %d, %d, false, f32, false, true>" % geo}[dom]
        kb = COMPACT_BYTES
    else:
        kname = ("k_fused<%d, %d, %d, %d, false, f32, false>" % geo if dom == "fused"
                 else "k_%s<f32%s>" % (dom, ", false" if dom == "pull" else ""))
        kb = kernel_bytes(args.storage)
    measured = n == 256 and args.storage == "fp32"
    traffic = measured_traffic(kname) if measured else None
    valu = measured_valu(kname) if measured else None
    sb = step_bytes(args.storage)
    hbm_frac = kern[dom]["gbs"] / HBM_PEAK_GBS
    roof = {"bound": "hbm", "achieved": round(kern[dom]["gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch", "algorithmic_bytes": kb[dom] * fluid, "kernel": kname}
    if valu is not None:
        # VALU issue rate of the dominant kernel: its counted wave64 VALU
        # instructions per launch x 64 lanes / the live mean launch time
        tops = valu * 64 / (kern[dom]["avg_ms"] * 1e-3) / 1e12
        if tops / VALU_PEAK_TOPS > hbm_frac:
            roof = {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
                    "unit": "TOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4),
                    "op_unit": "FP32 VALU lane operations issued (SQ_INSTS_VALU x 64)",
                    "traffic": traffic, "traffic_unit": "bytes per launch",
                    "hbm": {"achieved": round(kern[dom]["gbs"], 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(hbm_frac, 4),
                            "algorithmic_bytes": kb[dom] * fluid},
                    "kernel": kname}
        else:
            roof["valu_tops"] = round(tops, 2)
    line = {
        "metric": "MLUPS and % HBM roofline, FP32 vs FP16-storage vs batched, at fixed error",
        "value": round(main_r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": "translating droplet %d^3 periodic, density ratio 10, R=%g, "
                               "u=0.05, %s storage" % (n, w.radii[0], args.storage),
                   "nodes": fluid, "storage": args.storage, "schedule": main_r["schedule"]},
        "roofline": roof,
        "step_roofline_frac": round(main_r["mlups"] * 1e6 * sb / (HBM_PEAK_GBS * 1e9), 4),
        "graph_mlups": round(main_r["graph_mlups"], 1),
        "step_bytes_per_node": sb,
        "step_bytes_moved_per_node": (COMPACT_BYTES["pull"] + COMPACT_BYTES["fused"]) if compact
                                     else kernel_bytes(args.storage)["pull"] + kernel_bytes(args.storage)["fused"],
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                    for k, v in main_r["kernels"].items()},
        "fused_variant": var,
        "compact_variant": main_r["compact_variant"],
        "schedule": main_r["schedule"],
        "autotune_ms": [round(m, 4) for m in main_r["autotune_ms"]],
        "mass_drift": main_r["mass_drift"],
        "nonfinite": main_r["nonfinite"],
    }
    print("bench: main line %.1f MLUPS (%.1f s)" % (main_r["mlups"], time.perf_counter() - T0),
          file=sys.stderr, flush=True)
    forms = {}
    u_ref = 0.05
    for f in forms_req:
        if f in STORAGES:
            r = run_form([w], f, args.steps, args.warmup, args.variant, keep_fields=True)
            sbf = step_bytes(f)
            forms[f] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                        "graph_mlups": round(r["graph_mlups"], 1),
                        "schedule": r["schedule"],
                        "step_roofline_frac": round(r["mlups"] * 1e6 * sbf / (HBM_PEAK_GBS * 1e9), 4),
                        "step_bytes_per_node": sbf,
                        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                                    for k, v in r["kernels"].items()},
                        "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"],
                        "vs_fp32_after_same_steps": proxy_errors(r["fields"], main_r["fields"], u_ref)}
        elif f == "batched":
            boxes = WL.batched_boxes()
            steps_b = min(args.steps, 1000)
            r = run_form(boxes, "fp32p", steps_b, args.warmup, args.variant, schedule=2)
            forms["batched"] = {"workload": "96 periodic boxes, edges U{24..128}, density ratio "
                                            "in {1,10,100}, FP32 (colour-pair layout), compact schedule",
                                "nodes": r["fluid"],
                                "steps": steps_b, "mlups": round(r["mlups"], 1),
                                "ms_per_step": round(r["ms_per_step"], 4),
                                "graph_mlups": round(r["graph_mlups"], 1),
                                "schedule": r["schedule"],
                                "step_roofline_frac": round(r["mlups"] * 1e6 * 432 / (HBM_PEAK_GBS * 1e9), 4),
                                "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                                            for k, v in r["kernels"].items()},
                                "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"]}
        elif f == "inplace":
            r = run_form([w], args.storage, args.steps, args.warmup, args.variant, inplace=True)
            forms["inplace"] = {"workload": "the main line's workload with one population buffer",
                                "population_buffer_bytes": r["pop_buffer_bytes"],
                                "two_buffer_bytes": main_r["pop_buffer_bytes"],
                                "mlups": round(r["mlups"], 1),
                                "ms_per_step": round(r["ms_per_step"], 4),
                                "graph_mlups": round(r["graph_mlups"], 1),
                                "schedule": r["schedule"],
                                "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                                            for k, v in r["kernels"].items()},
                                "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"]}
        elif f == "small":
            ws = WL.static_droplet()
            steps_s = min(args.steps, 2000)
            r = run_form([ws], "fp32", steps_s, args.warmup, args.variant)
            forms["small"] = {"workload": "static droplet 32^3 (density ratio 1, R=8), FP32",
                              "nodes": r["fluid"], "steps": steps_s,
                              "mlups_direct_launches": round(r["mlups"], 1),
                              "graph_mlups": round(r["graph_mlups"], 1),
                              "schedule": r["schedule"],
                              "ms_per_step": round(r["ms_per_step"], 4),
                              "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"]}
        elif f == "rti":
            forms["rti"] = rti_form()
        elif f == "galilean":
            forms["galilean"] = galilean_form()
        elif f == "d2q9":
            forms["d2q9"] = d2q9_form(min(args.steps, 2000), args.warmup)
        elif f in ("d2q9_fp16", "d2q9_bf16"):
            forms[f] = d2q9_form(min(args.steps, 2000), args.warmup, f[5:])
        elif f == "table2":
            forms["table2"] = table2_form()
        print("bench: form %s done (%.1f s)" % (f, time.perf_counter() - T0), file=sys.stderr,
              flush=True)
    if forms:
        line["forms"] = forms
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        print("bench: cpu baseline done (%.1f s)" % (time.perf_counter() - T0), file=sys.stderr,
              flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
