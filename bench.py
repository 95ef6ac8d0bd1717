"""Benchmark of the colour-gradient LBM hot path on one MI355X.

Main line (`value`): the translating-droplet case -- 256^3 periodic box, red
droplet of radius 32 moving with u = 0.05 along x in a blue carrier, density
ratio 10, equal dynamic viscosities, shear rate 1.6 and bulk rate 1.0,
sigma = 0.005, beta = 0.7, +-1e-6 counter noise on the populations, FP32
storage and arithmetic.  A step is one full time update of every node
(pull-streaming, moments, interface stencils, collision, recolouring).  The
FP32 lines run the compact schedule (the state between the steps of a call
held as each node's 17-value post-collision state); `--schedule 0` runs the
population schedule.  The K timed steps are one cglbm_step call as the
library runs it by default (replays of its captured two-step graph), timed
between two device synchronizations; `repeats` times four more such calls
and reports the median; one more call of K steps launches every kernel
directly between HIP events for the per-kernel times (`kernels`, the
roofline) and `events_mlups`.

Prints ONE JSON line: MLUPS of the timed steps, the roofline of the dominant
kernel (against HBM: algorithmic bytes per launch / average launch time from
the HIP events; against the FP32 vector issue rate: the committed
SQ_INSTS_VALU count per launch x 64 lanes / the same time; reported against
the closer ceiling) and the FP64 CPU oracle timed on a bounded sample of the
same workload (all host threads and one thread, with the host's CPU model).

`forms` reports, beside the main line:
  * the population schedule and the other storage formats on the same
    workload (FP16 / BF16 with the constant or the colour-fraction-scaled
    shift, FP32 mass-exact), each with its difference to the FP32 run after
    the same steps and its per-colour mass drift after 5000 steps;
  * the 512^3 density-ratio-1000 droplets (c3) in FP32, FP16 and BF16 with
    either shift, and the walled 768x384x384 head-on collision (c5) in FP32
    and FP16, at their own sizes;
  * the 96-box batch, the 32^3 static droplet, the in-place layout, the
    Rayleigh-Taylor case at the paper's size (Models D and A), the
    translating droplet's deformation per equilibrium model, the D2Q9 model
    of App. A on a 4096^2 droplet field (FP32, FP16, BF16) and Table II;
  * `parity`: for every configuration a reduced-size run against the FP64
    oracle on the same seeded inputs (e_rho, e_u, e_phi max and L2, with the
    bar each format is held to and pass / fail).
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
REPEATS = 5         # calls of K timed steps (the first is `value`)
DRIFT_STEPS = 5000  # steps after which the C2 forms report per-colour mass drift
BIG_STEPS = 500     # timed steps of each format at the 512^3 and 768x384x384 sizes
STORAGES = {"fp32": 0, "fp16": 1, "bf16": 2, "fp32x": 3, "fp32p": 4, "fp16c": 5, "bf16c": 6}
DTYPE = {"fp32": "f32", "fp16": "f16 storage, f32 arithmetic", "bf16": "bf16 storage, f32 arithmetic",
         "fp32x": "f32", "fp32p": "f32", "fp16c": "f16 storage, f32 arithmetic",
         "bf16c": "bf16 storage, f32 arithmetic"}
SIXTEEN = ("fp16", "bf16", "fp16c", "bf16c")
# unit roundoff of each storage format (round to nearest even)
UNIT_ROUNDOFF = {"fp32": 2.0 ** -24, "fp32p": 2.0 ** -24, "fp32x": 2.0 ** -24,
                 "fp16": 2.0 ** -11, "fp16c": 2.0 ** -11, "bf16": 2.0 ** -8, "bf16c": 2.0 ** -8}


def kernel_bytes(storage: str):
    """Algorithmic bytes per node of each kernel: what it must read and write."""
    if storage in ("fp32", "fp32p"):
        pops, aux_rho = 54 * 4, 0
    else:
        s = 4 if storage == "fp32x" else 2
        pops, aux_rho = 52 * s + 2 * 8, 2 * 8      # moving populations + FP64 rest
        if storage in ("fp16c", "bf16c"):
            pops += 2                              # the node's stored colour fraction
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
# call the population pull starts it and the emission (17 in, 54 out) ends it.
# With the mass-exact FP32 storage the compact state adds the two FP64 colour
# densities (read by the pull for the node's own rest closure and written by
# the fused kernel), and the pull writes them beside the 11 moments.
COMPACT_BYTES_X = {"pull": 17 * 4 + 2 * 8 + 11 * 4 + 2 * 8, "fused": 11 * 4 + 2 * 8 + 17 * 4 + 2 * 8,
                   "pull_first": 52 * 4 + 2 * 8 + 11 * 4 + 2 * 8, "emit": 17 * 4 + 2 * 8 + 52 * 4 + 2 * 8}
COMPACT_BYTES = {"pull": 17 * 4 + 11 * 4, "fused": 11 * 4 + 17 * 4,
                 "pull_first": 54 * 4 + 11 * 4, "emit": 17 * 4 + 54 * 4}



def compact_bytes(storage: str):
    """Algorithmic bytes per node of the compact schedule's kernels.  The
    mass-exact and 16-bit formats carry FP64 colour densities in the compact
    state and the moments; the 16-bit ones decode (pull_first) and encode
    (emit) their own populations: 26 pairs of 16-bit values, the FP64 rest
    populations and, with the colour-fraction shift, a 16-bit fraction."""
    if storage in ("fp32", "fp32p"):
        return COMPACT_BYTES
    if storage == "fp32x":
        return COMPACT_BYTES_X
    pops = 26 * 2 * 2 + 2 * 8 + (2 if storage in ("fp16c", "bf16c") else 0)
    return dict(COMPACT_BYTES_X, pull_first=pops + 11 * 4 + 2 * 8, emit=17 * 4 + 2 * 8 + pops)


# storage format of the D2Q9 step kernel's template argument
SNAMES = {"fp32": "StoreF32P", "fp32p": "StoreF32P", "fp16": "StoreF16", "bf16": "StoreBF16",
          "fp32x": "StoreF32X"}


def step_bytes(storage: str) -> int:
    """The whole step's algorithmic bytes: every population read and written
    once, 2 * 54 * (bytes per stored population)."""
    return 2 * 54 * (2 if storage in SIXTEEN else 4)


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


DEFAULT_FORMS = ("fp32_population,fp16,bf16,fp16c,bf16c,fp16c_population,fp32x,fp32x_population,"
                 "c3,c5,batched,"
                 "inplace,small,rti,galilean,d2q9,d2q9_fp16,d2q9_bf16,table2,parity")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256, help="box edge (default 256)")
    ap.add_argument("--workload", default="droplet", choices=("droplet", "batched", "collision"),
                    help="main line's workload: the translating droplet (default), the 96-box "
                         "batch (FP32 pairs) or the 768x384x384 walled collision; the other two "
                         "serve profiling runs of those kernels")
    ap.add_argument("--storage", default="fp32", choices=sorted(STORAGES))
    ap.add_argument("--forms", default=DEFAULT_FORMS, help="extra forms ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-resident", action="store_true",
                    help="compact schedule: store the populations at the end of every call")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--schedule", type=int, default=None, choices=(0, 1, 2),
                    help="step schedule (default: the autotuner's choice)")
    ap.add_argument("--variant", type=int, default=-1,
                    help="fused launch geometry (default: autotune)")
    ap.add_argument("--copy-probe-check", action="store_true",
                    help="run only a 256 MiB copy and a 2 GiB fill (counter calibration check: also a fill and a sum of 2 GiB)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 2 GiB device copy (counter calibration)")
    return ap.parse_args()


def copy_probe(check=False):
    """A plain copy kernel of known size: 2 GiB read, 2 GiB written, 5 times
    (the calibration of the HBM counters).  check: a copy of 256 MiB, a fill
    of 2 GiB and a sum over 2 GiB, 5 times each, to check that the
    calibration scales with the size and holds for kernels that only write
    or only read."""
    import torch
    n = 2 ** 26 if check else 2 ** 29
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    out = {"copy_probe_bytes_each_way": n * 4, "launches": 5}
    if check:
        c = torch.empty(2 ** 29, dtype=torch.float32, device="cuda")
        for _ in range(5):
            c.fill_(2.0)
        for _ in range(5):
            c.sum()
        out["fill_bytes_written"] = out["sum_bytes_read"] = c.numel() * 4
    torch.cuda.synchronize()
    print(json.dumps(out))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_params(box):
    import oracle as O
    return O.Params(nx=box.nx, ny=box.ny, nz=box.nz, rho0_r=box.rho0_r, rho0_b=box.rho0_b,
                    alpha_r=box.alpha_r, alpha_b=box.alpha_b, nu_r=box.nu_r, nu_b=box.nu_b,
                    sigma=box.sigma, beta=box.beta, walls=box.walls,
                    body_force=tuple(box.body_force), model=box.model, use_q=box.use_q,
                    gravity=tuple(box.gravity), rho_ref=box.rho_ref,
                    omega=(box.omega_hi[0], 1.0, box.omega_bulk) + tuple(box.omega_hi[1:]))


def _window_rate(w, n, seconds, max_steps):
    """Oracle MLUPS on an n^3 window of workload w (noise keyed by the full
    box), stepped until about `seconds` of CPU work has elapsed."""
    import oracle as O
    box = w.box
    c = [int(v) for v in w.centres[0]]
    off = (c[0] + int(w.radii[0]) - n // 2, c[1] - n // 2, c[2] - n // 2)
    sl = [np.arange(o, o + n) % N for o, N in zip(off, (box.nx, box.ny, box.nz))]
    idx = np.ix_(sl[2], sl[1], sl[0])
    rr = w.rho_r[idx].astype(np.float64)
    rb = w.rho_b[idx].astype(np.float64)
    u = np.stack([w.u[a][idx] for a in range(3)]).astype(np.float64)
    import dataclasses
    P = _oracle_params(dataclasses.replace(box, nx=n, ny=n, nz=n))
    f = O.init_window(P, rr, rb, u, (box.nx, box.ny, box.nz), off, seed=w.seed, amp=w.noise)
    steps, t0 = 0, time.perf_counter()
    while True:
        O.step(P, f, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= max_steps:
            break
    return n ** 3 * steps / el / 1e6, steps, el


def cpu_baseline(w, seconds):
    """FP64 oracle on a 64^3 window of the main workload (centred on the
    droplet's leading edge, noise keyed by the full box): all host threads
    for about `seconds`, one thread for about a third of that; and the full
    32^3 static droplet of 200 steps on all threads."""
    import oracle as O
    threads = O.num_threads()
    v, steps, el = _window_rate(w, 64, seconds, 200)
    O.set_num_threads(1)
    v1, steps1, el1 = _window_rate(w, 64, seconds / 3.0, 50)
    O.set_num_threads(threads)
    s = WL.static_droplet()
    P = _oracle_params(s.box)
    f = O.init(P, s.rho_r.astype(np.float64), s.rho_b.astype(np.float64), s.u.astype(np.float64))
    t0 = time.perf_counter()
    O.step(P, f, s.steps)
    el_c1 = time.perf_counter() - t0
    box = w.box
    return {"value": v, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": "%d steps of a 64^3 window of the %dx%dx%d workload (FP64, plain "
                      "definitions), %.1f s on %d threads" % (steps, box.nx, box.ny, box.nz, el,
                                                              threads),
            "cpu_model": cpu_model(),
            "one_thread": {"value": v1, "unit": "MLUPS", "steps": steps1, "seconds": round(el1, 2)},
            "static_droplet_32_full": {"steps": s.steps, "seconds": round(el_c1, 3),
                                       "mlups": s.box.nodes * s.steps / el_c1 / 1e6,
                                       "threads": threads}}


def _time_steps(sim, steps):
    import torch
    sim.profile_begin(8 * steps + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, sim.profile_end()


def run_form(workloads, storage, steps, warmup, variant=-1, keep_fields=None,
             lattice="d3q27", inplace=False, schedule=None, repeats=1, drift_steps=0,
             resident=False):
    """Initialise, autotune, time `steps` steps (and `repeats - 1` more calls
    of as many); return throughput, per-kernel event timings, the per-colour
    mass drift, and (keep_fields "host" or "device") the fields of box 0
    after the timed steps."""
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
    wmode = sim.wall_mode() if lattice == "d3q27" else None
    # compact schedule: keep the compact state resident between calls (the
    # populations are stored when the state is read)
    resident = bool(resident) and sim.schedule() == 2
    sim.set_resident(resident)
    sim.step(max(warmup - 2, 0))  # also captures the step graph
    torch.cuda.synchronize()
    # timed region: `repeats` calls of K steps as the library runs them by
    # default (replays of the captured two-step graph)
    mlups, out_fields, dt = [], None, None
    for rep in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        dtr = time.perf_counter() - t0
        mlups.append(fluid * steps / dtr / 1e6)
        if rep == 0:
            dt = dtr
            if keep_fields:
                names = ("rho_r", "rho_b", "phi", "ux", "uy", "uz")
                f = sim.moments(0, names)
                out_fields = {k: (v.clone() if keep_fields == "device" else v.cpu().numpy())
                              for k, v in f.items()}
                del f
    # one more call of K steps with every kernel launched directly between
    # HIP events: the per-kernel times
    dte, prof = _time_steps(sim, steps)
    events_mlups = fluid * steps / dte / 1e6
    done = 2 + max(warmup - 2, 0) + steps * repeats + steps
    d1 = sim.reduce()
    drift_out = None
    if drift_steps > done:
        sim.step(drift_steps - done)
        d2 = sim.reduce()
        m0, m2 = d0[:, :2].sum(axis=0), d2[:, :2].sum(axis=0)
        drift_out = {"steps": drift_steps,
                     "red": float((m2[0] - m0[0]) / m0[0]), "blue": float((m2[1] - m0[1]) / m0[1]),
                     "nonfinite": int(d2[:, 12].sum())}
    if lattice != "d3q27":
        kb = {"fused": d2q9_bytes(storage)}
    elif sim.schedule() == 2:
        kb = compact_bytes(storage)
    else:
        kb = kernel_bytes(storage)
    kern = {}
    for k, (ms, cnt) in prof.items():
        if cnt:
            avg = ms / cnt / 1e3
            kern[k] = {"avg_ms": avg * 1e3, "gbs": kb[k] * fluid / avg / 1e9 if k in kb else None,
                       "launches": cnt, "share": ms / 1e3 / dte}
    nonres = None
    if resident:
        # the same K steps as one call that pulls the stored populations
        # first and stores them again at its end
        sim.set_resident(False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        nonres = fluid * steps / (time.perf_counter() - t0) / 1e6
    m0 = d0[:, :2].sum(axis=0)
    m1 = d1[:, :2].sum(axis=0)
    out = {"mlups": mlups[0], "resident": resident, "nonresident_mlups": nonres, "mlups_repeats": mlups, "mlups_median": float(np.median(mlups)),
           "ms_per_step": dt / steps * 1e3, "dt": dt, "events_mlups": events_mlups,
           "fluid": fluid, "kernels": kern, "variant": var, "autotune_ms": tune_ms,
           "schedule": ("fused", "three kernels", "compact")[sim.schedule()],
           "mass_drift": [float((m1[0] - m0[0]) / m0[0]), float((m1[1] - m0[1]) / m0[1])],
           "mass_drift_steps": done, "mass_drift_long": drift_out,
           "nonfinite": int(d1[:, 12].sum()), "steps": steps,
           "pop_buffer_bytes": sim.pop_a.numel() * (1 if inplace else 2), "compact_variant": cvar,
           "wall_mode": wmode, "fields": out_fields}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def _kern_round(kern):
    return {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
            for k, v in kern.items()}


def proxy_errors(g, ref, u_ref):
    """Difference of a run to the FP32 run after the same steps (the survey's
    proxy for full-size runs the oracle cannot afford); fields as numpy
    arrays or device tensors."""
    def np_(x):
        return x.double().cpu().numpy() if hasattr(x, "cpu") else np.asarray(x, np.float64)
    if hasattr(g["rho_r"], "cpu"):
        # device tensors: norms on the device, in FP64
        rho_g = (g["rho_r"].double() + g["rho_b"].double())
        rho_f = (ref["rho_r"].double() + ref["rho_b"].double())
        fluid = rho_f > 0  # solid wall nodes hold zero moments
        rel = ((rho_g - rho_f).abs() / rho_f)[fluid]
        du = ((g["ux"].double() - ref["ux"].double()) ** 2 + (g["uy"].double() - ref["uy"].double()) ** 2
              + (g["uz"].double() - ref["uz"].double()) ** 2).sqrt()[fluid]
        return {"e_rho": float(rel.max()), "e_u": float(du.max() / u_ref),
                "e_phi": float((g["phi"].double() - ref["phi"].double()).abs()[fluid].max()),
                "e_rho_l2": float((rel ** 2).mean().sqrt()),
                "e_u_l2": float((du ** 2).mean().sqrt() / u_ref)}
    g = {k: np_(v) for k, v in g.items()}
    ref = {k: np_(v) for k, v in ref.items()}
    rho_g, rho_f = g["rho_r"] + g["rho_b"], ref["rho_r"] + ref["rho_b"]
    m = rho_f > 0  # solid wall nodes hold zero moments
    du = np.sqrt((g["ux"] - ref["ux"]) ** 2 + (g["uy"] - ref["uy"]) ** 2 + (g["uz"] - ref["uz"]) ** 2)[m]
    rel = (np.abs(rho_g - rho_f)[m] / rho_f[m])
    return {"e_rho": float(rel.max()),
            "e_u": float(du.max() / u_ref), "e_phi": float(np.abs(g["phi"] - ref["phi"])[m].max()),
            "e_rho_l2": float(np.sqrt((rel ** 2).mean())),
            "e_u_l2": float(np.sqrt((du ** 2).mean()) / u_ref)}


def storage_form(r, storage, ref_fields=None, u_ref=None):
    """One storage form's throughput line."""
    sbf = step_bytes(storage)
    out = {"storage": storage, "mlups": round(r["mlups"], 1),
           "mlups_median": round(r["mlups_median"], 1), "ms_per_step": round(r["ms_per_step"], 4),
           "events_mlups": round(r["events_mlups"], 1), "schedule": r["schedule"],
           "resident": r["resident"],
           "wall_mode": r["wall_mode"],
           "step_roofline_frac": round(r["mlups"] * 1e6 * sbf / (HBM_PEAK_GBS * 1e9), 4),
           "step_bytes_per_node": sbf, "kernels": _kern_round(r["kernels"]),
           "mass_drift": r["mass_drift"], "mass_drift_steps": r["mass_drift_steps"],
           "nonfinite": r["nonfinite"]}
    if r["mass_drift_long"]:
        out["mass_drift_5000"] = r["mass_drift_long"]
    if ref_fields is not None and r["fields"] is not None:
        out["vs_fp32_after_same_steps"] = proxy_errors(r["fields"], ref_fields, u_ref)
    return out


def big_form(label, w, storages, steps, warmup, u_ref):
    """A configuration at its own size in several storage formats, each
    compared with the FP32 run after the same steps (on the device)."""
    import torch
    box = w.box
    out = {"workload": label, "nodes": box.fluid_nodes(), "steps": steps}
    ref = None
    for name in storages:
        # the compact schedule, or (a "_population" suffix) the population one
        st = name.split("_")[0]
        r = run_form([w], st, steps, warmup, keep_fields="device",
                     schedule=0 if name.endswith("_population") else 2, resident=name == "fp32")
        out[name] = storage_form(r, st, ref, u_ref)
        if name == "fp32":
            ref = r["fields"]
        else:
            del r["fields"]
        torch.cuda.empty_cache()
        print("bench:   %s %s %.1f MLUPS" % (label.split(",")[0], name, r["mlups"]), file=sys.stderr,
              flush=True)
    del ref
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
           "events_mlups": round(r["events_mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
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
            "wall_mode": sim.wall_mode(), "T_spike_bubble_saddle": hist, "nonfinite": int(d[0, 12])}
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


# ---------------------------------------------------------------------------
# Parity against the FP64 oracle at reduced sizes, one run per configuration
# ---------------------------------------------------------------------------

# FP32 storage: 1e-5, or 2 gamma 2^-24 at a density ratio gamma where that
# is larger (at a node of the light phase the heavy colour's FP32 values
# carry rounding of 2^-24 of the heavy density).  16-bit storage: the error
# its rounding alone produces is of the order of the unit roundoff u_s times
# the stored deviations; the bar is 8 u_s (e_rho, e_phi) and 32 u_s (e_u,
# which divides a momentum error by a velocity scale 10-25 times smaller
# than the populations), independent of the step count.
FP32_BAR = 1e-5


def format_bar(storage, gamma=1.0, steps=0, at_rest=False):
    """Bars of e_rho, e_u, e_phi.  Plain FP32 storage of a droplet at rest:
    e_rho and e_phi up to 4 N 2^-24 after N steps as well (its colour masses
    drift by rounding that repeats identically at every step of a steady
    state; the mass-exact format keeps to the bar above)."""
    if storage in ("fp32", "fp32p", "fp32x"):
        b = max(FP32_BAR, 2.0 * max(gamma, 1.0 / gamma) * 2.0 ** -24)
        br = max(b, 4.0 * steps * 2.0 ** -24) if (at_rest and storage != "fp32x") else b
        return {"rho": br, "u": b, "phi": br}
    us = UNIT_ROUNDOFF[storage]
    return {"rho": 8 * us, "u": 32 * us, "phi": 8 * us}


def _gpu_fields(ws, storage, steps, schedule, seed, noise):
    import torch
    import paper_2309_07801_amd as pkg
    sim = pkg.Simulation([pkg.box_params_of(w.box) for w in ws], [w.rho_r for w in ws],
                         [w.rho_b for w in ws], [w.u for w in ws], seed=seed, noise=noise,
                         storage=STORAGES[storage])
    if schedule is not None:
        sim.set_schedule(schedule)
    sim.step(steps)
    out = [{k: v.double().cpu().numpy() for k, v in sim.moments(b).items()} for b in range(len(ws))]
    torch.cuda.synchronize()
    sim.close()
    return out


def _a23_u_ref(box, U):
    """U_ref of e_u: the imposed velocity or the capillary scale sigma /
    mu_max, whichever is larger."""
    return max(U, box.sigma / max(box.rho0_r * box.nu_r, box.rho0_b * box.nu_b))


def _errors(g, o, box, U):
    m = np.ones(box.shape, bool)
    if box.walls & 1:
        m[:, 0, :] = m[:, -1, :] = False
    if box.walls & 2:
        m[0, :, :] = m[-1, :, :] = False
    rho_g, rho_o = g["rho_r"] + g["rho_b"], o["rho_r"] + o["rho_b"]
    rel = (np.abs(rho_g - rho_o) / rho_o)[m]
    du = np.sqrt((g["ux"] - o["ux"]) ** 2 + (g["uy"] - o["uy"]) ** 2 + (g["uz"] - o["uz"]) ** 2)[m]
    u_ref = _a23_u_ref(box, U)
    return {"e_rho": float(rel.max()), "e_u": float(du.max() / u_ref),
            "e_phi": float(np.abs(g["phi"] - o["phi"])[m].max()),
            "e_rho_l2": float(np.sqrt((rel ** 2).mean())), "e_u_l2": float(np.sqrt((du ** 2).mean()) / u_ref),
            "u_ref": u_ref, "e_u_vs_U": float(du.max() / U)}


def parity_form():
    """Every configuration at a reduced size against the FP64 oracle on the
    same seeded inputs: e_rho (relative to the oracle's density), e_u
    (relative to U_ref = max(U, sigma / mu_max); e_u_vs_U against the
    imposed velocity U alone), e_phi (absolute), max and L2 over fluid
    nodes.  The 16-bit formats run the population schedule (rounded to the
    format at every step) and, marked _compact, the compact schedule (one
    call: rounded when it stores the populations)."""
    import oracle as O
    cases = [
        ("c1", "32^3 static droplet (the configuration itself)", [WL.static_droplet()], 200, 0.01,
         (("fp32", 2), ("fp32", 0))),
        ("c2", "translating droplet at 64^3, R 8", [WL.translating_droplet(n=64, R=8.0)], 200, 0.05,
         (("fp32", 2), ("fp32", 0), ("fp32x", None), ("fp16", None), ("fp16c", None),
          ("fp16", 2), ("fp16c", 2))),
        ("c3", "density-ratio-1000 droplets at 96^3, R U[4, 9]",
         [WL.sheared_droplets(n=96, count=8, rmin=4.0, rmax=9.0)], 100, 0.04,
         (("fp32", 2), ("fp16", None), ("bf16", None), ("fp16c", None), ("bf16c", None),
          ("fp16c", 2), ("bf16c", 2))),
        ("c4", "the four smallest boxes of the 96-box batch",
         sorted(WL.batched_boxes(), key=lambda x: x.box.nodes)[:4], 200, 0.01,
         (("fp32p", 2),)),
        ("c5", "walled head-on collision at 192x96x96, R 12 (We, Re kept)",
         [WL.head_on_collision(nx=192, ny=96, nz=96, R=12.0)], 100, 0.05,
         (("fp32", 2), ("fp16", None), ("fp16c", None), ("fp16c", 2))),
    ]
    out = {}
    for key, label, ws, steps, u_ref, runs in cases:
        t0 = time.perf_counter()
        orc = []
        for b, w in enumerate(ws):
            P = _oracle_params(w.box)
            f = O.init(P, w.rho_r.astype(np.float64), w.rho_b.astype(np.float64),
                       w.u.astype(np.float64), seed=w.seed, amp=w.noise, box=b)
            O.step(P, f, steps)
            orc.append(O.fields(P, f))
        t_orc = time.perf_counter() - t0
        entry = {"workload": label, "steps": steps, "U": u_ref, "oracle_seconds": round(t_orc, 1)}
        for st, sched in runs:
            g = _gpu_fields(ws, st, steps, sched, ws[0].seed, ws[0].noise)
            errs = [_errors(gb, ob, w.box, u_ref) for gb, ob, w in zip(g, orc, ws)]
            e = {k: max(x[k] for x in errs) for k in errs[0] if k != "u_ref"}
            e["u_ref"] = [x["u_ref"] for x in errs]
            bar = format_bar(st, max(max(w.box.rho0_r / w.box.rho0_b, w.box.rho0_b / w.box.rho0_r)
                                     for w in ws), steps, at_rest=key in ("c1", "c4"))
            e["bar"] = bar
            e["status"] = "pass" if (e["e_rho"] <= bar["rho"] and e["e_u"] <= bar["u"]
                                     and e["e_phi"] <= bar["phi"]) else "fail"
            name = st + ("_" + ("population", "three_kernel", "compact")[sched] if sched is not None else "")
            entry[name] = e
        out[key] = entry
        print("bench:   parity %s done (oracle %.1f s)" % (key, t_orc), file=sys.stderr, flush=True)
    return out


def main():
    T0 = time.perf_counter()
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_probe or args.copy_probe_check:
        copy_probe(check=args.copy_probe_check)
        return
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.size
    w = WL.translating_droplet(n=n, R=32.0 * n / 256.0)
    main_ws, main_label = [w], None
    if args.workload == "batched":
        main_ws = WL.batched_boxes()
        args.storage = "fp32p"
        main_label = "96 periodic boxes, edges U{24..128}, density ratio in {1,10,100}, fp32p storage"
    elif args.workload == "collision":
        main_ws = [WL.head_on_collision()]
        main_label = "768x384x384 walled head-on collision, density ratio 10, %s storage" % args.storage
    forms_req = [f for f in args.forms.split(",") if f]
    sched = args.schedule
    if sched is None and args.storage in ("fp32", "fp32p"):
        sched = 2  # the compact schedule serves this periodic FP32 workload
    want_fields = any(f in STORAGES for f in forms_req)
    main_r = run_form(main_ws, args.storage, args.steps, args.warmup, args.variant,
                      keep_fields="device" if want_fields else None, schedule=sched,
                      repeats=REPEATS, drift_steps=DRIFT_STEPS if forms_req else 0,
                      resident=not args.no_resident and args.storage in ("fp32", "fp32p"))
    fluid = main_r["fluid"]
    compact = main_r["schedule"] == "compact"
    kern = {k: v for k, v in main_r["kernels"].items() if k in ("pull", "fused")}
    dom = max(kern, key=lambda k: kern[k]["share"])
    var = main_r["variant"]
    geo = (var["tx"], var["ty"], var["zc"], var["min_waves"])
    if compact:
        cv = main_r["compact_variant"]
        kname = {"pull": "k_cpull<%d, %d, %d, false, f32, false>" % (cv["tx"], cv["ty"], cv["zc"]),
                 "fused": "k_fused<%d, %d, %d, %d, false, f32, false, true>" % geo}[dom]
        kb = COMPACT_BYTES
    else:
        kname = ("k_fused<%d, %d, %d, %d, false, f32, false>" % geo if dom == "fused"
                 else "k_%s<f32%s>" % (dom, ", false, f32" if dom == "pull" else ""))
        kb = kernel_bytes(args.storage)
    measured = n == 256 and args.storage == "fp32" and args.workload == "droplet"
    traffic = measured_traffic(kname) if measured else None
    valu = measured_valu(kname) if measured else None
    sb = step_bytes(args.storage)
    hbm_frac = kern[dom]["gbs"] / HBM_PEAK_GBS
    roof = {"bound": "hbm", "achieved": round(kern[dom]["gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(hbm_frac, 4), "traffic": traffic,
            "traffic_unit": "bytes per launch", "algorithmic_bytes": kb[dom] * fluid, "kernel": kname,
            "launches_timed": kern[dom]["launches"]}
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
                    "kernel": kname, "launches_timed": kern[dom]["launches"]}
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
        "config": {"workload": main_label or ("translating droplet %d^3 periodic, density ratio "
                                              "10, R=%g, u=0.05, %s storage"
                                              % (n, w.radii[0], args.storage)),
                   "nodes": fluid, "storage": args.storage, "schedule": main_r["schedule"]},
        "roofline": roof,
        "step_roofline_frac": round(main_r["mlups"] * 1e6 * sb / (HBM_PEAK_GBS * 1e9), 4),
        "repeats": {"calls": REPEATS, "steps_each": args.steps,
                    "mlups": [round(v, 1) for v in main_r["mlups_repeats"]],
                    "median_mlups": round(main_r["mlups_median"], 1)},
        "events_mlups": round(main_r["events_mlups"], 1),
        "step_bytes_per_node": sb,
        "step_bytes_moved_per_node": (COMPACT_BYTES["pull"] + COMPACT_BYTES["fused"]) if compact
                                     else kernel_bytes(args.storage)["pull"] + kernel_bytes(args.storage)["fused"],
        "kernels": _kern_round(main_r["kernels"]),
        "fused_variant": var,
        "compact_variant": main_r["compact_variant"],
        "schedule": main_r["schedule"],
        "resident": main_r["resident"],
        "nonresident_mlups": (round(main_r["nonresident_mlups"], 1)
                              if main_r["nonresident_mlups"] else None),
        "autotune_ms": [round(m, 4) for m in main_r["autotune_ms"]],
        "mass_drift": main_r["mass_drift"],
        "mass_drift_steps": main_r["mass_drift_steps"],
        "nonfinite": main_r["nonfinite"],
    }
    if main_r["mass_drift_long"]:
        line["mass_drift_5000"] = main_r["mass_drift_long"]
    print("bench: main line %.1f MLUPS (%.1f s)" % (main_r["mlups"], time.perf_counter() - T0),
          file=sys.stderr, flush=True)
    forms = {}
    u_ref = 0.05
    ref_fields = main_r["fields"]
    for f in forms_req:
        if f in STORAGES:
            # every format runs the compact schedule (the mass-exact and
            # 16-bit ones with FP64 colour densities in the compact state;
            # the 16-bit populations are decoded and encoded at the ends of
            # each call)
            r = run_form([w], f, args.steps, args.warmup, args.variant, keep_fields="device",
                         drift_steps=DRIFT_STEPS, schedule=2)
            forms[f] = storage_form(r, f, ref_fields, u_ref)
            del r["fields"]
        elif f.endswith("_population") and f.split("_")[0] in STORAGES:
            # the population schedule: the stored format between every two
            # steps
            st = f.split("_")[0]
            sixteen = st in SIXTEEN
            r = run_form([w], st, args.steps, args.warmup, args.variant, schedule=0,
                         drift_steps=DRIFT_STEPS, keep_fields="device" if sixteen else None)
            forms[f] = storage_form(r, st, ref_fields if sixteen else None, u_ref)
            r.pop("fields", None)
        elif f == "c3":
            w3 = WL.sheared_droplets()
            forms["c3"] = big_form("512^3 periodic, 8 droplets R U[20,48], density ratio 1000, "
                                   "sinusoidal shear 0.04", w3, ("fp32", "fp16", "bf16", "fp16c",
                                                                 "bf16c"),
                                   min(args.steps, BIG_STEPS), args.warmup, 0.04)
            del w3
        elif f == "c5":
            w5 = WL.head_on_collision()
            forms["c5"] = big_form("768x384x384, walls y/z, head-on collision of two R 48 droplets, "
                                   "relative velocity 0.1, density ratio 10, Re 5000, We 50", w5,
                                   ("fp32", "fp16", "fp16c", "fp16c_population"),
                                   min(args.steps, BIG_STEPS),
                                   args.warmup, 0.05)
            del w5
        elif f == "batched":
            boxes = WL.batched_boxes()
            steps_b = min(args.steps, 1000)
            r = run_form(boxes, "fp32p", steps_b, args.warmup, args.variant, schedule=2,
                         resident=True)
            forms["batched"] = {"workload": "96 periodic boxes, edges U{24..128}, density ratio "
                                            "in {1,10,100}, FP32 (colour-pair layout), compact schedule",
                                "nodes": r["fluid"], "steps": steps_b, "mlups": round(r["mlups"], 1),
                                "mlups_median": round(r["mlups_median"], 1),
                                "resident": r["resident"],
                                "nonresident_mlups": round(r["nonresident_mlups"], 1),
                                "ms_per_step": round(r["ms_per_step"], 4),
                                "events_mlups": round(r["events_mlups"], 1),
                                "schedule": r["schedule"], "fused_variant": r["variant"],
                                "compact_variant": r["compact_variant"],
                                "step_roofline_frac": round(r["mlups"] * 1e6 * 432 / (HBM_PEAK_GBS * 1e9), 4),
                                "kernels": _kern_round(r["kernels"]),
                                "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"]}
        elif f == "inplace":
            r = run_form([w], args.storage, args.steps, args.warmup, args.variant, inplace=True)
            forms["inplace"] = {"workload": "the main line's workload with one population buffer",
                                "population_buffer_bytes": r["pop_buffer_bytes"],
                                "two_buffer_bytes": main_r["pop_buffer_bytes"],
                                "mlups": round(r["mlups"], 1),
                                "ms_per_step": round(r["ms_per_step"], 4),
                                "events_mlups": round(r["events_mlups"], 1),
                                "schedule": r["schedule"],
                                "kernels": _kern_round(r["kernels"]),
                                "mass_drift": r["mass_drift"], "nonfinite": r["nonfinite"]}
        elif f == "small":
            ws = WL.static_droplet()
            steps_s = min(args.steps, 2000)
            r = run_form([ws], "fp32", steps_s, args.warmup, args.variant)
            forms["small"] = {"workload": "static droplet 32^3 (density ratio 1, R=8), FP32",
                              "nodes": r["fluid"], "steps": steps_s,
                              "mlups": round(r["mlups"], 1),
                              "events_mlups": round(r["events_mlups"], 1),
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
        elif f == "parity":
            forms["parity"] = parity_form()
        print("bench: form %s done (%.1f s)" % (f, time.perf_counter() - T0), file=sys.stderr,
              flush=True)
    del ref_fields
    main_r["fields"] = None
    if "parity" in forms:
        # each storage form carries the oracle verdict of its format on the
        # reduced-size run of the same configuration
        par = forms["parity"]
        for key, st in (("fp16", "fp16"), ("bf16", "bf16"), ("fp16c", "fp16c"), ("bf16c", "bf16c"),
                        ("fp32x", "fp32x")):
            if key in forms:
                for cfg in ("c2", "c3"):
                    if st in par.get(cfg, {}):
                        forms[key]["oracle_parity_" + cfg] = {
                            k: par[cfg][st][k] for k in ("e_rho", "e_u", "e_phi", "status")}
        for cfg in ("c3", "c5"):
            for st in SIXTEEN + ("fp32",):
                name = st if st != "fp32" else "fp32_compact"
                if cfg in forms and st in forms[cfg] and name in par.get(cfg, {}):
                    forms[cfg][st]["oracle_parity"] = {
                        k: par[cfg][name][k] for k in ("e_rho", "e_u", "e_phi", "status")}
        line["parity_status"] = {cfg: {k: v["status"] for k, v in e.items() if isinstance(v, dict)}
                                 for cfg, e in par.items()}
    if forms:
        line["forms"] = forms
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        print("bench: cpu baseline done (%.1f s)" % (time.perf_counter() - T0), file=sys.stderr,
              flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
