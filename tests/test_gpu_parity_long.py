"""Long parity runs against the FP64 oracle after 1000 steps on the laminar
cases:

* P1: the 32^3 static droplet (density and viscosity ratio 1, sigma 0.01,
  beta 0.7, tau 1, R 8), after 200 and 1000 steps;
* P2: the translating-droplet physics (density ratio 10, shear rate 1.6,
  bulk rate 1, sigma 0.005, beta 0.7, u = 0.05 along x, +-1e-6 noise) at
  64^3 with R = 8, after 1000 steps;
* P4: the eight smallest boxes of the 96-box batch (density ratios 1, 10
  and 100, uneven extents, droplets at rest), run as one batch, after 1000
  steps.

Each case runs in the population schedule (0) and the compact schedule (2),
with plain FP32 storage and with the mass-exact FP32 storage (FP64 colour
densities and rest populations).  Error measures over fluid nodes:
e_rho = max |d rho| / rho_oracle, e_phi = max |d phi|, e_u = max |d u|_2 /
U_ref with U_ref = max(U, sigma / mu_max) (the imposed velocity or the
capillary velocity scale, whichever is larger); the log also holds e_u
against the imposed velocity alone (P2: 0.05) or 0.01 for the droplets at
rest.

Bars: the mass-exact storage meets 1e-5 for e_rho, e_u and e_phi on every
case and schedule, and so does plain FP32 storage on the moving droplet.
For droplets at rest, plain FP32 storage meets 1e-5 for e_u; its colour
masses drift by the FP32 rounding of the stored populations, which in a
steady state repeats the same way at every step, so e_rho and e_phi are held
to 4 N 2^-24 after N steps (2.4e-4 at 1000).  Measured values are written to
the JSON file named by CGLBM_PARITY_LOG, if set, before the checks."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as WL
from _common import errors, gpu_fields, oracle_params

pytestmark = pytest.mark.gpu

BAR = 1e-5
STEPS = 1000


def _bar_fp32_at_rest(steps):
    return 4.0 * steps * 2.0 ** -24


def _log(key, value):
    path = os.environ.get("CGLBM_PARITY_LOG")
    if not path:
        return
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = value
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def _oracle(box, rr, rb, u, checkpoints, seed=0, noise=0.0, box_index=0):
    P = oracle_params(box)
    f = O.init(P, np.asarray(rr, np.float64), np.asarray(rb, np.float64),
               np.asarray(u, np.float64), seed=seed, amp=noise, box=box_index)
    out, done = {}, 0
    for n in checkpoints:
        O.step(P, f, n - done)
        done = n
        out[n] = O.fields(P, f)
    return out


def _gpu(workloads, schedule, storage, checkpoints, seed=0, noise=0.0):
    """Fields of every box after each checkpoint (one cglbm_step call per
    stretch) and the per-colour mass drift over the run."""
    import paper_2309_07801_amd as pkg
    sim = pkg.Simulation([pkg.box_params_of(w.box) for w in workloads],
                         [w.rho_r for w in workloads], [w.rho_b for w in workloads],
                         [w.u for w in workloads], seed=seed, noise=noise, storage=storage)
    sim.set_schedule(schedule)
    assert sim.schedule() == schedule
    m0 = sim.reduce()[:, :2].copy()
    out, done = {}, 0
    for n in checkpoints:
        sim.step(n - done)
        done = n
        out[n] = [gpu_fields(sim, k) for k in range(len(workloads))]
    d = sim.reduce()
    drift = ((d[:, :2] - m0) / m0).tolist()
    assert d[:, 12].sum() == 0
    sim.close()
    return out, drift


_ORACLE = {}


def _cached(key, fn):
    if key not in _ORACLE:
        _ORACLE[key] = fn()
    return _ORACLE[key]


def _u_ref(box, U):
    return max(U, box.sigma / max(box.rho0_r * box.nu_r, box.rho0_b * box.nu_b))


def _check(name, g, o, box, U, U_strict, bar_rho_phi=BAR):
    e = errors(g, o, box, _u_ref(box, U))
    e["u_strict"] = errors(g, o, box, U_strict)["u"]
    print(name, e)
    _log(name, e)
    assert e["rho"] <= bar_rho_phi and e["u"] <= BAR and e["phi"] <= bar_rho_phi, (name, e)


# (schedule, storage): population and compact schedule, plain and mass-exact FP32
RUNS = [(0, 0), (2, 0), (0, 3), (2, 3)]
IDS = ["population", "compact", "population_exact", "compact_exact"]


@pytest.mark.parametrize("schedule,storage", RUNS, ids=IDS)
def test_p1_static_droplet_1000_steps(schedule, storage):
    w = WL.static_droplet()
    o = _cached("p1", lambda: _oracle(w.box, w.rho_r, w.rho_b, w.u, (200, STEPS)))
    g, drift = _gpu([w], schedule, storage, (200, STEPS))
    tag = "p1_sched%d_storage%d" % (schedule, storage)
    _log(tag + "_mass_drift", drift)
    for n in (200, STEPS):
        _check("%s_%d" % (tag, n), g[n][0], o[n], w.box, 0.0, 0.01,
               BAR if storage == 3 else _bar_fp32_at_rest(n))


@pytest.mark.parametrize("schedule,storage", RUNS, ids=IDS)
def test_p2_translating_droplet_64_cubed_1000_steps(schedule, storage):
    w = WL.translating_droplet(n=64, R=8.0)
    o = _cached("p2", lambda: _oracle(w.box, w.rho_r, w.rho_b, w.u, (STEPS,), seed=w.seed,
                                      noise=w.noise))
    g, drift = _gpu([w], schedule, storage, (STEPS,), seed=w.seed, noise=w.noise)
    tag = "p2_sched%d_storage%d" % (schedule, storage)
    _log(tag + "_mass_drift", drift)
    _check(tag, g[STEPS][0], o[STEPS], w.box, 0.05, 0.05)


def _p4_boxes():
    bs = WL.batched_boxes()
    order = sorted(range(len(bs)), key=lambda k: bs[k].box.nodes)[:8]
    return [bs[k] for k in order]


_P4_GPU = {}
P4_RUNS = [(0, 4), (2, 4), (0, 3), (2, 3)]


@pytest.mark.parametrize("k", range(8))
@pytest.mark.parametrize("schedule,storage", P4_RUNS, ids=IDS)
def test_p4_smallest_batched_boxes_1000_steps(schedule, storage, k):
    ws = _p4_boxes()
    if (schedule, storage) not in _P4_GPU:
        _P4_GPU[(schedule, storage)] = _gpu(ws, schedule, storage, (STEPS,))
    g, drift = _P4_GPU[(schedule, storage)]
    w = ws[k]
    o = _cached(("p4", k), lambda: _oracle(w.box, w.rho_r, w.rho_b, w.u, (STEPS,), box_index=k))
    tag = "p4_sched%d_storage%d_box%d" % (schedule, storage, k)
    _log(tag + "_mass_drift", drift[k])
    _check(tag, g[STEPS][k], o[STEPS], w.box, 0.0, 0.01,
           BAR if storage == 3 else _bar_fp32_at_rest(STEPS))
