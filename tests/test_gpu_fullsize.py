"""Parity at the full benchmark sizes, on sampled nodes.

One step's update of a node depends on the stored state within a distance
of 4 nodes (1 for the pull, 3 for the phase-field, normal, curvature and
correction stencils), so after k steps a node of the full box equals the
centre of an oracle window of edge W > 8k + 1 that starts from the same
state (noise keyed by the node index of the full box).  The HIP path runs
the full box in the launch geometry the benchmark uses (autotuned); the
oracle computes a 20^3 window around every sampled node.  Near solid walls
the window starts at the wall layer and carries the same wall flag; its far
layer is then solid as well, at more than 8 nodes from the sample.

Samples: nodes on the initial interface (distance to a droplet centre within
1.5 of its radius), nodes inside and outside the droplets, and (walled box)
nodes next to the walls.  Errors follow the survey's normalisation: density
relative to the oracle's density at the node, velocity relative to
U_ref = max(U, sigma / mu_max) (the capillary velocity scale bounds the
spurious and transient currents; at density ratio 1000 it is 24 lattice
units), phase field absolute.  Bars: FP32 storage 2e-5 (as for the small
boxes after a few steps); FP16 / BF16 storage the same bars as the small-box
storage tests."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as WL

from _common import FP32_BAR, bars_16bit, oracle_params

pytestmark = pytest.mark.gpu

STEPS = 2
W = 20          # window edge
HALF = 10       # sample position inside the window along an open axis
FIELDS = ("rho_r", "rho_b", "phi", "ux", "uy", "uz")
# per storage: (density relative, velocity / U_ref, phi absolute)
BARS = {0: (FP32_BAR,) * 3, 1: bars_16bit(1), 2: bars_16bit(2)}


def _gpu_run(w, storage, steps, schedule=None):
    import torch
    import paper_2309_07801_amd as pkg
    sim = pkg.Simulation([pkg.box_params_of(w.box)], [w.rho_r], [w.rho_b], [w.u], seed=w.seed,
                         noise=w.noise, storage=storage)
    sim.autotune(reps=1)
    if schedule is not None:
        sim.set_schedule(schedule)
    sim.step(steps)
    torch.cuda.synchronize()
    return sim


def _sample_values(sim, nodes):
    import torch
    out = {}
    idx = torch.as_tensor(np.asarray(nodes, dtype=np.int64))
    for name in FIELDS:
        f = sim.moments(0, (name,))[name].reshape(-1)
        out[name] = f[idx.to(f.device)].double().cpu().numpy()
        del f
    torch.cuda.synchronize()
    return out


def _window(w, sample, wall_axes):
    """Oracle fields at `sample` (x, y, z) after STEPS steps, from a W^3
    window; wall_axes: bit0 the window starts at the y wall, bit1 at z."""
    box = w.box
    pos, idx = [], []
    for a, (c, n) in enumerate(zip(sample, (box.nx, box.ny, box.nz))):
        at_wall = (a == 1 and wall_axes & 1) or (a == 2 and wall_axes & 2)
        o = 0 if at_wall else c - HALF
        pos.append(c - o)
        idx.append(np.mod(o + np.arange(W), n))
    sub = np.ix_(idx[2], idx[1], idx[0])
    wbox = dataclasses.replace(box, nx=W, ny=W, nz=W, walls=wall_axes)
    P = oracle_params(wbox)
    f = O.init_window(P, w.rho_r[sub], w.rho_b[sub], w.u[(slice(None),) + sub],
                      (box.nx, box.ny, box.nz), (int(idx[0][0]), int(idx[1][0]), int(idx[2][0])),
                      seed=w.seed, amp=w.noise)
    O.step(P, f, STEPS)
    F = O.fields(P, f)
    x, y, z = pos
    return {k: float(F[k][z, y, x]) for k in FIELDS}


def _samples(w, rng, n_iface=6, n_in=2, n_out=2, wall_margin=HALF + 1):
    """Interface, inside and outside nodes away from solid walls."""
    box = w.box
    lo = [0, wall_margin if box.walls & 1 else 0, wall_margin if box.walls & 2 else 0]
    hi = [box.nx, box.ny - wall_margin if box.walls & 1 else box.ny,
          box.nz - wall_margin if box.walls & 2 else box.nz]
    out = []
    for c, r in zip(w.centres, w.radii):
        for kind, count, dr in (("iface", n_iface, (-1.5, 1.5)), ("in", n_in, (-0.8 * r, -0.3 * r)),
                                ("out", n_out, (0.5 * r, 1.5 * r))):
            got = 0
            while got < count:
                d = rng.normal(size=3)
                d /= np.linalg.norm(d)
                rad = r + rng.uniform(*dr)
                p = [int(round(c[a] + rad * d[a])) for a in range(3)]
                p[0] %= box.nx
                if not (box.walls & 1):
                    p[1] %= box.ny
                if not (box.walls & 2):
                    p[2] %= box.nz
                if all(lo[a] <= p[a] < hi[a] for a in range(3)):
                    out.append((tuple(p), 0))
                    got += 1
    return out


def _u_ref(box, U):
    mu_max = max(box.rho0_r * box.nu_r, box.rho0_b * box.nu_b)
    return max(U, box.sigma / mu_max)


def _check(w, storage, samples, U, schedule=None):
    sim = _gpu_run(w, storage, STEPS, schedule)
    box = w.box
    u_ref = _u_ref(box, U)
    nodes = [x + box.nx * (y + box.ny * z) for (x, y, z), _ in samples]
    g = _sample_values(sim, nodes)
    sim.close()
    br, bu, bp = BARS[storage]
    worst = {"rho": 0.0, "u": 0.0, "phi": 0.0}
    for k, (p, wall_axes) in enumerate(samples):
        o = _window(w, p, wall_axes)
        rho_o = o["rho_r"] + o["rho_b"]
        e_rho = abs(g["rho_r"][k] + g["rho_b"][k] - rho_o) / rho_o
        e_u = np.sqrt(sum((g[c][k] - o[c]) ** 2 for c in ("ux", "uy", "uz"))) / u_ref
        e_phi = abs(g["phi"][k] - o["phi"])
        worst = {"rho": max(worst["rho"], e_rho), "u": max(worst["u"], e_u),
                 "phi": max(worst["phi"], e_phi)}
        assert e_rho <= br and e_u <= bu and e_phi <= bp, (p, wall_axes, e_rho, e_u, e_phi)
    print(box.nx, box.ny, box.nz, "storage", storage, "samples", len(samples), "u_ref", u_ref, worst)
    import torch
    torch.cuda.empty_cache()


def test_translating_droplet_256_sampled():
    w = WL.translating_droplet()
    rng = np.random.Generator(np.random.PCG64(21))
    _check(w, 0, _samples(w, rng), 0.05)


def test_translating_droplet_256_sampled_compact_schedule():
    """The same workload in the compact schedule (two steps in one call: the
    population pull, the compact pull, the emission back to populations)."""
    w = WL.translating_droplet()
    rng = np.random.Generator(np.random.PCG64(21))
    _check(w, 0, _samples(w, rng), 0.05, schedule=2)


@pytest.fixture(scope="module")
def sheared_512():
    return WL.sheared_droplets()


@pytest.mark.parametrize("storage", [0, 1, 2])
def test_sheared_droplets_512_sampled(sheared_512, storage):
    w = sheared_512
    rng = np.random.Generator(np.random.PCG64(22))
    _check(w, storage, _samples(w, rng, n_iface=2, n_in=1, n_out=1), 0.04)


@pytest.mark.parametrize("storage,schedule", [(0, None), (1, None), (0, 2)])
def test_head_on_collision_768_sampled(storage, schedule):
    """Walls in y and z; the compact schedule's wall stashes included."""
    w = WL.head_on_collision()
    box = w.box
    rng = np.random.Generator(np.random.PCG64(23))
    samples = _samples(w, rng, n_iface=4, n_in=1, n_out=1)
    # next to the walls: first fluid layers of y, of z, and of both
    for wall_axes, (y, z) in ((1, (1, 190)), (1, (2, 100)), (2, (190, 1)), (3, (1, 1)), (3, (2, 3))):
        samples.append(((int(rng.integers(0, box.nx)), y, z), wall_axes))
    _check(w, storage, samples, 0.1, schedule=schedule)


@pytest.mark.parametrize("schedule", [None, 2])
def test_batched_96_boxes_sampled(schedule):
    """The 96-box batch as the benchmark runs it (FP32 colour-pair storage,
    autotuned geometry, 44.9 M nodes; the autotuner's schedule and the
    compact schedule): after 2 steps, nodes of six boxes (the smallest and
    the largest among them) on the droplet interface and inside and outside
    it, against 20^3 oracle windows of the same box."""
    import torch
    import paper_2309_07801_amd as pkg
    ws = WL.batched_boxes()
    sim = pkg.Simulation([pkg.box_params_of(w.box) for w in ws], [w.rho_r for w in ws],
                         [w.rho_b for w in ws], [w.u for w in ws], seed=ws[0].seed,
                         noise=ws[0].noise, storage=pkg.FP32_PAIRS)
    sim.autotune(reps=1)
    if schedule is not None:
        sim.set_schedule(schedule)
    sim.step(STEPS)
    torch.cuda.synchronize()
    sizes = [w.box.nodes for w in ws]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 31, 58, 90})
    rng = np.random.Generator(np.random.PCG64(24))
    worst = {"rho": 0.0, "u": 0.0, "phi": 0.0}
    for k in picks:
        w = ws[k]
        box = w.box
        samples = _samples(w, rng, n_iface=2, n_in=1, n_out=1)
        nodes = [x + box.nx * (y + box.ny * z) for (x, y, z), _ in samples]
        idx = torch.as_tensor(np.asarray(nodes, dtype=np.int64))
        g = {}
        for name in FIELDS:
            f = sim.moments(k, (name,))[name].reshape(-1)
            g[name] = f[idx.to(f.device)].double().cpu().numpy()
        # the droplets start at rest and move by spurious currents only;
        # sigma / mu_max (up to 1.8 here) would make the velocity bar loose,
        # so velocities are compared on a fixed 0.01 scale
        u_ref = 0.01
        for j, (p, _) in enumerate(samples):
            pos, sl = [], []
            for c, n in zip(p, (box.nx, box.ny, box.nz)):
                pos.append(HALF)
                sl.append(np.mod(c - HALF + np.arange(W), n))
            sub = np.ix_(sl[2], sl[1], sl[0])
            wbox = dataclasses.replace(box, nx=W, ny=W, nz=W)
            P = oracle_params(wbox)
            f = O.init_window(P, w.rho_r[sub], w.rho_b[sub], w.u[(slice(None),) + sub],
                              (box.nx, box.ny, box.nz), (int(sl[0][0]), int(sl[1][0]), int(sl[2][0])),
                              seed=w.seed, amp=w.noise, box=k)
            O.step(P, f, STEPS)
            F = O.fields(P, f)
            o = {n: float(F[n][HALF, HALF, HALF]) for n in FIELDS}
            rho_o = o["rho_r"] + o["rho_b"]
            e_rho = abs(g["rho_r"][j] + g["rho_b"][j] - rho_o) / rho_o
            e_u = np.sqrt(sum((g[c][j] - o[c]) ** 2 for c in ("ux", "uy", "uz"))) / u_ref
            e_phi = abs(g["phi"][j] - o["phi"])
            worst = {"rho": max(worst["rho"], e_rho), "u": max(worst["u"], e_u),
                     "phi": max(worst["phi"], e_phi)}
            assert e_rho <= 2e-5 and e_u <= 2e-5 and e_phi <= 2e-5, (k, p, e_rho, e_u, e_phi)
    sim.close()
    print("batch of", len(ws), "boxes, samples from", picks, worst)
    torch.cuda.empty_cache()
