"""The two-dimensional model of App. A (D2Q9 lattice, generalized equilibrium
of Eq. A10) on the GPU, against the FP64 oracle of the same model.

* every exported field after 0 and 1 steps, for each tile shape of the step
  kernel, on a ragged box that spans several tiles;
* 200 steps of a translating droplet (periodic and between walls);
* a batch of boxes of unlike sizes, including boxes narrower than a tile
  and a one-column layered channel;
* the full-size throughput case (4096^2, 256 droplets) on sampled nodes
  against oracle windows;
* Table II: the stationary droplet's surface tension from Laplace's law
  (Eq. 68) for the eight printed density ratios and tensions;
* the mass-exact storage formats (FP32 exact, FP16 / BF16 shifted) against
  the oracle, their per-colour mass conservation, and bitwise agreement of
  the tile shapes in every format.
Bars as for the D3Q27 path: FP32 arithmetic against FP64."""
import dataclasses
import json
import os

import numpy as np
import pytest

import workloads as WL
from oracle import d2q9 as O2

from _common import (FP32_BAR, bars_16bit, check, errors, gpu_fields, oracle_params_2d,
                     run_oracle_2d, u_ref)

pytestmark = pytest.mark.gpu

FIELDS = ("rho_r", "rho_b", "phi", "p", "ux", "uy", "Fx", "Fy", "Qx", "Qy")
HERE = os.path.dirname(os.path.abspath(__file__))


def _box(shape, gamma=10.0, sigma=0.01, nu=0.1, visc_ratio=1.0, walls=0, beta=0.7, **kw):
    return WL.Box(nx=shape[0], ny=shape[1], nz=1, rho0_r=gamma, rho0_b=1.0,
                  alpha_r=WL.alpha_heavy_2d(gamma), alpha_b=WL.ALPHA_LIGHT_2D, nu_r=nu,
                  nu_b=nu / visc_ratio, sigma=sigma, beta=beta, walls=walls, **kw)


def _droplet(box, R, u=(0.04, -0.02, 0.0)):
    c = ((box.nx - 1) / 2.0, (box.ny - 1) / 2.0, 0.0)
    return WL.droplet_fields(box, [c], [R], u_carrier=u)


def _sim(boxes, fields, seed=0, noise=0.0, storage=0):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(b) for b in boxes], [f[0] for f in fields],
                          [f[1] for f in fields], [f[2] for f in fields], seed=seed, noise=noise,
                          storage=storage, lattice="d2q9")


@pytest.mark.parametrize("variant", range(4))
@pytest.mark.parametrize("steps", [0, 1])
def test_fields_match_oracle(variant, steps):
    box = _box((77, 45), visc_ratio=3.0)
    fl = _droplet(box, 11.5)
    sim = _sim([box], [fl], seed=5, noise=1e-5)
    sim.set_variant(variant)
    assert sim.variant() == variant
    sim.step(steps)
    g = gpu_fields(sim)
    sim.close()
    o, _ = run_oracle_2d(box, *fl, steps, seed=5, noise=1e-5)
    for name in FIELDS:
        scale = max(np.abs(o[name]).max(), 1e-30)
        err = np.abs(g[name] - o[name]).max()
        assert err <= 2e-5 * scale + 1e-12, (name, err, scale)
    # curvature and normal where the interface is resolved (their FP32 error
    # grows like eps / |grad phi|)
    gphi = np.hypot(*(np.roll(o["phi"], -1, a) - np.roll(o["phi"], 1, a) for a in (2, 1))) / 2
    band = gphi > 0.05
    for name in ("kappa", "nx", "ny"):
        scale = np.abs(o[name]).max()
        assert np.abs(g[name] - o[name])[band].max() <= 2e-5 * scale, name
    assert np.all(g["uz"] == 0) and np.all(g["Fz"] == 0) and np.all(g["Qz"] == 0)


@pytest.mark.parametrize("walls", [0, 1])
def test_translating_droplet_200_steps(walls):
    box = _box((70, 41), gamma=3.0, sigma=0.005, nu=0.05, visc_ratio=2.0, walls=walls)
    fl = _droplet(box, 10.0, u=(0.05, 0.0, 0.0))
    sim = _sim([box], [fl], seed=9, noise=1e-6)
    sim.step(200)
    g = gpu_fields(sim)
    d = sim.reduce()
    sim.close()
    o, _ = run_oracle_2d(box, *fl, 200, seed=9, noise=1e-6)
    e = errors(g, o, box, u_ref(box, 0.05))
    print(walls, e)
    check(e)
    assert d[0, 12] == 0


def test_batch_of_unlike_boxes():
    """Boxes smaller than a tile, a one-column channel between walls and a
    box of several tiles, advanced together; each against the oracle run
    alone (noise keyed by the box index)."""
    w, _ = WL.layered_channel("A", a=6, b=12)   # Table III's rest fractions
    lay = w.box
    cases = [
        (_box((5, 3), gamma=2.0), None),
        (_box((130, 70), gamma=10.0, visc_ratio=5.0), 14.0),
        (lay, "layered"),
        (_box((33, 17), gamma=1.0, sigma=0.02, walls=1), 5.0),
    ]
    boxes, fields = [], []
    for b, R in cases:
        if R == "layered":
            fields.append((w.rho_r, w.rho_b, w.u))
        elif R is None:
            rr = np.full(b.shape, b.rho0_r, np.float32)
            fields.append((rr, np.zeros(b.shape, np.float32), np.zeros((3,) + b.shape, np.float32)))
        else:
            fields.append(_droplet(b, R))
        boxes.append(b)
    sim = _sim(boxes, fields, seed=3, noise=1e-6)
    sim.step(60)
    for k, (b, fl) in enumerate(zip(boxes, fields)):
        o, _ = run_oracle_2d(b, *fl, 60, seed=3, noise=1e-6, box_index=k)
        e = errors(gpu_fields(sim, k), o, b, u_ref(b, 0.05))
        print(k, e)
        check(e, k)
    sim.close()


def test_graph_replays_match_direct_launches():
    box = _box((96, 50))
    fl = _droplet(box, 12.0)
    out = []
    for graph in (True, False):
        sim = _sim([box], [fl], seed=1, noise=1e-5)
        sim.set_graph(graph)
        sim.step(7)
        out.append(gpu_fields(sim))
        sim.close()
    for name in FIELDS:
        assert np.array_equal(out[0][name], out[1][name]), name


def test_fullsize_droplets_4096_sampled():
    """The throughput case (4096^2, 16 x 16 droplets of R = 48, density ratio
    10, carried at U = 0.05) after 2 autotuned steps, on nodes at the
    interfaces and inside and outside droplets, against the oracle on
    20^2 windows (a step's update depends on the state within 4 nodes)."""
    import torch
    import paper_2309_07801_amd as pkg
    w = WL.droplets_2d()
    box = w.box
    sim = pkg.Simulation([pkg.box_params_of(box)], [w.rho_r], [w.rho_b], [w.u], seed=w.seed,
                         noise=w.noise, lattice="d2q9")
    sim.autotune(reps=1)
    sim.step(2)
    rng = np.random.Generator(np.random.PCG64(31))
    samples = []
    for c, r in zip(w.centres[::17], w.radii[::17]):
        for dr in (-1.0, 0.0, 1.0, -0.6 * r, 0.5 * r):
            a = rng.uniform(0, 2 * np.pi)
            samples.append((int(round(c[0] + (r + dr) * np.cos(a))) % box.nx,
                            int(round(c[1] + (r + dr) * np.sin(a))) % box.ny))
    idx = torch.as_tensor([x + box.nx * y for x, y in samples])
    g = {}
    for name in ("rho_r", "rho_b", "phi", "ux", "uy"):
        f = sim.moments(0, (name,))[name].reshape(-1)
        g[name] = f[idx.to(f.device)].double().cpu().numpy()
    sim.close()
    W, H = 20, 10
    wbox = dataclasses.replace(box, nx=W, ny=W)
    P = oracle_params_2d(wbox)
    worst = {"rho": 0.0, "u": 0.0, "phi": 0.0}
    for k, (x, y) in enumerate(samples):
        ix = np.mod(x - H + np.arange(W), box.nx)
        iy = np.mod(y - H + np.arange(W), box.ny)
        sub = np.ix_([0], iy, ix)
        f = O2.init_window(P, w.rho_r[sub][0], w.rho_b[sub][0], w.u[(slice(0, 2),) + sub][:, 0],
                           (box.nx, box.ny), (int(ix[0]), int(iy[0])), seed=w.seed, amp=w.noise)
        O2.step(P, f, 2)
        F = O2.fields(P, f)
        rho_o = F["rho_r"][H, H] + F["rho_b"][H, H]
        e_rho = abs(g["rho_r"][k] + g["rho_b"][k] - rho_o) / rho_o
        e_u = np.hypot(g["ux"][k] - F["ux"][H, H], g["uy"][k] - F["uy"][H, H]) / 0.05
        e_phi = abs(g["phi"][k] - F["phi"][H, H])
        worst = {"rho": max(worst["rho"], e_rho), "u": max(worst["u"], e_u),
                 "phi": max(worst["phi"], e_phi)}
        assert e_rho <= 2e-5 and e_u <= 2e-5 and e_phi <= 2e-5, ((x, y), e_rho, e_u, e_phi)
    print(len(samples), "samples", worst)


def test_table_ii_surface_tension():
    """Table II: sigma_cal = R dp (Eq. 68) of the stationary droplet for the
    eight printed cases, all in one batch of 100^2 boxes, after 20000 steps.
    R and dp as measured by the diagnostics (R_eff = (A/pi)^(1/2), p_in
    over |x - c| < R_eff - 3, p_out over |x - c| > R_eff + 5).  The paper
    reports errors of 0.1-0.9 %; the unprinted parameters it takes from its
    reference (rest fractions, beta, run length) are ours here.  Every case
    is held to 1 % (measured: 0.16-0.88 %, the density ratio 1000 case
    0.88 % against the paper's 0.89 %).  FP32 storage: each colour's mass
    drifts by FP32 rounding of the collision, below 5e-4 over the run."""
    rows = json.load(open(os.path.join(HERE, "golden", "table2_stationary_droplet_2d.json")))["rows"]
    ws = [WL.stationary_droplet_2d(gamma=float(g), sigma=float(s)) for g, s, _, _ in rows]
    sim = _sim([w.box for w in ws], [(w.rho_r, w.rho_b, w.u) for w in ws])
    d0 = sim.reduce(centres=[w.centres[0] for w in ws])
    sim.step(ws[0].steps)
    d = sim.reduce(centres=[w.centres[0] for w in ws])
    sim.close()
    assert np.all(d[:, 12] == 0)
    res = []
    for k, ((g, s_th, s_paper, e_paper), w) in enumerate(zip(rows, ws)):
        s_cal = d[k, 7] * (d[k, 5] - d[k, 6])
        e = abs(s_cal - s_th) / s_th * 100
        drift = max(abs(d[k, c] - d0[k, c]) / d0[k, c] for c in (0, 1))
        print("gamma %6g sigma_th %.4f sigma_cal %.5f E %.2f %%  (paper %.5f, %.2f %%)  "
              "mass drift %.1e" % (g, s_th, s_cal, e, s_paper, e_paper, drift))
        res.append((g, e, drift))
    for g, e, drift in res:
        assert e < 1.0, (g, e)
        assert drift <= 5e-4, (g, drift)


def test_reduce_matches_oracle_fields():
    """FP64 diagnostics of a D2Q9 box: colour masses, momentum, R_eff =
    (A/pi)^(1/2) with A = sum (1 + phi)/2, the Laplace pressures over the
    bands |x - c| < R_eff - 3 and > R_eff + 5, and the red centroid, against
    the same sums over the oracle's fields."""
    box = _box((61, 47), gamma=5.0, sigma=0.02)
    c = (30.0, 23.0, 0.0)
    fl = WL.droplet_fields(box, [c], [12.0], u_carrier=(0.03, 0.01, 0.0))
    sim = _sim([box], [fl], seed=2, noise=1e-6)
    sim.step(20)
    d = sim.reduce(centres=[c])[0]
    sim.close()
    o, _ = run_oracle_2d(box, *fl, 20, seed=2, noise=1e-6)
    rho = o["rho_r"] + o["rho_b"]
    assert d[0] == pytest.approx(o["rho_r"].sum(), rel=1e-6)
    assert d[1] == pytest.approx(o["rho_b"].sum(), rel=1e-6)
    jx, jy = (rho * o["ux"]).sum(), (rho * o["uy"]).sum()
    print("momentum", d[2], jx, abs(d[2] - jx) / abs(jx), d[3], jy, abs(d[3] - jy) / abs(jy))
    assert d[2] == pytest.approx(jx, rel=1e-6)
    assert d[3] == pytest.approx(jy, rel=1e-6)
    assert d[4] == 0
    A = ((1 + o["phi"]) / 2).sum()
    reff = np.sqrt(A / np.pi)
    assert d[7] == pytest.approx(reff, rel=1e-6)
    dist = WL.periodic_distance((box.nx, box.ny, 1), c)
    p = o["p"]
    assert d[5] == pytest.approx(p[dist < reff - 3].mean(), rel=1e-5)
    assert d[6] == pytest.approx(p[dist > reff + 5].mean(), rel=1e-5)
    assert d[12] == 0


# (e_rho, e_u, e_phi) bars after 50 steps, as for D3Q27: FP32 1e-5, 16-bit
# formats from their unit roundoff (bars_16bit)
def _storage_bars(storage):
    return (FP32_BAR,) * 3 if storage == 3 else bars_16bit(storage)


@pytest.mark.parametrize("storage", [3, 1, 2])
@pytest.mark.parametrize("walls", [0, 1])
def test_storage_parity_with_oracle(storage, walls):
    """The mass-exact formats (FP32 exact, FP16 and BF16 shifted by the D2Q9
    pure-phase rest equilibrium) against the FP64 oracle after 50 steps of a
    translating droplet on a ragged box of several tiles."""
    box = _box((77, 45), gamma=10.0, visc_ratio=3.0, walls=walls)
    fl = _droplet(box, 11.5, u=(0.02, -0.01, 0.0))
    sim = _sim([box], [fl], seed=3, noise=1e-6, storage=storage)
    sim.step(50)
    g = gpu_fields(sim)
    sim.close()
    o, _ = run_oracle_2d(box, *fl, 50, seed=3, noise=1e-6)
    e = errors(g, o, box, u_ref(box, 0.02))
    print("storage", storage, "walls", walls, e)
    br, bu, bp = _storage_bars(storage)
    check(e, rho=br, u=bu, phi=bp)


@pytest.mark.parametrize("storage", [3, 1, 2])
def test_mass_exact_storage_conserves_colour_mass(storage):
    """Per-colour mass over 200 steps of a droplet carried by a uniform flow
    at density ratio 10 stays at FP64 rounding level (FP32 storage drifts by
    its rounding of the collision)."""
    box = _box((72, 48), gamma=10.0)
    fl = _droplet(box, 12.0, u=(0.05, 0.0, 0.0))
    sim = _sim([box], [fl], seed=5, noise=1e-6, storage=storage)
    d0 = sim.reduce()[0]
    sim.step(200)
    d1 = sim.reduce()[0]
    sim.close()
    drift = [(d1[k] - d0[k]) / d0[k] for k in (0, 1)]
    print("storage", storage, "mass drift", drift)
    assert abs(drift[0]) < 1e-12 and abs(drift[1]) < 1e-12
    assert d1[12] == 0


@pytest.mark.parametrize("storage", [4, 1, 2, 3])
def test_storage_variants_agree_bitwise(storage):
    """Every tile shape gives the same bits in every storage format (FP32
    pairs bitwise equal to FP32 as well), on a two-box batch with walls."""
    cases = [(_box((77, 45), walls=1), 11.5), (_box((30, 21)), 6.0)]
    boxes = [b for b, _ in cases]
    fields = [_droplet(b, R) for b, R in cases]
    ref = None
    if storage == 4:
        sim = _sim(boxes, fields, seed=8, noise=1e-6, storage=0)
        sim.step(12)
        ref = [gpu_fields(sim, k) for k in range(2)]
        sim.close()
    for v in range(4):
        sim = _sim(boxes, fields, seed=8, noise=1e-6, storage=storage)
        sim.set_variant(v)
        sim.step(12)
        out = [gpu_fields(sim, k) for k in range(2)]
        sim.close()
        if ref is None:
            ref = out
        for a, b in zip(ref, out):
            for name in a:
                assert np.array_equal(a[name], b[name]), (storage, v, name)
