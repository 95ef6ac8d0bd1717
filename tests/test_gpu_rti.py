"""Rayleigh-Taylor instability (Sec. IV.E): the buoyancy force
-(rho - rho_ref) g with walls at the bottom and top.

* parity with the FP64 oracle on an 8 x 8 x 32 box (Re = 64) for Models D
  and A over 100 steps, bars as for the translating droplet, and for
  Model D in the compact schedule as the benchmark runs it (walls through
  its wall stashes);
* the single-mode instability grows: at W = 32, Re = 1024, by T = 3
  (T = t (g/W)^(1/2)) the heavy spike has risen and the light bubble fallen
  by more than 0.7 W each (Model D);
* inviscid stability (nu = 0): Model D stays finite through T = 4 while
  Model C breaks down, as the paper reports for its Re = infinity runs."""

import numpy as np
import pytest

import workloads as WL

from _common import check, errors, fluid_mask, gpu_fields, run_oracle, u_ref

pytestmark = pytest.mark.gpu


def _sim(w):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(w.box)], [w.rho_r], [w.rho_b], [w.u], seed=w.seed,
                          noise=w.noise)


@pytest.mark.parametrize("model,schedule", [(3, None), (0, None), (3, 2)])
def test_rti_matches_oracle(model, schedule):
    w = WL.rayleigh_taylor(W=8, Re=64.0, model=model)
    sim = _sim(w)
    if schedule is not None:
        sim.set_schedule(schedule)
    sim.step(100)
    g = gpu_fields(sim)
    sim.close()
    o, _ = run_oracle(w.box, w.rho_r, w.rho_b, w.u, 100)
    e = errors(g, o, w.box, u_ref(w.box, 0.04))
    print(model, e)
    check(e)
    # the buoyancy force is in the exported F (no interfacial tension here)
    rho = o["rho_r"] + o["rho_b"]
    m = fluid_mask(w.box)
    assert np.allclose(o["Fz"][m], (-(rho - w.box.rho_ref) * w.box.gravity[2])[m],
                       rtol=1e-12, atol=1e-15)
    assert np.abs(g["Fz"] - o["Fz"])[m].max() <= 2e-5 * np.abs(o["Fz"]).max()


def _run(W, Re, model, T_list):
    w = WL.rayleigh_taylor(W=W, Re=Re, model=model)
    g = -w.box.gravity[2]
    tu = np.sqrt(W / g)
    sim = _sim(w)
    out, done = {}, 0
    for T in T_list:
        n = int(round(T * tu))
        sim.step(n - done)
        done = n
        phi = sim.moments(0, ("phi",))["phi"].double().cpu().numpy()
        if sim.reduce()[0, 12] > 0 or not np.isfinite(phi).all():
            out[T] = None
            break
        out[T] = (WL.interface_height(phi, 0, 0) / W, WL.interface_height(phi, W // 2, W // 2) / W)
    sim.close()
    return out


def test_rti_single_mode_grows():
    W = 32
    z0 = (4 * W - 1) / 2.0 / W
    r = _run(W, 1024.0, 3, [1.0, 2.0, 3.0])
    print(r)
    spike, bubble = r[3.0]
    assert spike - z0 > 0.7 and z0 - bubble > 0.7
    assert r[1.0][0] < r[2.0][0] < spike and r[1.0][1] > r[2.0][1] > bubble


def test_rti_inviscid_stability_model_d_not_c():
    d = _run(32, None, 3, [1.0, 2.0, 3.0, 4.0])
    c = _run(32, None, 2, [1.0, 2.0, 3.0, 4.0])
    print("D", d, "C", c)
    assert all(v is not None for v in d.values()) and len(d) == 4
    assert any(v is None for v in c.values())
