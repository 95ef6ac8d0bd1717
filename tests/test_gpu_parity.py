"""Parity of the HIP path with the FP64 oracle on the same seeded inputs.

Tolerances: the HIP path computes in FP32 (unit roundoff 6e-8).  One step
rounds each population a few dozen times; differences then grow slowly with
the step count through the nonlinear recolouring and curvature terms.  The
bars below are the spec bar for FP32 (1e-5 relative after 1000 steps)
or tighter for short runs; every test prints its measured errors."""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as WL

from _common import check, errors, gpu_fields, oracle_params, run_oracle, u_ref

pytestmark = pytest.mark.gpu


def _sim(boxes, fields, seed=0, noise=0.0):
    import paper_2309_07801_amd as pkg
    params = [pkg.box_params_of(b) for b in boxes]
    return pkg.Simulation(params, [f[0] for f in fields], [f[1] for f in fields],
                          [f[2] for f in fields], seed=seed, noise=noise)


def _case(shape=(13, 11, 10), gamma=10.0, tau=0.7, sigma=0.01, R=3.5, u=(0.02, -0.01, 0.005),
          walls=0):
    box = WL.two_phase_box(shape, gamma, 1.0, tau, sigma, 0.7, walls=walls)
    c = tuple((n - 1) / 2.0 for n in shape)
    rr, rb, uu = WL.droplet_fields(box, [c], [R], u_carrier=u)
    return box, (rr, rb, uu)


ALL = ("rho_r", "rho_b", "phi", "p", "ux", "uy", "uz", "nx", "ny", "nz", "kappa", "Fx", "Fy",
       "Fz", "Qx", "Qy", "Qz")


@pytest.mark.parametrize("steps", [0, 1])
def test_fields_match_oracle_on_ragged_box(steps):
    """Every exported field (moments, normal, curvature, force, Q) after 0 and
    1 steps on a box whose extents are not multiples of the 8^3 tile."""
    box, fl = _case()
    sim = _sim([box], [fl], seed=5, noise=1e-5)
    sim.step(steps)
    g = gpu_fields(sim)
    o, _ = run_oracle(box, *fl, steps, seed=5, noise=1e-5)
    # Measured: at most 6.4e-6 of the field's scale (the curvature after one
    # step), 1.5e-6 for the moments, and 3.6e-7 for n in the band.
    for name in ALL:
        scale = max(np.abs(o[name]).max(), 1e-30)
        err = np.abs(g[name] - o[name]).max()
        print(steps, name, err, scale)
        if name in ("nx", "ny", "nz"):
            # the normal is ill-conditioned where |grad phi| is at rounding
            # level; compare where the interface is resolved
            band = np.abs(o["phi"]) < 0.999
            if steps == 0:
                band = (o["nx"] ** 2 + o["ny"] ** 2 + o["nz"] ** 2) > 0.5
            assert band.any()
            err = np.abs(g[name] - o[name])[band].max()
            print(steps, name, "in the interface band", err)
            assert err < 1e-6, name
        else:
            assert err <= 1e-5 * scale + 1e-12, name


def test_multi_step_translating_droplet():
    box, fl = _case(shape=(17, 9, 12), R=3.0)
    sim = _sim([box], [fl], seed=9, noise=1e-6)
    sim.step(50)
    e = errors(gpu_fields(sim), run_oracle(box, *fl, 50, seed=9, noise=1e-6)[0], box,
               u_ref(box, 0.02))
    print(e)
    check(e)


def test_static_droplet_32_cubed_200_steps_and_laplace():
    """The 32^3 static droplet (density and viscosity ratio 1, sigma 0.01,
    beta 0.7, tau 1, R 8): parity after 200 steps and Laplace's law from the
    FP64 GPU diagnostics."""
    w = WL.static_droplet()
    sim = _sim([w.box], [(w.rho_r, w.rho_b, w.u)])
    sim.step(200)
    g = gpu_fields(sim)
    o, _ = run_oracle(w.box, w.rho_r, w.rho_b, w.u, 200)
    e = errors(g, o, w.box, u_ref(w.box, 0.0))
    print(e)
    check(e)
    d = sim.reduce([w.centres[0]])[0]
    dp = d[5] - d[6]
    print("dp", dp, "R_eff", d[7], "theory", 2 * w.box.sigma / d[7])
    assert dp == pytest.approx(2 * w.box.sigma / d[7], rel=0.10)


def test_walls_droplet_and_channel():
    """Full-way bounce-back layers on y and z, with a droplet touching
    neither wall, and the layered channel with a body force."""
    box, fl = _case(shape=(14, 12, 11), R=3.0, walls=3, u=(0.01, 0.0, 0.0))
    sim = _sim([box], [fl], seed=3, noise=1e-6)
    sim.step(30)
    e = errors(gpu_fields(sim), run_oracle(box, *fl, 30, seed=3, noise=1e-6)[0], box,
               u_ref(box, 0.01))
    print("walls droplet", e)
    check(e, "droplet")
    # G 1e-5 rather than the paper's 1.5e-8: the per-step increment 3 w G of
    # a population must be well above its FP32 resolution
    w, _ = WL.layered_channel("A", a=6, b=12, nu=0.1, G=1e-5)
    w.box.nx = 3
    rr = np.repeat(w.rho_r, 3, axis=2)
    rb = np.repeat(w.rho_b, 3, axis=2)
    uu = np.repeat(w.u, 3, axis=3)
    sim = _sim([w.box], [(rr, rb, uu)])
    sim.step(300)
    g = gpu_fields(sim)
    o, _ = run_oracle(w.box, rr, rb, uu, 300)
    # velocity reference max(U, sigma/mu_max) (creeping flow: FP32 resolves
    # u only to about 1e-7 absolute)
    u_ref_l = u_ref(w.box, np.abs(o["ux"]).max())
    e = errors(g, o, w.box, u_ref_l)
    print("layered", e)
    # a flow uniform along x: every node of a layer rounds its update the
    # same way at every step, so the velocity's rounding accumulates over
    # the N steps (4 N 2^-24, measured 2.5e-5)
    check(e, "layered", u=4 * 300 * 2.0 ** -24)


def test_batched_boxes_match_solo_bitwise_and_oracle():
    cases = [_case(shape=(9, 8, 7), gamma=1.0, R=2.5),
             _case(shape=(12, 10, 9), gamma=10.0, tau=0.9, sigma=0.02, R=3.0),
             _case(shape=(16, 5, 11), gamma=100.0, tau=1.0, sigma=0.005, R=2.0, u=(0, 0, 0))]
    boxes = [c[0] for c in cases]
    fields = [c[1] for c in cases]
    sim = _sim(boxes, fields, seed=4, noise=1e-6)
    sim.step(20)
    for b, (box, fl) in enumerate(cases):
        g = gpu_fields(sim, b)
        # noise is keyed by the box index: the reference run holds the same
        # box at the same index, with only the boxes before it
        solo_b = _sim(boxes[:b] + [box], fields[:b] + [fl], seed=4, noise=1e-6)
        solo_b.step(20)
        gs = gpu_fields(solo_b, b)
        for k in g:
            assert np.array_equal(g[k], gs[k]), (b, k)
        o, _ = run_oracle(box, *fl, 20, seed=4, noise=1e-6, box_index=b)
        e = errors(g, o, box, u_ref(box, 0.02))
        print("box", b, e)
        check(e, b)


def test_reduce_matches_oracle_fields():
    box, fl = _case(shape=(16, 14, 12), R=4.0)
    sim = _sim([box], [fl], seed=1, noise=1e-6)
    sim.step(10)
    d = sim.reduce()[0]
    o, f = run_oracle(box, *fl, 10, seed=1, noise=1e-6)
    rho = o["rho_r"] + o["rho_b"]
    assert d[0] == pytest.approx(o["rho_r"].sum(), rel=1e-6)
    assert d[1] == pytest.approx(o["rho_b"].sum(), rel=1e-6)
    jx = (rho * o["ux"]).sum()
    print("x momentum", d[2], jx, abs(d[2] - jx) / abs(jx))
    assert d[2] == pytest.approx(jx, rel=1e-6)
    V = ((1 + o["phi"]) / 2).sum()
    assert d[7] == pytest.approx((3 * V / (4 * np.pi)) ** (1 / 3), rel=1e-6)
    assert d[12] == 0
    # mass of the initial state is kept
    rr0, rb0 = fl[0].astype(np.float64).sum(), fl[1].astype(np.float64).sum()
    print("mass drift", (d[0] - rr0) / rr0, (d[1] - rb0) / rb0)


def test_runs_are_bitwise_deterministic():
    box, fl = _case(shape=(15, 13, 9))
    outs = []
    for _ in range(2):
        sim = _sim([box], [fl], seed=8, noise=1e-6)
        sim.step(12)
        outs.append((gpu_fields(sim), sim.reduce()))
    for k in outs[0][0]:
        assert np.array_equal(outs[0][0][k], outs[1][0][k]), k
    assert np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("walls", [0, 3])
def test_fused_and_three_kernel_schedules_agree_bitwise(walls):
    """The column-marching fused kernel and the three-kernel schedule perform
    the same arithmetic in the same order: states and fields are identical."""
    box, fl = _case(shape=(37, 19, 41), R=5.0, walls=walls, u=(0.02, 0.01, -0.01))
    out = []
    for sched in (0, 1):
        sim = _sim([box], [fl], seed=6, noise=1e-6)
        sim.set_schedule(sched)
        sim.step(7)
        out.append(gpu_fields(sim))
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_fused_variants_agree_bitwise_and_autotune_keeps_state():
    """Every launch geometry of the fused kernel gives the same bits; the
    autotuner re-runs the fused kernel on fixed inputs and leaves the state
    unchanged."""
    import paper_2309_07801_amd as pkg
    box, fl = _case(shape=(70, 21, 37), R=6.0, u=(0.02, 0.01, -0.01))
    ref = None
    for v in range(pkg.num_variants()):
        sim = _sim([box], [fl], seed=2, noise=1e-6)
        sim.set_variant(v)
        sim.step(5)
        g = gpu_fields(sim)
        if ref is None:
            ref = g
        else:
            for k in ref:
                assert np.array_equal(ref[k], g[k]), (v, k)
    sim = _sim([box], [fl], seed=2, noise=1e-6)
    sim.step(3)
    ms = sim.autotune(reps=2)
    print("autotune ms", ms, "chosen", sim.variant())
    assert all(m > 0 for m in ms)
    sim.step(2)
    g = gpu_fields(sim)
    for k in ref:
        assert np.array_equal(ref[k], g[k]), k


@pytest.mark.parametrize("schedule", [0, 1])
def test_degenerate_boxes(schedule):
    """The method's degenerate cases in one batch, each against the oracle
    after 20 steps: a one-node box; a pure single phase (phi = 1 everywhere,
    so the normal's guard holds at every node and F = Q = 0); beta = 0 and
    sigma = 0 (no recolouring and no tension: the colours interdiffuse);
    boxes one node wide in x and in y; the smallest walled box (ny = 3: a
    single fluid row between the walls)."""
    cases = []
    one = WL.two_phase_box((1, 1, 1), 10.0, 1.0, 0.7, 0.01, 0.7)
    cases.append((one, (np.full(one.shape, 1.0, np.float32), np.full(one.shape, 0.05, np.float32),
                        np.full((3,) + one.shape, 0.01, np.float32))))
    pure = WL.two_phase_box((9, 7, 6), 10.0, 1.0, 0.7, 0.01, 0.7)
    u = np.zeros((3,) + pure.shape, np.float32)
    u[0] = 0.02
    cases.append((pure, (np.full(pure.shape, 1.0, np.float32), np.zeros(pure.shape, np.float32), u)))
    cases.append(_case(shape=(8, 7, 6), sigma=0.0, R=2.5))
    cases[-1] = (dataclasses.replace(cases[-1][0], beta=0.0), cases[-1][1])
    cases.append(_case(shape=(1, 11, 9), R=3.0))
    cases.append(_case(shape=(10, 1, 8), R=3.0))
    cases.append(_case(shape=(9, 3, 7), R=2.0, walls=1))
    boxes = [b for b, _ in cases]
    sim = _sim(boxes, [f for _, f in cases], seed=8, noise=1e-6)
    sim.set_schedule(schedule)
    sim.step(20)
    for k, (b, fl) in enumerate(cases):
        o, _ = run_oracle(b, *fl, 20, seed=8, noise=1e-6, box_index=k)
        g = gpu_fields(sim, k)
        e = errors(g, o, b, u_ref(b, 0.02))
        print(k, (b.nx, b.ny, b.nz), e)
        check(e, k)
        assert np.isfinite(g["kappa"]).all() and np.isfinite(g["Fx"]).all()
    assert np.all(sim.reduce()[:, 12] == 0)
    sim.close()
