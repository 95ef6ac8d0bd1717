"""The compact schedule (schedule 2): the state of a node between the steps
of one cglbm_step call is its compact post-collision state (17 values) and
the pull rebuilds the collided populations of a column and its ring in
registers.  Checks:

* one step per call is bit for bit the fused schedule (the call is the
  population pull, the compact fused kernel and the emission, whose
  populations equal the fused kernel's);
* many steps per call against the FP64 oracle with the FP32 bars, on a
  ragged box and on a batch of unlike boxes, in both FP32 layouts;
* close to the fused schedule after many steps (FP32 rounding of the moment
  sums in another order), mass drift at FP32 rounding level;
* boxes with solid walls (the wall stashes of the bounce-back): one step per
  call bitwise, many steps against the oracle;
* the equilibrium families A, B, C and Model D without Q (the interface and
  collide kernels writing compact states): one step per call bitwise equal
  to the three-kernel schedule, many steps against the oracle;
* layouts it does not serve are refused with CGLBM_EUNSUPPORTED."""
import numpy as np
import pytest

import workloads as WL
from _common import check, errors, gpu_fields, run_oracle, u_ref

pytestmark = pytest.mark.gpu


def _case(shape=(17, 13, 11), gamma=10.0, R=3.5, u=(0.02, -0.01, 0.005), walls=0, **kw):
    box = WL.two_phase_box(shape, gamma, 1.0, 0.7, 0.01, 0.7, walls=walls, **kw)
    c = tuple((n - 1) / 2.0 for n in shape)
    return box, WL.droplet_fields(box, [c], [R], u_carrier=u)


def _sim(cases, storage=0, **kw):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=4, noise=1e-6,
                          storage=storage, **kw)


@pytest.mark.parametrize("storage", [0, 4, 3])
def test_single_step_calls_equal_fused_schedule(storage):
    cases = [_case(), _case((40, 33, 21), R=6.0)]
    out = []
    for sched in (0, 2):
        sim = _sim(cases, storage)
        sim.set_schedule(sched)
        assert sim.schedule() == sched
        for _ in range(6):
            sim.step(1)
        out.append([gpu_fields(sim, k) for k in range(2)])
        sim.close()
    for a, b in zip(out[0], out[1]):
        for name in a:
            assert np.array_equal(a[name], b[name]), name


@pytest.mark.parametrize("storage", [0, 4, 3])
def test_compact_schedule_parity_with_oracle(storage):
    cases = [_case(), _case((24, 20, 9), gamma=3.0, R=4.0, u=(0.05, 0.0, 0.0)),
             _case((40, 12, 45), R=4.0)]
    sim = _sim(cases, storage)
    sim.set_schedule(2)
    sim.step(50)
    for k, (box, fl) in enumerate(cases):
        o = run_oracle(box, *fl, 50, seed=4, noise=1e-6, box_index=k)[0]
        e = errors(gpu_fields(sim, k), o, box, u_ref(box, 0.05))
        print(k, e)
        check(e, k)
    d = sim.reduce()
    assert d[:, 12].sum() == 0
    sim.close()


def test_compact_schedule_close_to_fused_and_conserves_mass():
    cases = [_case((48, 40, 36), R=8.0, u=(0.05, 0.0, 0.0))]
    out, drift = [], []
    for sched in (0, 2):
        sim = _sim(cases)
        sim.set_schedule(sched)
        d0 = sim.reduce()[0]
        sim.step(300)
        d1 = sim.reduce()[0]
        drift.append([(d1[k] - d0[k]) / d0[k] for k in (0, 1)])
        out.append(gpu_fields(sim))
        sim.close()
    print("mass drift fused / compact", drift)
    # The schedules differ only in the FP32 order of the moment sums; after
    # 300 steps the fields were measured 1.2e-6 apart in density and 4.4e-6 U
    # in velocity, and the compact run's colour masses 5e-8 from the start.
    for name in ("rho_r", "rho_b"):
        print(name, np.abs(out[0][name] - out[1][name]).max() / np.abs(out[0][name]).max())
        assert np.abs(out[0][name] - out[1][name]).max() <= 5e-6 * np.abs(out[0][name]).max(), name
    for name in ("ux", "uy", "uz"):
        print(name, np.abs(out[0][name] - out[1][name]).max() / 0.05)
        assert np.abs(out[0][name] - out[1][name]).max() <= 2e-5 * 0.05, name
    assert max(abs(x) for x in drift[1]) < 1e-6


def test_compact_schedule_refuses_other_layouts():
    import dataclasses
    import paper_2309_07801_amd as pkg
    b, f = _case()
    refused = [
        ([(dataclasses.replace(b, model=0), f)], {"storage": 1}),
        ([(dataclasses.replace(b, use_q=0), f)], {"storage": 5}),
        ([(b, f)], {"inplace": True}),
        ([(b, f)], {"storage": 2, "inplace": True}),
        ([(dataclasses.replace(b, omega_hi=(1.0, 1.2) + (1.0,) * 7), f)], {}),
        ([(dataclasses.replace(b, model=0), f)], {"storage": 3}),
    ]
    for cases, kw in refused:
        sim = _sim(cases, **kw)
        with pytest.raises(pkg.CglbmError) as ei:
            sim.set_schedule(2)
        assert ei.value.code == -3
        sim.close()


def test_compact_pull_geometries_agree_bitwise():
    """Every column tile and z chunk of the compact pull gives the same bits
    (each node sums its arrivals in the same order whatever the tile), and
    the autotuner keeps the stored state while choosing one."""
    cases = [_case((70, 21, 37), R=6.0, u=(0.02, 0.01, -0.01)), _case()]
    ref = None
    for v in range(5):
        sim = _sim(cases)
        sim.set_schedule(2)
        sim.set_compact_variant(v)
        assert sim.compact_variant()["index"] == v
        sim.step(9)
        out = [gpu_fields(sim, k) for k in range(2)]
        sim.close()
        if ref is None:
            ref = out
        for a, b in zip(ref, out):
            for name in a:
                assert np.array_equal(a[name], b[name]), (v, name)
    out = []
    for tune in (False, True):
        sim = _sim(cases)
        sim.step(2)
        if tune:
            sim.autotune(reps=2)
            print("compact pull chosen", sim.compact_variant())
        sim.set_schedule(2)
        sim.step(7)
        out.append([gpu_fields(sim, k) for k in range(2)])
        sim.close()
    for a, b in zip(out[0], out[1]):
        for name in a:
            assert np.array_equal(a[name], b[name]), name


WALLED = (((17, 13, 11), 3), ((24, 20, 9), 1), ((20, 9, 14), 2), ((23, 16, 12), 0))


def _walled_cases():
    out = []
    for shape, walls in WALLED:
        out.append(_case(shape, R=3.0, u=(0.02, 0.0, 0.01), walls=walls))
    return out


@pytest.mark.parametrize("storage", [0, 4, 3])
def test_walls_single_step_calls_equal_fused_schedule(storage):
    cases = _walled_cases()
    out = []
    for sched in (0, 2):
        sim = _sim(cases, storage)
        sim.set_schedule(sched)
        for _ in range(5):
            sim.step(1)
        out.append([gpu_fields(sim, k) for k in range(len(cases))])
        sim.close()
    for a, b in zip(out[0], out[1]):
        for name in a:
            assert np.array_equal(a[name], b[name]), name


@pytest.mark.parametrize("storage", [0, 4, 3])
def test_walls_parity_with_oracle(storage):
    """A batch of boxes with every wall combination, 60 steps in one call
    (graph pairs, the wall stashes alternating), against the oracle."""
    cases = _walled_cases()
    sim = _sim(cases, storage)
    sim.set_schedule(2)
    sim.step(60)
    for k, (box, fl) in enumerate(cases):
        o = run_oracle(box, *fl, 60, seed=4, noise=1e-6, box_index=k)[0]
        e = errors(gpu_fields(sim, k), o, box, u_ref(box, 0.02))
        print(k, box.walls, e)
        check(e, k)
    d = sim.reduce()
    assert d[:, 12].sum() == 0
    sim.close()


def test_walls_close_to_fused_over_many_steps():
    cases = [_case((40, 24, 30), R=6.0, u=(0.04, 0.0, 0.0), walls=3)]
    out = []
    for sched in (0, 2):
        sim = _sim(cases)
        sim.set_schedule(sched)
        sim.step(250)
        out.append(gpu_fields(sim))
        sim.close()
    for name in ("rho_r", "rho_b"):
        print(name, np.abs(out[0][name] - out[1][name]).max() / np.abs(out[0][name]).max())
        assert np.abs(out[0][name] - out[1][name]).max() <= 5e-6 * np.abs(out[0][name]).max(), name
    for name in ("ux", "uy", "uz"):
        print(name, np.abs(out[0][name] - out[1][name]).max() / 0.04)
        assert np.abs(out[0][name] - out[1][name]).max() <= 2e-5 * 0.04, name


def _general_cases():
    import dataclasses
    out = []
    for k, (model, use_q) in enumerate(((0, 1), (1, 1), (2, 1), (3, 0))):
        b, f = _case((17 + 2 * k, 13, 11), R=3.0, u=(0.03, 0.0, 0.01), walls=k % 2)
        out.append((dataclasses.replace(b, model=model, use_q=use_q), f))
    return out


def test_general_models_single_step_calls_equal_three_kernel_schedule():
    cases = _general_cases()
    out = []
    for sched in (1, 2):
        sim = _sim(cases)
        sim.set_schedule(sched)
        assert sim.schedule() == sched
        for _ in range(4):
            sim.step(1)
        out.append([gpu_fields(sim, k) for k in range(len(cases))])
        sim.close()
    for a, b in zip(out[0], out[1]):
        for name in a:
            assert np.array_equal(a[name], b[name]), name


def test_general_models_parity_with_oracle():
    """Models A, B, C with Q and Model D without Q in one batch (two of the
    boxes walled), 50 steps in one call, against the oracle."""
    cases = _general_cases()
    sim = _sim(cases)
    sim.set_schedule(2)
    sim.step(50)
    for k, (box, fl) in enumerate(cases):
        o = run_oracle(box, *fl, 50, seed=4, noise=1e-6, box_index=k)[0]
        e = errors(gpu_fields(sim, k), o, box, u_ref(box, 0.03))
        print(k, box.model, box.use_q, e)
        check(e, k)
    sim.close()


@pytest.mark.parametrize("walls", [0, 3])
def test_mass_exact_compact_schedule_conserves_colour_mass(walls):
    """The mass-exact FP32 storage in the compact schedule: FP64 colour
    densities in the compact state, each node's rest population closed on
    them, FP64 sums of the arrivals; 300 steps in one call of a translating
    droplet at density ratio 10 keep each colour's mass to FP64 rounding
    (periodic; with walls the bounce-back stashes hold the solid nodes' share,
    which the reduction does not count, so the box is chosen with the
    droplet and its flow away from the walls), and stay close to the
    population schedule with the same storage."""
    cases = [_case((24, 20, 18), R=5.0, u=(0.05, 0.0, 0.0), walls=walls)]
    out, drift = [], []
    for sched in (0, 2):
        sim = _sim(cases, 3)
        sim.set_schedule(sched)
        d0 = sim.reduce()[0]
        sim.step(300)
        d1 = sim.reduce()[0]
        drift.append([(d1[k] - d0[k]) / d0[k] for k in (0, 1)])
        out.append(gpu_fields(sim))
        sim.close()
    print("mass drift population / compact", drift)
    if walls == 0:
        assert max(abs(x) for x in drift[1]) < 1e-12
    for name in ("rho_r", "rho_b"):
        assert np.abs(out[0][name] - out[1][name]).max() <= 5e-5 * np.abs(out[0][name]).max(), name
