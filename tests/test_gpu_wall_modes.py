"""Wall modes of the tiled launches over boxes with walls: tiles within a
kernel's reach of a solid layer run the kernel with the wall logic, the
others the one without it; bit 0 of the mode gives the slabs next to z walls
short chunks of their own, bit 1 runs the near-wall launch on a side stream
beside the other (fork and join by events, also inside the captured graphs).

The boxes are large enough for both tile lists to be non-empty and for the
short z-edge chunks to exist.  Checks, in the population and the compact
schedule:

* the four modes give bitwise identical fields after 7 steps (three graph
  pairs and one direct step);
* with the side stream, graph replays match direct launches bit for bit,
  with eager work (field export, diagnostics) between replays;
* the autotuner leaves a mode in 0..3 for each schedule, and the fields
  after it equal those of a fixed mode."""
import numpy as np
import pytest

import workloads as WL
from _common import gpu_fields

pytestmark = pytest.mark.gpu

SHAPES = (((70, 40, 100), 3, 10.0), ((48, 33, 90), 2, 8.0), ((40, 36, 20), 1, 6.0))


def _cases():
    out = []
    for shape, walls, R in SHAPES:
        box = WL.two_phase_box(shape, 10.0, 1.0, 0.7, 0.01, 0.7, walls=walls)
        c = tuple((n - 1) / 2.0 for n in shape)
        out.append((box, WL.droplet_fields(box, [c], [R], u_carrier=(0.03, 0.0, 0.01))))
    return out


def _sim(cases):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=5, noise=1e-6)


def _fields(sim, n):
    return [gpu_fields(sim, k) for k in range(n)]


def _same(ref, got, tag):
    for a, b in zip(ref, got):
        for name in a:
            assert np.array_equal(a[name], b[name]), (tag, name)


@pytest.mark.parametrize("schedule", [0, 2])
def test_wall_modes_bitwise_equal(schedule):
    cases = _cases()
    ref = None
    for mode in (3, 0, 1, 2):
        sim = _sim(cases)
        sim.set_wall_mode(mode)
        sim.set_schedule(schedule)
        assert sim.wall_mode() == mode
        sim.step(7)
        got = _fields(sim, len(cases))
        assert sim.reduce()[:, 12].sum() == 0
        sim.close()
        if ref is None:
            ref = got
        else:
            _same(ref, got, (schedule, mode))


@pytest.mark.parametrize("schedule", [0, 2])
def test_side_stream_graph_replays_match_direct_launches(schedule):
    cases = _cases()
    g, d = _sim(cases), _sim(cases)
    for s in (g, d):
        s.set_wall_mode(3)
        s.set_schedule(schedule)
    d.set_graph(False)
    for n in (4, 6, 2, 5):
        g.step(n)
        d.step(n)
        _same(_fields(d, len(cases)), _fields(g, len(cases)), n)
        assert np.array_equal(g.reduce(), d.reduce())
    g.close()
    d.close()


def test_autotuned_wall_modes():
    cases = _cases()
    sim, ref = _sim(cases), _sim(cases)
    sim.autotune(reps=2)
    for schedule in (0, 2):
        sim.set_schedule(schedule)
        assert 0 <= sim.wall_mode() <= 3
        print("schedule", schedule, "wall mode", sim.wall_mode())
    ref.set_wall_mode(0)
    sim.set_schedule(2)
    ref.set_schedule(2)
    sim.step(5)
    ref.step(5)
    _same(_fields(ref, len(cases)), _fields(sim, len(cases)), "autotuned")
    sim.close()
    ref.close()


def test_wall_mode_argument_checks():
    """Modes outside 0..3 are refused with CGLBM_EINVAL and leave the mode as
    it was; a D2Q9 handle has no wall modes (CGLBM_EUNSUPPORTED)."""
    import paper_2309_07801_amd as pkg
    cases = _cases()[2:]
    sim = _sim(cases)
    sim.set_wall_mode(1)
    for bad in (-1, 4):
        with pytest.raises(pkg.CglbmError) as ei:
            sim.set_wall_mode(bad)
        assert ei.value.code == -1
    assert sim.wall_mode() == 1
    sim.close()
    box = WL.Box(nx=40, ny=30, nz=1, rho0_r=10.0, rho0_b=1.0, alpha_r=WL.alpha_heavy_2d(10.0),
                 alpha_b=WL.ALPHA_LIGHT_2D, nu_r=0.1, nu_b=0.1, sigma=0.01, beta=0.7, walls=1)
    rr, rb, u = WL.droplet_fields(box, [(19.5, 14.5, 0.0)], [6.0])
    sim2 = pkg.Simulation([pkg.box_params_of(box)], [rr], [rb], [u], lattice="d2q9")
    with pytest.raises(pkg.CglbmError) as ei:
        sim2.set_wall_mode(0)
    assert ei.value.code == -3
    sim2.close()
