"""The in-place layout (one population buffer, pop_b = NULL) against the
two-buffer layout: bitwise equal fields after an odd number of steps (graph
pairs, then a direct launch) for every storage format and both schedules,
on a batch of boxes with every wall combination (the wall stash and its
copy kernel); the autotuner in place advances the state by exactly one
step; a checkpoint of the one buffer resumes bit for bit."""
import numpy as np
import pytest

import workloads as WL
from _common import gpu_fields

pytestmark = pytest.mark.gpu

SHAPES = (((17, 13, 11), 3), ((24, 20, 9), 0), ((20, 9, 14), 1), ((9, 16, 12), 2))


def _cases():
    out = []
    for shape, walls in SHAPES:
        box = WL.two_phase_box(shape, 10.0, 1.0, 0.7, 0.01, 0.7, walls=walls)
        c = tuple((n - 1) / 2.0 for n in shape)
        out.append((box, WL.droplet_fields(box, [c], [3.0], u_carrier=(0.02, 0.0, 0.01))))
    return out


def _sim(cases, storage, inplace):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=6, noise=1e-5,
                          storage=storage, inplace=inplace)


def _fields(sim):
    return [gpu_fields(sim, k) for k in range(sim.nboxes)]


def _same(a, b):
    for k, (x, y) in enumerate(zip(a, b)):
        for name in x:
            assert np.array_equal(x[name], y[name]), (k, name)


@pytest.mark.parametrize("storage", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("schedule", [0, 1])
def test_inplace_equals_two_buffers(storage, schedule):
    cases = _cases()
    out = []
    for inplace in (False, True):
        sim = _sim(cases, storage, inplace)
        sim.set_schedule(schedule)
        sim.step(41)
        out.append(_fields(sim))
        d = sim.reduce()
        assert d[:, 12].sum() == 0
        sim.close()
    _same(out[0], out[1])


def test_inplace_autotune_advances_one_step():
    cases = _cases()
    ref = _sim(cases, 0, False)
    ref.step(10)
    want = _fields(ref)
    ref.close()
    sim = _sim(cases, 0, True)
    sim.step(5)
    sim.autotune(reps=2)
    assert sim.steps_done == 6
    sim.step(4)
    _same(want, _fields(sim))
    sim.close()


def test_inplace_checkpoint_resume():
    cases = _cases()
    ref = _sim(cases, 1, True)
    ref.step(6)
    ck = ref.checkpoint()
    assert ref.state_tensor() is ref.pop_a
    ref.step(7)
    want = _fields(ref)
    ref.close()
    sim = _sim(cases, 1, True)
    sim.load_state(ck)
    sim.step(7)
    _same(want, _fields(sim))
    sim.close()
