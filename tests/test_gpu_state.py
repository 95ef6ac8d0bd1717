"""Checkpoint / resume and the detection of non-finite populations.

* A checkpoint (device copy of the state buffer) loaded into a fresh handle
  with the same boxes continues bit for bit as the uninterrupted run, for
  each storage format, with an odd step count before the checkpoint (the
  state then sits in the other population buffer), and for D2Q9.
* A NaN written from the host into one population of one box is counted by
  cglbm_reduce for that box only, the host-output reduce returns
  CGLBM_EUNSTABLE, and the count grows as the NaN streams."""
import numpy as np
import pytest

import workloads as WL
from _common import gpu_fields

pytestmark = pytest.mark.gpu


def _cases():
    out = []
    for shape, R in (((17, 13, 11), 3.5), ((24, 20, 9), 4.0)):
        box = WL.two_phase_box(shape, 10.0, 1.0, 0.7, 0.01, 0.7)
        c = tuple((n - 1) / 2.0 for n in shape)
        out.append((box, WL.droplet_fields(box, [c], [R], u_carrier=(0.02, -0.01, 0.005))))
    return out


def _sim(cases, storage=0, lattice="d3q27"):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=4, noise=1e-5,
                          storage=storage, lattice=lattice)


def _fields(sim, n):
    return [gpu_fields(sim, k) for k in range(n)]


def _same(a, b):
    for x, y in zip(a, b):
        for k in x:
            assert np.array_equal(x[k], y[k]), k


@pytest.mark.parametrize("storage", [0, 1, 2, 3, 4, 5, 6])
def test_checkpoint_resume_is_bitwise(storage):
    cases = _cases()
    ref = _sim(cases, storage)
    ref.step(7)
    ck = ref.checkpoint()
    ref.step(9)
    want = _fields(ref, 2)
    ref.close()
    # a fresh handle, stepped elsewhere first, then loaded from the checkpoint
    sim = _sim(cases, storage)
    sim.step(2)
    sim.load_state(ck)
    sim.step(9)
    _same(want, _fields(sim, 2))
    sim.close()


def test_checkpoint_resume_d2q9():
    import dataclasses
    w = WL.stationary_droplet_2d(n=40, R=9.0)
    b2 = dataclasses.replace(w.box, nx=45, ny=31)
    rr, rb, u = WL.droplet_fields(b2, [(22.0, 15.0, 0.0)], [8.0], u_carrier=(0.03, 0.01, 0.0))
    cases = [(w.box, (w.rho_r, w.rho_b, w.u)), (b2, (rr, rb, u))]
    ref = _sim(cases, 1, "d2q9")
    ref.step(5)
    ck = ref.checkpoint()
    ref.step(6)
    want = _fields(ref, 2)
    ref.close()
    sim = _sim(cases, 1, "d2q9")
    sim.load_state(ck)
    sim.step(6)
    _same(want, _fields(sim, 2))
    sim.close()


def test_load_state_rejects_a_foreign_checkpoint():
    import torch
    cases = _cases()
    sim = _sim(cases)
    with pytest.raises(ValueError):
        sim.load_state(torch.zeros(16, dtype=torch.uint8, device=sim.device))
    sim.close()


def test_nan_injection_is_detected():
    import torch
    cases = _cases()
    sim = _sim(cases)             # FP32: plane 27 c + i of floats
    sim.step(3)
    d = sim.reduce()
    assert not sim.last_reduce_unstable and d[:, 12].sum() == 0
    state = sim.state_tensor().view(torch.float32)
    b = 1
    node = sim.box_offset(b) + 5 + 24 * (7 + 20 * 4)          # (x, y, z) = (5, 7, 4)
    state[(27 + 3) * sim.total + node] = float("nan")           # blue, direction 3
    torch.cuda.synchronize()
    d = sim.reduce()
    assert sim.last_reduce_unstable
    assert d[0, 12] == 0 and d[1, 12] == 1
    sim.step(2)
    d = sim.reduce()
    assert sim.last_reduce_unstable and d[0, 12] == 0 and d[1, 12] > 1
    sim.close()
