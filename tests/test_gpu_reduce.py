"""The device-output path of cglbm_reduce: the packed per-box diagnostics
are written on the device with no host round trip, equal bit for bit those
of the host-output path (same kernels and summation order), and carry each
box's count of non-finite values in column 12."""
import numpy as np
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu


def _sim(storage=0):
    import paper_2309_07801_amd as pkg
    cases = []
    for shape, R, walls in (((17, 13, 11), 3.5, 0), ((24, 20, 9), 4.0, 3), ((70, 33, 29), 9.0, 1)):
        box = WL.two_phase_box(shape, 10.0, 1.0, 0.7, 0.01, 0.7, walls=walls)
        c = tuple((n - 1) / 2.0 for n in shape)
        cases.append((box, WL.droplet_fields(box, [c], [R], u_carrier=(0.02, -0.01, 0.005))))
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=4, noise=1e-5,
                          storage=storage)


@pytest.mark.parametrize("storage", [0, 1])
def test_device_output_equals_host_output(storage):
    import torch
    sim = _sim(storage)
    sim.step(5)
    centres = [(8.2, 6.0, 5.1), (11.5, 9.5, 4.0), (34.0, 16.0, 14.0)]
    for c in (None, centres):
        host = sim.reduce(centres=c)
        dev = sim.reduce_device(centres=c)
        torch.cuda.synchronize()
        assert np.array_equal(dev.cpu().numpy(), host)
        assert np.all(host[:, 0] > 0) and np.all(host[:, 12] == 0)
    sim.close()


def test_device_output_counts_nonfinite_values():
    import torch
    sim = _sim()
    sim.step(3)
    state = sim.state_tensor().view(torch.float32)
    node = sim.box_offset(1) + 5 + 24 * (7 + 20 * 4)        # box 1, (x, y, z) = (5, 7, 4)
    state[(27 + 3) * sim.total + node] = float("nan")         # blue, direction 3
    torch.cuda.synchronize()
    dev = sim.reduce_device().cpu().numpy()
    assert list(dev[:, 12]) == [0.0, 1.0, 0.0]
    host = sim.reduce()
    assert sim.last_reduce_unstable and np.array_equal(dev, host)
    sim.close()
