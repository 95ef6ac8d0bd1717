"""The whole 96-box batch (edges drawn from U{24..128}, density ratios 1,
10 and 100, uneven tensions and viscosities) against each box run alone:
every field of every box and its diagnostics are bitwise equal after 5
steps (two captured graph pairs and a direct step), in the population and
the compact schedule.  A box's update depends only on its own nodes and
parameters, whatever the other boxes of the launch, the tile lists that
interleave them, or the launch geometry (the batch has no noise, so a box
alone is the same input as the box inside the batch)."""
import numpy as np
import pytest

import workloads as WL
from _common import gpu_fields

pytestmark = pytest.mark.gpu

STEPS = 5


def _sim(ws, storage):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(w.box) for w in ws], [w.rho_r for w in ws],
                          [w.rho_b for w in ws], [w.u for w in ws], storage=storage)


@pytest.mark.parametrize("schedule", [0, 2])
def test_batch_of_96_equals_each_box_alone(schedule):
    ws = WL.batched_boxes()
    assert all(w.noise == 0.0 for w in ws)
    batch = _sim(ws, 4)
    batch.set_schedule(schedule)
    batch.step(STEPS)
    d_batch = batch.reduce()
    got = [gpu_fields(batch, k) for k in range(len(ws))]
    batch.close()
    for k, w in enumerate(ws):
        solo = _sim([w], 4)
        solo.set_schedule(schedule)
        solo.step(STEPS)
        g = gpu_fields(solo)
        d = solo.reduce()[0]
        solo.close()
        for name in g:
            assert np.array_equal(g[name], got[k][name]), (k, name)
        assert np.array_equal(d, d_batch[k]), k
