"""Graph execution of the time step: replays of the captured two-step graph
give the same state, bit for bit, as launching every kernel directly --
with eager work (field export, diagnostics) and synchronisations between
replays, odd step counts, and recapture after a change of launch geometry
or schedule."""
import numpy as np
import pytest

import workloads as WL

from _common import gpu_fields

pytestmark = pytest.mark.gpu


def _pair(walls):
    import paper_2309_07801_amd as pkg
    box = WL.two_phase_box((13, 11, 10), 10.0, 1.0, 0.7, 0.01, 0.7, walls=walls)
    c = tuple((n - 1) / 2.0 for n in (13, 11, 10))
    rr, rb, u = WL.droplet_fields(box, [c], [3.5], u_carrier=(0.02, -0.01, 0.005))
    sims = [pkg.Simulation([pkg.box_params_of(box)], [rr], [rb], [u], seed=7, noise=1e-5)
            for _ in range(2)]
    sims[1].set_graph(False)
    return sims


def _same(a, b):
    ga, gb = gpu_fields(a), gpu_fields(b)
    for k in ga:
        assert np.array_equal(ga[k], gb[k]), k
    ra, rb = a.reduce(), b.reduce()
    assert np.array_equal(ra, rb)


@pytest.mark.parametrize("walls", [0, 3])
def test_graph_replays_match_direct_launches(walls):
    g, d = _pair(walls)
    for n in (4, 6, 2, 5, 1, 3):
        g.step(n)
        d.step(n)
        _same(g, d)
    g.set_variant(3)
    d.set_variant(3)
    g.step(7)
    d.step(7)
    _same(g, d)
    g.set_schedule(1)
    d.set_schedule(1)
    g.step(4)
    d.step(4)
    _same(g, d)
    g.close()
    d.close()
