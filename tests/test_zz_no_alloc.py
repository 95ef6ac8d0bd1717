"""cglbm_reduce_noalloc, the allocation-free variant of cglbm_reduce (its
scratch is the library's static device array): through the C ABI its output
equals cglbm_reduce's bit for bit, on two calls in a row whose second has a
smaller input, with and without caller-given centres; captured into a HIP
graph and replayed with other work in between, every replay equals the
eager reduction of the state it sees; handles beyond the scratch's limits
are refused."""
import ctypes as C

import numpy as np
import pytest

import workloads as WL

pytestmark = pytest.mark.gpu


def _lib():
    import paper_2309_07801_amd as pkg
    L = pkg.lib()
    L.cglbm_reduce_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.cglbm_reduce_noalloc.restype = C.c_int
    return L


def _noalloc(sim, out, centre=None, stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _lib().cglbm_reduce_noalloc(sim.h, None if centre is None else centre.data_ptr(),
                                       out.data_ptr(), s.cuda_stream)


def _sim(specs, storage=0):
    import paper_2309_07801_amd as pkg
    cases = []
    for shape, R, walls in specs:
        box = WL.two_phase_box(shape, 10.0, 1.0, 0.7, 0.01, 0.7, walls=walls)
        c = tuple((n - 1) / 2.0 for n in shape)
        cases.append((box, WL.droplet_fields(box, [c], [R], u_carrier=(0.02, -0.01, 0.005))))
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=4, noise=1e-5,
                          storage=storage)


BIG = (((17, 13, 11), 3.5, 0), ((24, 20, 9), 4.0, 3), ((130, 65, 40), 12.0, 1))
SMALL = (((9, 8, 7), 2.5, 0),)


def test_noalloc_equals_reduce_on_two_calls_second_smaller():
    import torch
    big = _sim(BIG)
    big.step(5)
    out = torch.full((3, 13), float("nan"), dtype=torch.float64, device=big.device)
    assert _noalloc(big, out) == 0
    got = out.cpu().numpy()
    want = big.reduce()
    assert np.array_equal(got, want) and np.all(want[:, 0] > 0)
    centres = [(8.2, 6.0, 5.1), (11.5, 9.5, 4.0), (64.0, 32.0, 19.5)]
    cdev = torch.tensor(centres, dtype=torch.float64, device=big.device)
    assert _noalloc(big, out, cdev) == 0
    assert np.array_equal(out.cpu().numpy(), big.reduce(centres=centres))
    big.close()
    # the second call: a smaller handle on the same GPU (the scratch still
    # holds the first call's partials)
    small = _sim(SMALL, storage=1)
    small.step(3)
    out2 = torch.full((1, 13), float("nan"), dtype=torch.float64, device=small.device)
    assert _noalloc(small, out2) == 0
    assert np.array_equal(out2.cpu().numpy(), small.reduce())
    small.close()


def test_noalloc_replays_from_a_captured_graph():
    import torch
    sim = _sim(BIG)
    sim.step(2)
    out = torch.zeros((3, 13), dtype=torch.float64, device=sim.device)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rc = _noalloc(sim, out, stream=torch.cuda.current_stream())
    assert rc == 0
    for k in range(3):
        # eager work between the replays; two steps keep the state in the
        # buffer the graph was captured on
        sim.step(2)
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        want = sim.reduce()
        assert np.array_equal(out.cpu().numpy(), want), k
    del g
    sim.close()


def test_noalloc_refuses_handles_beyond_the_scratch():
    import torch
    import paper_2309_07801_amd as pkg
    n = 4097
    box = WL.two_phase_box((1, 1, 1), 1.0, 1.0, 0.8, 0.0, 0.0)
    one = [np.ones((1, 1, 1), np.float32)]
    sim = pkg.Simulation([pkg.box_params_of(box)] * n, one * n, [np.zeros((1, 1, 1), np.float32)] * n,
                         [np.zeros((3, 1, 1, 1), np.float32)] * n)
    out = torch.zeros((n, 13), dtype=torch.float64, device=sim.device)
    assert _noalloc(sim, out) == -1
    assert "4096 boxes" in _lib().cglbm_last_error().decode()
    d = sim.reduce()
    np.testing.assert_allclose(d[:, 0], 1.0, rtol=1e-6)   # FP32 populations, FP64 sums
    assert np.all(d[:, 1] == 0.0) and np.all(d[:, 12] == 0.0)
    sim.close()
