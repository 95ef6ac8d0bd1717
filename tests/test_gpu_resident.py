"""The compact schedule with its state resident between calls
(cglbm_set_resident): a call no longer stores the populations at its end and
the next call continues from the compact state, so that a sequence of calls
is bit for bit one call of as many steps.  Checks, each bitwise against a
run without residency:

* calls of 3, 1, 4 and 2 steps against one call of 10 (the odd counts leave
  the wall stashes at both parities between calls), periodic and walled, in
  the FP32, colour-pair, mass-exact FP32 and 16-bit colour-fraction storages,
  with graph replays and with direct launches: fields, the stored
  populations (checkpoint) and the FP64 diagnostics; and for a batch of
  Models A, B, C and Model D without Q;
* the state is stored before a reader, before a step in another schedule and
  by cglbm_set_resident(0), and a loaded checkpoint replaces it;
* argument checks of the new entry points."""
import numpy as np
import pytest

import workloads as WL
from _common import gpu_fields

pytestmark = pytest.mark.gpu


def _case(shape=(40, 33, 21), gamma=10.0, R=6.0, u=(0.03, -0.01, 0.005), walls=0):
    box = WL.two_phase_box(shape, gamma, 1.0, 0.7, 0.01, 0.7, walls=walls)
    c = tuple((n - 1) / 2.0 for n in shape)
    return box, WL.droplet_fields(box, [c], [R], u_carrier=u)


def _sim(cases, storage=0, resident=False, graph=True):
    import paper_2309_07801_amd as pkg
    sim = pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                         [f[1] for _, f in cases], [f[2] for _, f in cases], seed=4,
                         noise=1e-6, storage=storage)
    sim.set_schedule(2)
    sim.set_graph(graph)
    sim.set_resident(resident)
    assert sim.resident() == resident
    return sim


def _state(sim):
    import torch
    st = sim.checkpoint().cpu()
    torch.cuda.synchronize()
    return st


def _same(a, b):
    for k in range(len(a)):
        for name in a[k]:
            assert np.array_equal(a[k][name], b[k][name]), (k, name)


@pytest.mark.parametrize("storage,walls,graph", [(0, 0, True), (0, 3, True), (0, 3, False),
                                                 (4, 2, True), (3, 3, True), (5, 3, True)])
def test_calls_equal_one_long_call(storage, walls, graph):
    cases = [_case(walls=walls), _case((24, 20, 30), R=5.0, walls=walls)]
    ref = _sim(cases, storage, graph=graph)
    ref.step(10)
    f_ref = [gpu_fields(ref, k) for k in range(2)]
    d_ref = ref.reduce()
    s_ref = _state(ref)
    ref.close()
    res = _sim(cases, storage, resident=True, graph=graph)
    for n in (3, 1, 4, 2):
        res.step(n)
    s_res = _state(res)  # stores the resident state first
    f_res = [gpu_fields(res, k) for k in range(2)]
    d_res = res.reduce()
    res.close()
    assert np.array_equal(s_ref.numpy(), s_res.numpy())
    _same(f_ref, f_res)
    assert np.array_equal(d_ref, d_res)


def test_general_models_calls_equal_one_long_call():
    """Models A, B, C and Model D without Q run schedule 2 through the
    interface and collide kernels writing compact states."""
    import dataclasses
    cases = []
    for k, (model, use_q) in enumerate(((0, 1), (1, 1), (2, 1), (3, 0))):
        b, f = _case((17 + 2 * k, 13, 11), R=3.0, u=(0.03, 0.0, 0.01), walls=k % 2)
        cases.append((dataclasses.replace(b, model=model, use_q=use_q), f))
    ref = _sim(cases)
    ref.step(6)
    f_ref = [gpu_fields(ref, k) for k in range(len(cases))]
    ref.close()
    res = _sim(cases, resident=True)
    for n in (3, 1, 2):
        res.step(n)
    f_res = [gpu_fields(res, k) for k in range(len(cases))]
    res.close()
    _same(f_ref, f_res)


def test_readers_and_other_schedules_store_the_state_first():
    cases = [_case(walls=3)]
    # reference: calls of 5 (compact) then 4 (population schedule) steps,
    # fields read in between
    ref = _sim(cases)
    ref.step(5)
    f5 = gpu_fields(ref)
    ref.set_schedule(0)
    ref.step(4)
    f9 = gpu_fields(ref)
    ref.close()
    res = _sim(cases, resident=True)
    res.step(2)
    res.step(3)
    g5 = gpu_fields(res)  # moments store the state; the next call pulls again
    res.set_schedule(0)
    res.step(4)
    g9 = gpu_fields(res)
    res.close()
    _same([f5, f9], [g5, g9])


def test_set_resident_off_stores_and_load_state_replaces():
    cases = [_case(walls=1)]
    ref = _sim(cases)
    ref.step(3)
    s3 = _state(ref)
    ref.step(4)
    s7 = _state(ref)
    ref.close()
    res = _sim(cases, resident=True)
    ck = res.checkpoint()  # the initial state
    res.step(3)
    res.set_resident(False)  # stores the state of step 3
    assert not res.resident()
    import torch
    assert np.array_equal(res.state_tensor().cpu().numpy(), s3.numpy())
    res.set_resident(True)
    res.step(2)
    res.load_state(ck)  # replaces the resident state
    res.step(3)
    res.set_resident(False)  # the state of step 3 again
    res.set_resident(True)
    res.step(2)
    res.step(2)  # with the call before: one call of 4 steps
    s = res.state_tensor().cpu()
    torch.cuda.synchronize()
    res.close()
    assert np.array_equal(s.numpy(), s7.numpy())


def test_argument_checks():
    import paper_2309_07801_amd as pkg
    lib = pkg.lib()
    estate, einval = -5, -1
    assert lib.cglbm_set_resident(None, 1, None) == estate
    assert lib.cglbm_get_resident(None) == -1
    assert lib.cglbm_sync_state(None, None) == estate
    sim = _sim([_case()])
    assert lib.cglbm_set_resident(sim.h, 2, None) == einval
    assert lib.cglbm_sync_state(sim.h, None) == pkg.CGLBM_OK  # nothing to store
    sim.close()


def test_full_size_droplet_256_in_the_bench_geometry():
    """The 256^3 translating droplet in the autotuned geometry the benchmark
    times: resident calls of 999, 1 and 1000 steps equal one call of 2000
    steps bit for bit (stored populations compared on the device)."""
    import torch
    import paper_2309_07801_amd as pkg
    w = WL.translating_droplet()
    states, geometry = [], None
    for resident in (False, True):
        sim = pkg.Simulation([pkg.box_params_of(w.box)], [w.rho_r], [w.rho_b], [w.u],
                             seed=w.seed, noise=w.noise)
        if geometry is None:
            sim.autotune(reps=1)
            sim.set_schedule(2)
            geometry = (sim.variant(), sim.compact_variant()["index"])
        else:
            sim.set_schedule(2)
            sim.set_variant(geometry[0])
            sim.set_compact_variant(geometry[1])
        assert (sim.variant(), sim.compact_variant()["index"]) == geometry
        sim.set_resident(resident)
        for n in ((999, 1, 1000) if resident else (2000,)):
            sim.step(n)
        states.append(sim.checkpoint())
        assert sim.reduce()[0, 12] == 0  # no non-finite values
        torch.cuda.synchronize()
        sim.close()
    print("geometry", geometry)
    assert torch.equal(states[0], states[1])
