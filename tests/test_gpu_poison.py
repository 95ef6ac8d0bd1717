"""Padding is never read: every byte the kernels must not read is poisoned
with all-one bits (a NaN in every float format) before stepping — the
alignment gaps between boxes and the plane tail of the stored state, all of
the second population buffer and all of aux — and the fields after 21
steps must equal, bit for bit, those of an unpoisoned run, with no
non-finite value counted.  Every storage format (with the colour fractions
of the colour-fraction-shifted formats), both layouts, a batch of
four ragged boxes with every wall combination; D2Q9 batches as well."""
import numpy as np
import pytest

import workloads as WL
from _common import gpu_fields

pytestmark = pytest.mark.gpu

SHAPES = (((17, 13, 11), 3), ((24, 20, 9), 0), ((20, 9, 14), 1), ((9, 16, 12), 2))


def _align256(v):
    return (v + 255) // 256 * 256


def _planes(storage, total):
    """(byte offset, element bytes, plane count) of the population planes."""
    if storage == 0:
        return [(0, 4, 54)]
    if storage == 4:
        return [(0, 8, 27)]
    w = 8 if storage == 3 else 4
    planes = [(0, w, 26), (_align256(26 * total * w), 8, 2)]
    if storage in (5, 6):  # the per-node colour fractions
        planes.append((_align256(26 * total * w) + 2 * total * 8, 2, 1))
    return planes


def _sim(cases, storage, inplace):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(b) for b, _ in cases], [f[0] for _, f in cases],
                          [f[1] for _, f in cases], [f[2] for _, f in cases], seed=2, noise=1e-5,
                          storage=storage, inplace=inplace)


def _poison(sim, storage):
    import torch
    total = sim.total
    used = np.zeros(total, bool)
    for k, p in enumerate(sim.params):
        b = sim.box_offset(k)
        used[b:b + p.nx * p.ny * p.nz] = True
    gap = torch.from_numpy(np.nonzero(~used)[0]).to(sim.device)
    assert gap.numel() > 0
    state = sim.state_tensor()
    for off, es, count in _planes(storage, total):
        seg = state[off:off + count * total * es].view({2: torch.int16, 4: torch.int32,
                                                         8: torch.int64}[es])
        seg.view(count, total)[:, gap] = -1
    if sim.pop_b is not None:
        other = sim.pop_b if state is sim.pop_a else sim.pop_a
        other.fill_(255)
    sim.aux.fill_(255)
    torch.cuda.synchronize()


@pytest.mark.parametrize("storage", [0, 1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("inplace", [False, True])
def test_poisoned_padding_is_never_read(storage, inplace):
    cases = []
    for shape, walls in SHAPES:
        box = WL.two_phase_box(shape, 10.0, 1.0, 0.7, 0.01, 0.7, walls=walls)
        c = tuple((n - 1) / 2.0 for n in shape)
        cases.append((box, WL.droplet_fields(box, [c], [3.0], u_carrier=(0.02, 0.0, 0.01))))
    out = []
    for poison in (False, True):
        sim = _sim(cases, storage, inplace)
        if poison:
            _poison(sim, storage)
        sim.step(21)
        d = sim.reduce()
        assert d[:, 12].sum() == 0 and not sim.last_reduce_unstable
        out.append([gpu_fields(sim, k) for k in range(len(cases))])
        sim.close()
    for k, (a, b) in enumerate(zip(out[0], out[1])):
        for name in a:
            assert np.array_equal(a[name], b[name]), (k, name)


def _planes_2d(storage, total):
    if storage in (0, 4):
        return [(0, 8, 9)]
    w = 8 if storage == 3 else 4
    return [(0, w, 8), (_align256(8 * total * w), 8, 2)]


@pytest.mark.parametrize("storage", [0, 1, 3])
def test_poisoned_padding_is_never_read_d2q9(storage):
    import dataclasses
    import torch
    import paper_2309_07801_amd as pkg
    base = WL.stationary_droplet_2d(n=40, R=9.0).box
    boxes = [dataclasses.replace(base, nx=37, ny=29), dataclasses.replace(base, nx=70, ny=21, walls=1),
             dataclasses.replace(base, nx=5, ny=7)]
    fields = [WL.droplet_fields(b, [((b.nx - 1) / 2, (b.ny - 1) / 2, 0.0)], [min(b.nx, b.ny) / 4],
                                u_carrier=(0.02, 0.01, 0.0)) for b in boxes]
    out = []
    for poison in (False, True):
        sim = pkg.Simulation([pkg.box_params_of(b) for b in boxes], [f[0] for f in fields],
                             [f[1] for f in fields], [f[2] for f in fields], seed=3, noise=1e-5,
                             storage=storage, lattice="d2q9")
        if poison:
            used = np.zeros(sim.total, bool)
            for k, p in enumerate(sim.params):
                used[sim.box_offset(k):sim.box_offset(k) + p.nx * p.ny] = True
            gap = torch.from_numpy(np.nonzero(~used)[0]).to(sim.device)
            state = sim.state_tensor()
            for off, es, count in _planes_2d(storage, sim.total):
                seg = state[off:off + count * sim.total * es].view(torch.int32 if es == 4 else torch.int64)
                seg.view(count, sim.total)[:, gap] = -1
            (sim.pop_b if state is sim.pop_a else sim.pop_a).fill_(255)
            sim.aux.fill_(255)
            torch.cuda.synchronize()
        sim.step(21)
        d = sim.reduce()
        assert d[:, 12].sum() == 0
        out.append([gpu_fields(sim, k) for k in range(len(boxes))])
        sim.close()
    for k, (a, b) in enumerate(zip(out[0], out[1])):
        for name in a:
            assert np.array_equal(a[name], b[name]), (k, name)
