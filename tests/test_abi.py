"""The C-ABI library loads without a GPU, exports every symbol declared in
include/cglbm.h, and validates parameters on the host (no compute calls)."""
import os
import re

import pytest

import paper_2309_07801_amd as pkg
import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "cglbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cglbm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = pkg.lib()
    names = _declared_functions()
    assert "cglbm_init" in names and "cglbm_step" in names
    assert "cglbm_moments" in names and "cglbm_reduce" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(pkg.EXPORTED) == set(names)


def test_query_sizes_layout():
    boxes = [WL.two_phase_box((10, 7, 5), 10.0, 1.0, 0.8, 0.01, 0.7),
             WL.two_phase_box((3, 4, 5), 1.0, 1.0, 0.8, 0.01, 0.7)]
    pop, aux, total = pkg.query_sizes([pkg.box_params_of(b) for b in boxes])
    # box 0: 350 nodes -> aligned to 384; box 1: 60 nodes -> 448 total
    assert total == 448
    assert pop == total * 54 * 4
    assert aux == total * 21 * 4


@pytest.mark.parametrize("field,value,code", [
    ("nx", 0, -1), ("walls", 4, -1), ("sigma", -1.0, -1), ("beta", float("nan"), -1),
    ("omega_bulk", 2.0, -1), ("omega_hi", 2.5, -1), ("omega_hi", 0.0, -1), ("model", 4, -1),
    ("model", -1, -1),
    ("q_correction", 2, -1)])
def test_parameter_validation(field, value, code):
    b = WL.two_phase_box((8, 8, 8), 10.0, 1.0, 0.8, 0.01, 0.7)
    p = pkg.box_params_of(b)
    if field == "omega_hi":
        p.omega_hi[3] = value
    else:
        setattr(p, field, value)
    with pytest.raises(pkg.CglbmError) as ei:
        pkg.query_sizes([p])
    assert ei.value.code == code


def test_storage_buffer_sizes():
    b = WL.two_phase_box((10, 7, 5), 10.0, 1.0, 0.8, 0.01, 0.7)
    pb = [pkg.box_params_of(b)]
    pop32, aux32, total = pkg.query_sizes(pb, pkg.FP32)
    pop16, aux16, _ = pkg.query_sizes(pb, pkg.FP16_SHIFT)
    popx, auxx, _ = pkg.query_sizes(pb, pkg.FP32_EXACT)
    align = lambda v: (v + 255) // 256 * 256
    # 350 nodes -> 384 (multiple of 64) -> 448 (odd multiple of 64)
    assert total == 448
    assert pop32 == 54 * total * 4 and aux32 == 21 * total * 4
    assert pop16 == align(52 * total * 2) + 2 * total * 8
    assert popx == align(52 * total * 4) + 2 * total * 8
    assert aux16 == align(21 * total * 4) + 2 * total * 8 == auxx
    assert pkg.query_sizes(pb, pkg.FP32_PAIRS) == (pop32, aux32, total)
    # colour-fraction shift: one 16-bit fraction per node after the rest planes
    for st in (pkg.FP16_CSHIFT, pkg.BF16_CSHIFT):
        assert pkg.query_sizes(pb, st) == (pop16 + 2 * total, aux16, total)
    with pytest.raises(pkg.CglbmError):
        pkg.query_sizes(pb, 7)


def test_phase_validation_and_storage():
    b = WL.two_phase_box((8, 8, 8), 10.0, 1.0, 0.8, 0.01, 0.7)
    p = pkg.box_params_of(b)
    p.red.alpha = 1.0
    with pytest.raises(pkg.CglbmError):
        pkg.query_sizes([p])
    p = pkg.box_params_of(b)
    with pytest.raises(pkg.CglbmError) as ei:
        pkg.query_sizes([p], storage=7)
    assert ei.value.code in (-1, -3)


def _box2d(nx=40, ny=30, **kw):
    b = WL.stationary_droplet_2d(n=nx, R=8.0).box
    import dataclasses
    return dataclasses.replace(b, nx=nx, ny=ny, **kw)


def _align256(v):
    return (v + 255) // 256 * 256


def test_d2q9_sizes_and_validation():
    """The D2Q9 entry points: 9 pair planes of 2 x float per node (either
    FP32 format), or 8 pair planes and two FP64 rest planes (mass-exact
    formats, whose aux also carries the FP64 colour densities); the aux
    layout of D3Q27; nz = 1, Eq. (A10) only."""
    p = [pkg.box_params_of(_box2d())]
    pop, aux, total = pkg.query_sizes(p, pkg.FP32, lattice="d2q9")
    assert total == 1216          # 1200 -> 1216 (multiple of 64) is odd multiple of 64 (19)
    assert pop == 9 * 8 * total and aux == 21 * 4 * total
    assert pkg.query_sizes(p, pkg.FP32_PAIRS, lattice="d2q9") == (pop, aux, total)
    aux_x = _align256(21 * 4 * total) + 2 * 8 * total
    for st, word in ((pkg.FP16_SHIFT, 4), (pkg.BF16_SHIFT, 4), (pkg.FP32_EXACT, 8)):
        assert pkg.query_sizes(p, st, lattice="d2q9") == (
            _align256(8 * word * total) + 2 * 8 * total, aux_x, total), st
    for field, value, code in (("nz", 2, -1), ("walls", 2, -1), ("model", 0, -3)):
        q = pkg.box_params_of(_box2d())
        setattr(q, field, value)
        with pytest.raises(pkg.CglbmError) as ei:
            pkg.query_sizes([q], pkg.FP32, lattice="d2q9")
        assert ei.value.code == code, field
    q = pkg.box_params_of(_box2d())
    q.omega_hi[2] = 1.5
    with pytest.raises(pkg.CglbmError) as ei:
        pkg.query_sizes([q], pkg.FP32, lattice="d2q9")
    assert ei.value.code == -3
    with pytest.raises(pkg.CglbmError) as ei:
        pkg.query_sizes(p, pkg.FP16_CSHIFT, lattice="d2q9")   # D3Q27 only
    assert ei.value.code == -3
    with pytest.raises(pkg.CglbmError) as ei:
        pkg.query_sizes(p, 7, lattice="d2q9")
    assert ei.value.code == -1
    with pytest.raises(ValueError):
        pkg.query_sizes(p, pkg.FP32, lattice="d3q19")


def test_empty_and_oversized_inputs_are_rejected():
    """No boxes, and all boxes together beyond the node limit (every plane of
    8-byte values must stay below 4 GiB), are CGLBM_EINVAL on the host."""
    import ctypes as C
    pop, aux, tot = C.c_size_t(), C.c_size_t(), C.c_int64()
    rc = pkg.lib().cglbm_query_sizes(0, None, pkg.FP32, C.byref(pop), C.byref(aux), C.byref(tot))
    assert rc == -1
    big = WL.two_phase_box((1024, 1024, 512), 10.0, 1.0, 0.8, 0.01, 0.7)   # 2^29 nodes
    with pytest.raises(pkg.CglbmError) as ei:
        pkg.query_sizes([pkg.box_params_of(big)])
    assert ei.value.code == -1
    # just below the limit in two boxes: accepted, total stays under 2^29 nodes
    a = WL.two_phase_box((1024, 1024, 255), 10.0, 1.0, 0.8, 0.01, 0.7)
    pop_b, aux_b, total = pkg.query_sizes([pkg.box_params_of(a), pkg.box_params_of(a)])
    assert total < (1 << 29) and pop_b == 54 * 4 * total
    with pytest.raises(pkg.CglbmError):
        pkg.query_sizes([pkg.box_params_of(a)] * 3)


def test_null_handle_calls_fail_cleanly():
    """Host-side error paths of the handle calls (no device work): a NULL
    handle gives CGLBM_ESTATE or a NULL / -1 result, never a crash."""
    import ctypes as C
    L = pkg.lib()
    assert L.cglbm_state_buffer(None) is None
    assert L.cglbm_load_state(None, None, None) == -5
    assert L.cglbm_step(None, 1, None) == -5
    assert L.cglbm_lattice(None) == -1
    assert L.cglbm_box_offset(None, 0) == -1
    out = (C.c_double * 13)()
    assert L.cglbm_reduce(None, None, out, 1, None) == -5
    assert L.cglbm_set_wall_mode(None, 0, None) == -5
    assert L.cglbm_get_wall_mode(None) == -1
    assert L.cglbm_set_resident(None, 1, None) == -5
    assert L.cglbm_get_resident(None) == -1
    assert L.cglbm_sync_state(None, None) == -5


def test_inplace_layout_restrictions():
    """pop_b = NULL (one population buffer) is refused on the host, before any
    device work, where a kernel reads populations after the pull: D2Q9 (one
    kernel pulls and stores) and non-unit higher-order rates (the collision
    pulls again)."""
    import ctypes as C
    L = pkg.lib()
    fake = C.c_void_p(0x1000)     # never dereferenced: the calls fail first
    h = C.c_void_p()

    def init(fn, params):
        arr = (pkg.BoxParams * 1)(params)
        return fn(C.byref(h), 1, arr, pkg.FP32, fake, None, fake, fake, fake, fake, 0, 0.0, None)

    assert init(L.cglbm_init_d2q9, pkg.box_params_of(_box2d())) == -3
    q = pkg.box_params_of(WL.two_phase_box((8, 8, 8), 10.0, 1.0, 0.7, 0.01, 0.7))
    q.omega_hi[3] = 1.2
    assert init(L.cglbm_init, q) == -3
    assert "pop_b" in L.cglbm_last_error().decode()
