"""Seeded input generators: the bounding-box sphere marking gives the same
arrays as a brute-force periodic-distance definition."""
import numpy as np
import pytest

import workloads as WL


def _brute(box, centres, radii, u_drop=None, u_carrier=None):
    red = np.zeros(box.shape, dtype=bool)
    for c, r in zip(centres, radii):
        red |= WL.periodic_distance((box.nx, box.ny, box.nz), c, box.walls) <= r
    rho_r = np.where(red, box.rho0_r, 0.0).astype(np.float32)
    rho_b = np.where(red, 0.0, box.rho0_b).astype(np.float32)
    u = np.zeros((3,) + box.shape, dtype=np.float32)
    if u_carrier is not None:
        u[:] = np.asarray(u_carrier, dtype=np.float32).reshape(3, 1, 1, 1)
    if u_drop is not None:
        for c, r, ud in zip(centres, radii, u_drop):
            m = WL.periodic_distance((box.nx, box.ny, box.nz), c, box.walls) <= r
            for a in range(3):
                u[a][m] = ud[a]
    return rho_r, rho_b, u


@pytest.mark.parametrize("walls", [0, 1, 2, 3])
def test_droplet_fields_match_brute_force(walls):
    rng = np.random.Generator(np.random.PCG64(11 + walls))
    for trial in range(6):
        n = rng.integers(6, 20, size=3)
        box = WL.two_phase_box(tuple(int(v) for v in n), 10.0, 1.0, 0.8, 0.01, 0.7, walls=walls)
        k = int(rng.integers(1, 4))
        centres = [tuple(rng.uniform(-1.0, float(v)) for v in n) for _ in range(k)]
        radii = [float(rng.uniform(0.5, 0.6 * min(n))) for _ in range(k)]
        ud = [tuple(rng.uniform(-0.1, 0.1, size=3)) for _ in range(k)]
        got = WL.droplet_fields(box, centres, radii, u_drop=ud, u_carrier=(0.01, 0.0, -0.02))
        ref = _brute(box, centres, radii, u_drop=ud, u_carrier=(0.01, 0.0, -0.02))
        for g, r in zip(got, ref):
            assert np.array_equal(g, r)


def test_full_size_generators_are_fast_and_deterministic():
    import time
    t = time.time()
    a = WL.head_on_collision(nx=192, ny=96, nz=96, R=12.0)
    b = WL.head_on_collision(nx=192, ny=96, nz=96, R=12.0)
    assert time.time() - t < 20
    for x, y in zip((a.rho_r, a.rho_b, a.u), (b.rho_r, b.rho_b, b.u)):
        assert np.array_equal(x, y)
    assert a.rho_r.sum() > 0
