"""Writes p5_head_on_collision_192.json: the FP64 oracle after 100 and 750
steps of the walled head-on collision at 192x96x96 (two droplets of radius 12
approaching at relative velocity 0.1, density ratio 10, solid layers at the
y and z walls; the Weber and Reynolds numbers of the 768x384x384 case kept
by scaling sigma and nu with the radius), the reduced-size parity run of
that configuration.

Stored: the order parameter, colour densities and velocity at sampled fluid
nodes (the two lines of nodes through the droplet centres along x, 1024
nodes drawn in the slab |x - 95.5| < 40 where the droplets meet, 512 drawn
from the rest), and the oracle's integrals over the fluid nodes.  The
script calls only the oracle and the seeded input generators.  Run from the
repository root: python tests/golden/make_p5_collision.py (about half an
hour on eight threads)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import workloads as WL  # noqa: E402
import oracle as O  # noqa: E402
from _common import fluid_mask, oracle_params  # noqa: E402

CHECKPOINTS = (100, 750)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "p5_head_on_collision_192.json")


def sample_nodes(box):
    m = fluid_mask(box)
    nz, ny, nx = box.shape
    pts = [(47, 47, x) for x in range(nx)] + [(48, 48, x) for x in range(nx)]
    rng = np.random.Generator(np.random.PCG64(5))
    z, y, x = np.nonzero(m)
    near = np.abs(x - (nx - 1) / 2.0) < 40
    for sel, count in ((near, 1024), (~near, 512)):
        idx = rng.choice(np.flatnonzero(sel), size=count, replace=False)
        pts += [(int(z[i]), int(y[i]), int(x[i])) for i in idx]
    return pts


def record(o, pts, m):
    zz, yy, xx = (np.array(c) for c in zip(*pts))
    rho = o["rho_r"] + o["rho_b"]
    return {
        "fields": {k: [float(v) for v in o[k][zz, yy, xx]]
                   for k in ("rho_r", "rho_b", "ux", "uy", "uz", "phi")},
        "integrals": {
            "mass_r": float(o["rho_r"][m].sum()),
            "mass_b": float(o["rho_b"][m].sum()),
            "momentum": [float((rho * o[k])[m].sum()) for k in ("ux", "uy", "uz")],
            "kinetic_energy": float((0.5 * rho * (o["ux"] ** 2 + o["uy"] ** 2 + o["uz"] ** 2))[m].sum()),
            "red_volume": float(((1.0 + o["phi"]) / 2.0)[m].sum()),
        },
    }


def main():
    w = WL.head_on_collision(nx=192, ny=96, nz=96, R=12.0)
    P = oracle_params(w.box)
    f = O.init(P, w.rho_r.astype(np.float64), w.rho_b.astype(np.float64),
               w.u.astype(np.float64), seed=w.seed, amp=w.noise, box=0)
    pts = sample_nodes(w.box)
    m = fluid_mask(w.box)
    out = {"what": "FP64 oracle, walled head-on collision 192x96x96, R 12",
           "nodes_zyx": [list(p) for p in pts], "checkpoints": {}}
    done = 0
    for n in CHECKPOINTS:
        O.step(P, f, n - done)
        done = n
        out["checkpoints"][str(n)] = record(O.fields(P, f), pts, m)
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
