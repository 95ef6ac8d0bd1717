"""Storage formats on the density-ratio-1000 sheared droplets (the 512^3
workload's physics at 96^3: eight droplets of radius U[4, 9], light carrier
with a sinusoidal shear of amplitude 0.04, equal kinematic viscosities from
Re = 1000, sigma = 1e-4, beta = 0.2), against the FP64 oracle after 200
steps, and the 16-bit formats against the FP32 run over 2000 steps by
their integral diagnostics (the oracle cannot afford that many steps in a
test).

Formats: FP32, FP32 mass-exact, FP16 and BF16 with the constant per-colour
shift, and FP16 and BF16 with the colour-fraction-scaled shift.  The
errors (A23 normalisation, U_ref = 0.04) are written to the JSON file named
by CGLBM_PARITY_LOG, if set, before the checks.

Bars (e_rho, e_u, e_phi), from the formats' rounding:
* FP32: 2 gamma 2^-24 = 1.2e-4 (gamma = 1000).  At a node of the light
  phase the heavy colour's populations (its tail, or for the mass-exact
  storage its shift) carry FP32 rounding of order 2^-24 of the heavy
  density, gamma times 2^-24 of the light one.
* 16-bit: 8 u_s for e_rho and e_phi and 32 u_s for e_u (u_s the format's
  unit roundoff, 2^-11 for FP16 and 2^-8 for BF16; e_u divides a momentum
  error by a velocity scale 10-25 times smaller than the populations).  The
  colour-fraction-scaled shift meets them (measured about 1-3 u_s); the
  constant shift misses them by an order of magnitude or more at this
  density ratio, which the test asserts too: it is the reason for the
  scaled form."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as WL
from _common import errors, gpu_fields, oracle_params

pytestmark = pytest.mark.gpu

STEPS = 200
U_REF = 0.04
NAMES = {0: "fp32", 3: "fp32_exact", 1: "fp16_shift", 2: "bf16_shift", 5: "fp16_cshift",
         6: "bf16_cshift"}
GAMMA = 1000.0
FP32_BAR = 2.0 * GAMMA * 2.0 ** -24
UNIT_ROUNDOFF = {1: 2.0 ** -11, 5: 2.0 ** -11, 2: 2.0 ** -8, 6: 2.0 ** -8}


def _bars(storage):
    """(e_rho, e_u, e_phi) after 200 steps against the oracle."""
    if storage in (0, 3):
        return FP32_BAR, FP32_BAR, FP32_BAR
    us = UNIT_ROUNDOFF[storage]
    return 8 * us, 32 * us, 8 * us


def _log(key, value):
    path = os.environ.get("CGLBM_PARITY_LOG")
    if not path:
        return
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data[key] = value
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


def _workload():
    return WL.sheared_droplets(n=96, count=8, rmin=4.0, rmax=9.0)


_ORACLE = {}


def _oracle():
    if "p3" not in _ORACLE:
        w = _workload()
        P = oracle_params(w.box)
        f = O.init(P, w.rho_r.astype(np.float64), w.rho_b.astype(np.float64),
                   w.u.astype(np.float64), seed=w.seed, amp=w.noise)
        O.step(P, f, STEPS)
        _ORACLE["p3"] = O.fields(P, f)
    return _ORACLE["p3"]


def _sim(w, storage):
    import paper_2309_07801_amd as pkg
    return pkg.Simulation([pkg.box_params_of(w.box)], [w.rho_r], [w.rho_b], [w.u], seed=w.seed,
                          noise=w.noise, storage=storage)


@pytest.mark.parametrize("storage", list(NAMES), ids=list(NAMES.values()))
def test_p3_storage_against_oracle(storage):
    w = _workload()
    sim = _sim(w, storage)
    d0 = sim.reduce()[0]
    sim.step(STEPS)
    g = gpu_fields(sim)
    d1 = sim.reduce()[0]
    sim.close()
    e = errors(g, _oracle(), w.box, U_REF)
    e["mass_drift"] = [(d1[k] - d0[k]) / d0[k] for k in (0, 1)]
    print(NAMES[storage], e)
    _log("p3_%s" % NAMES[storage], e)
    br, bu, bp = _bars(storage)
    ok = e["rho"] <= br and e["u"] <= bu and e["phi"] <= bp
    if storage in (1, 2):
        # the constant shift at density ratio 1000: outside the bar
        assert not ok and max(e["rho"] / br, e["u"] / bu, e["phi"] / bp) > 5, e
    else:
        assert ok, e


def test_p3_16bit_integrals_over_2000_steps():
    """Kinetic energy and per-colour mass of each 16-bit format against the
    FP32 run after 2000 steps."""
    w = _workload()
    out = {}
    for storage in (0, 1, 2, 5, 6):
        sim = _sim(w, storage)
        d0 = sim.reduce()[0]
        sim.step(2000)
        d1 = sim.reduce()[0]
        sim.close()
        out[storage] = (d0, d1)
    ke32 = out[0][1][11]
    res = {}
    for storage in (1, 2, 5, 6):
        d0, d1 = out[storage]
        res[NAMES[storage]] = {"ke_vs_fp32": float(d1[11] / ke32 - 1.0),
                               "mass_drift": [float((d1[k] - d0[k]) / d0[k]) for k in (0, 1)]}
    res["fp32_mass_drift"] = [float((out[0][1][k] - out[0][0][k]) / out[0][0][k]) for k in (0, 1)]
    print(res)
    _log("p3_2000_integrals", res)
    for storage in (1, 2, 5, 6):
        r = res[NAMES[storage]]
        assert abs(r["mass_drift"][0]) < 1e-12 and abs(r["mass_drift"][1]) < 1e-12
        assert np.isfinite(r["ke_vs_fp32"])
