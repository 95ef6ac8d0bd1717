"""Shared helpers of the tests: run the HIP path and the FP64 oracle on the
same seeded inputs and measure their differences (error norms of density,
velocity and order parameter as relative or absolute maxima)."""
import json
import os

import numpy as np

import oracle as O
import workloads as WL
from oracle import d2q9 as O2


def oracle_params(box: WL.Box, **kw) -> O.Params:
    d = dict(nx=box.nx, ny=box.ny, nz=box.nz, rho0_r=box.rho0_r, rho0_b=box.rho0_b,
             alpha_r=box.alpha_r, alpha_b=box.alpha_b, nu_r=box.nu_r, nu_b=box.nu_b,
             sigma=box.sigma, beta=box.beta, walls=box.walls, body_force=tuple(box.body_force),
             model=box.model, use_q=box.use_q, gravity=tuple(box.gravity), rho_ref=box.rho_ref,
             omega=(box.omega_hi[0], 1.0, box.omega_bulk) + tuple(box.omega_hi[1:]))
    d.update(kw)
    return O.Params(**d)


def run_oracle(box: WL.Box, rr, rb, u, steps, seed=0, noise=0.0, box_index=0):
    P = oracle_params(box)
    f = O.init(P, np.asarray(rr, np.float64), np.asarray(rb, np.float64),
               np.asarray(u, np.float64), seed=seed, amp=noise, box=box_index)
    if steps:
        O.step(P, f, steps)
    return O.fields(P, f), f


def gpu_fields(sim, box_index=0):
    import torch
    out = {k: v.double().cpu().numpy() for k, v in sim.moments(box_index).items()}
    torch.cuda.synchronize()
    return out


def fluid_mask(box: WL.Box):
    m = np.ones(box.shape, bool)
    if box.walls & 1:
        m[:, 0, :] = False
        m[:, -1, :] = False
    if box.walls & 2:
        m[0, :, :] = False
        m[-1, :, :] = False
    return m


def errors(g, o, box: WL.Box, u_ref: float):
    """e_rho = max |d rho| / rho_oracle; e_u = max |d u|_2 / u_ref;
    e_phi = max |d phi|, over fluid nodes."""
    m = fluid_mask(box)
    rho_g = g["rho_r"] + g["rho_b"]
    rho_o = o["rho_r"] + o["rho_b"]
    du = np.sqrt((g["ux"] - o["ux"]) ** 2 + (g["uy"] - o["uy"]) ** 2 + (g["uz"] - o["uz"]) ** 2)
    return {
        "rho": float((np.abs(rho_g - rho_o) / rho_o)[m].max()),
        "rho_r": float(np.abs(g["rho_r"] - o["rho_r"])[m].max() / box.rho0_r),
        "rho_b": float(np.abs(g["rho_b"] - o["rho_b"])[m].max() / box.rho0_b),
        "u": float(du[m].max() / u_ref),
        "phi": float(np.abs(g["phi"] - o["phi"])[m].max()),
        "rho_l2": float(np.sqrt((((rho_g - rho_o) / rho_o)[m] ** 2).mean())),
        "u_l2": float(np.sqrt((du[m] ** 2).mean()) / u_ref),
    }


# FP32 bar of the error measures below (e_rho relative, e_u against U_ref,
# e_phi absolute)
FP32_BAR = 1e-5
# unit roundoff of the 16-bit storage formats (by storage id)
UNIT_ROUNDOFF_16 = {1: 2.0 ** -11, 5: 2.0 ** -11, 2: 2.0 ** -8, 6: 2.0 ** -8}


def bars_16bit(storage):
    """(e_rho, e_u, e_phi) bars of a 16-bit storage format: 8 u_s for the
    density and phi and 32 u_s for the velocity (a momentum error divided by
    a velocity scale 10-25 times smaller than the populations), u_s the
    format's unit roundoff."""
    us = UNIT_ROUNDOFF_16[storage]
    return 8 * us, 32 * us, 8 * us


def u_ref(box: WL.Box, U: float) -> float:
    """Velocity scale of e_u: the imposed velocity U or the capillary scale
    sigma / mu_max, whichever is larger."""
    return max(U, box.sigma / max(box.rho0_r * box.nu_r, box.rho0_b * box.nu_b))


def log_parity(key, value):
    """Append a measured error record to the JSON file named by
    CGLBM_PARITY_LOG (if set)."""
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


def check(e, ctx="", rho=FP32_BAR, u=FP32_BAR, phi=FP32_BAR):
    """Log the error record under the running test's id (and ctx), then hold
    it to the bars."""
    name = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    if ctx != "":
        name += ":%s" % (ctx,)
    log_parity(name, e)
    assert e["rho"] <= rho and e["u"] <= u and e["phi"] <= phi, (name, e)


# ---- two-dimensional (D2Q9) boxes: workloads.Box with nz = 1 ----

def oracle_params_2d(box: WL.Box, **kw) -> O2.Params:
    d = dict(nx=box.nx, ny=box.ny, rho0_r=box.rho0_r, rho0_b=box.rho0_b, alpha_r=box.alpha_r,
             alpha_b=box.alpha_b, nu_r=box.nu_r, nu_b=box.nu_b, sigma=box.sigma, beta=box.beta,
             walls=box.walls, body_force=tuple(box.body_force[:2]), use_q=box.use_q,
             omega=(1.0, 1.0, box.omega_bulk, 1.0, 1.0))
    d.update(kw)
    return O2.Params(**d)


def run_oracle_2d(box: WL.Box, rr, rb, u, steps, seed=0, noise=0.0, box_index=0):
    """Oracle fields as (1, ny, nx) arrays (the shape of the GPU's fields),
    with zero z components."""
    P = oracle_params_2d(box)
    sh = (box.ny, box.nx)
    f = O2.init(P, np.asarray(rr, np.float64).reshape(sh), np.asarray(rb, np.float64).reshape(sh),
                np.asarray(u, np.float64)[:2].reshape((2,) + sh), seed=seed, amp=noise,
                box=box_index)
    if steps:
        O2.step(P, f, steps)
    F = {k: v.reshape((1,) + sh) for k, v in O2.fields(P, f).items()}
    for k in ("uz", "nz", "Fz", "Qz"):
        F[k] = np.zeros((1,) + sh)
    return F, f
