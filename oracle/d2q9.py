"""FP64 CPU oracle for the two-colour D2Q9 colour-gradient LBM step with the
two-dimensional generalized equilibrium of App. A (Saito et al.,
arXiv:2309.07801).

TEST INFRASTRUCTURE ONLY, like the rest of this package: a thin ctypes
wrapper around ``d2q9_oracle.c``, where all of the arithmetic lives.  Arrays
use the layout ``f[colour, i, y, x]`` (colour 0 red, 1 blue; i in the
velocity order of Eq. A1), float64, C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import dataclasses

import numpy as np

from . import lib as _lib3

NQ = 9
FIELD_NAMES = ("rho_r", "rho_b", "phi", "p", "ux", "uy", "nx", "ny", "kappa", "Fx", "Fy",
               "Qx", "Qy")


class _CParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("walls", C.c_uint32), ("use_q", C.c_int32),
        ("rho0_r", C.c_double), ("rho0_b", C.c_double),
        ("alpha_r", C.c_double), ("alpha_b", C.c_double),
        ("nu_r", C.c_double), ("nu_b", C.c_double),
        ("sigma", C.c_double), ("beta", C.c_double),
        ("omega", C.c_double * 5), ("body_force", C.c_double * 2),
    ]


@dataclasses.dataclass
class Params:
    """Physical parameters of one two-dimensional box."""
    nx: int
    ny: int
    rho0_r: float
    rho0_b: float
    alpha_r: float
    alpha_b: float
    nu_r: float
    nu_b: float
    sigma: float
    beta: float
    omega: tuple = (1.0,) * 5       # omega_0, omega_1 (per node), omega_2, omega_3, omega_4
    body_force: tuple = (0.0, 0.0)
    walls: int = 0
    use_q: int = 1

    def c(self) -> _CParams:
        cp = _CParams()
        for name in ("nx", "ny", "walls", "use_q", "rho0_r", "rho0_b", "alpha_r", "alpha_b",
                     "nu_r", "nu_b", "sigma", "beta"):
            setattr(cp, name, getattr(self, name))
        cp.omega = (C.c_double * 5)(*[float(v) for v in self.omega])
        cp.body_force = (C.c_double * 2)(*[float(v) for v in self.body_force])
        return cp

    @property
    def shape(self):
        return (self.ny, self.nx)


_L = None


def lib():
    global _L
    if _L is None:
        L = _lib3()
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_CParams)
        L.orc2_lattice.argtypes = [C.POINTER(C.c_int32), dp]
        L.orc2_hermite.argtypes = [C.c_int32] * 3
        L.orc2_hermite.restype = C.c_double
        L.orc2_isotropic_E.argtypes = [C.c_int32]
        L.orc2_isotropic_E.restype = C.c_double
        L.orc2_xi.restype = C.c_double
        L.orc2_geq4.argtypes = [C.c_double, dp, dp]
        L.orc2_feq.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc2_central_moments.argtypes = [dp, dp, dp]
        L.orc2_raw_moments.argtypes = [dp, dp]
        L.orc2_cm_to_f.argtypes = [dp, dp, dp]
        L.orc2_collide.argtypes = [C.c_int32, dp, C.c_double, dp, C.c_double, dp, dp, dp, dp]
        L.orc2_recolour.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, C.c_double,
                                    dp, dp]
        L.orc2_noise.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_double]
        L.orc2_noise.restype = C.c_double
        L.orc2_fields.argtypes = [P, dp, dp]
        L.orc2_init.argtypes = [P, dp, dp, dp, C.c_uint64, C.c_double, C.c_int32, dp]
        L.orc2_step.argtypes = [P, dp, C.c_int32]
        L.orc2_init_window.argtypes = [P, dp, dp, dp, C.c_uint64, C.c_double, C.c_int32,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
        for fn in ("orc2_fields", "orc2_init", "orc2_init_window", "orc2_step"):
            getattr(L, fn).restype = C.c_int
        _L = L
    return _L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(v, n=2) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))


def lattice():
    c = np.zeros((NQ, 2), dtype=np.int32)
    w = np.zeros(NQ)
    lib().orc2_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return c, w


def hermite(i, a, b) -> float:
    return lib().orc2_hermite(i, a, b)


def isotropic_E() -> np.ndarray:
    return np.array([lib().orc2_isotropic_E(i) for i in range(NQ)])


def xi() -> float:
    return lib().orc2_xi()


def geq4(rho, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc2_geq4(rho, _dp(_vec(u)), _dp(out))
    return out


def feq(rho, p, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc2_feq(rho, p, _dp(_vec(u)), _dp(out))
    return out


def central_moments(f, u) -> np.ndarray:
    """k[a + 3 b] = sum_i f_i (cx - ux)^a (cy - uy)^b."""
    out = np.zeros(NQ)
    lib().orc2_central_moments(_dp(_vec(f, NQ)), _dp(_vec(u)), _dp(out))
    return out


def raw_moments(f) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc2_raw_moments(_dp(_vec(f, NQ)), _dp(out))
    return out


def cm_to_f(k, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc2_cm_to_f(_dp(_vec(k, NQ)), _dp(_vec(u)), _dp(out))
    return out


def collide(use_q, f, rho, u, p, F, Q, omega) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc2_collide(use_q, _dp(_vec(f, NQ)), rho, _dp(_vec(u)), p, _dp(_vec(F)),
                       _dp(_vec(Q)), _dp(_vec(omega, 5)), _dp(out))
    return out


def recolour(fstar, rho_r, rho_b, p, n, beta):
    fr = np.zeros(NQ)
    fb = np.zeros(NQ)
    lib().orc2_recolour(_dp(_vec(fstar, NQ)), rho_r, rho_b, p, _dp(_vec(n)), beta, _dp(fr),
                        _dp(fb))
    return fr, fb


def noise(seed, box, node, i, amp) -> float:
    return lib().orc2_noise(C.c_uint64(seed), box, node, i, amp)


def fields(P: Params, f: np.ndarray) -> dict:
    out = np.zeros((len(FIELD_NAMES),) + P.shape)
    cp = P.c()
    if lib().orc2_fields(C.byref(cp), _dp(f), _dp(out)) != 0:
        raise MemoryError("orc2_fields failed")
    return {name: out[k] for k, name in enumerate(FIELD_NAMES)}


def init(P: Params, rho_r, rho_b, u, seed=0, amp=0.0, box=0) -> np.ndarray:
    rho_r = np.ascontiguousarray(rho_r, dtype=np.float64).reshape(P.shape)
    rho_b = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(P.shape)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape((2,) + P.shape)
    f = np.zeros((2, NQ) + P.shape)
    cp = P.c()
    if lib().orc2_init(C.byref(cp), _dp(rho_r), _dp(rho_b), _dp(u), C.c_uint64(seed), amp, box,
                       _dp(f)) != 0:
        raise ValueError("orc2_init: non-positive total density")
    return f


def init_window(P: Params, rho_r, rho_b, u, global_dims, offset, seed=0, amp=0.0,
                box=0) -> np.ndarray:
    """Initial state of a window of a larger periodic box (noise keyed by the
    larger box's node index).  global_dims, offset: (x, y)."""
    rho_r = np.ascontiguousarray(rho_r, dtype=np.float64).reshape(P.shape)
    rho_b = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(P.shape)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape((2,) + P.shape)
    f = np.zeros((2, NQ) + P.shape)
    cp = P.c()
    gd = (C.c_int32 * 2)(*[int(v) for v in global_dims])
    go = (C.c_int32 * 2)(*[int(v) for v in offset])
    if lib().orc2_init_window(C.byref(cp), _dp(rho_r), _dp(rho_b), _dp(u), C.c_uint64(seed), amp,
                              box, gd, go, _dp(f)) != 0:
        raise ValueError("orc2_init_window: non-positive total density")
    return f


def step(P: Params, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
    """Advance the pre-collision state f in place by nsteps steps."""
    assert f.shape == (2, NQ) + P.shape
    cp = P.c()
    if lib().orc2_step(C.byref(cp), _dp(f), nsteps) != 0:
        raise MemoryError("orc2_step failed")
    return f
