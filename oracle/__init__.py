"""FP64 CPU oracle for the two-colour D3Q27 colour-gradient LBM step with
generalized equilibria (Saito et al., arXiv:2309.07801).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product path
(the HIP library and its Python binding) never imports, links or executes it,
and the two share no code.

This module is a thin ctypes wrapper around ``cglbm_oracle.c``; all of the
method's arithmetic lives in that C file.  Arrays use the layout
``f[colour, i, z, y, x]`` (colour 0 red, 1 blue; i in the velocity order of
Eq. 1), float64, C-contiguous.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

from . import build as _build

MODEL_A, MODEL_B, MODEL_C, MODEL_D = 0, 1, 2, 3
NQ = 27
FIELD_NAMES = ("rho_r", "rho_b", "phi", "p", "ux", "uy", "uz", "nx", "ny", "nz",
               "kappa", "Fx", "Fy", "Fz", "Qx", "Qy", "Qz")


class _CParams(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("walls", C.c_uint32), ("model", C.c_int32), ("use_q", C.c_int32),
        ("rho0_r", C.c_double), ("rho0_b", C.c_double),
        ("alpha_r", C.c_double), ("alpha_b", C.c_double),
        ("nu_r", C.c_double), ("nu_b", C.c_double),
        ("sigma", C.c_double), ("beta", C.c_double),
        ("omega", C.c_double * 11), ("body_force", C.c_double * 3),
        ("gravity", C.c_double * 3), ("rho_ref", C.c_double),
    ]


@dataclasses.dataclass
class Params:
    """Physical parameters of one box, in the paper's terms."""
    nx: int
    ny: int
    nz: int
    rho0_r: float
    rho0_b: float
    alpha_r: float
    alpha_b: float
    nu_r: float
    nu_b: float
    sigma: float
    beta: float
    omega: tuple = (1.0,) * 11          # omega_0..omega_10; omega_1 is per node
    body_force: tuple = (0.0, 0.0, 0.0)
    gravity: tuple = (0.0, 0.0, 0.0)   # buoyancy force -(rho - rho_ref) g, Sec. IV.E
    rho_ref: float = 0.0
    walls: int = 0
    model: int = MODEL_D
    use_q: int = 1

    def c(self) -> _CParams:
        cp = _CParams()
        for name in ("nx", "ny", "nz", "walls", "model", "use_q", "rho0_r", "rho0_b",
                     "alpha_r", "alpha_b", "nu_r", "nu_b", "sigma", "beta"):
            setattr(cp, name, getattr(self, name))
        cp.omega = (C.c_double * 11)(*[float(v) for v in self.omega])
        cp.body_force = (C.c_double * 3)(*[float(v) for v in self.body_force])
        cp.gravity = (C.c_double * 3)(*[float(v) for v in self.gravity])
        cp.rho_ref = float(self.rho_ref)
        return cp

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or any(
                os.path.getmtime(src) > os.path.getmtime(_build.LIB)
                for src in _build.SRC + [os.path.splitext(x)[0] + ".h" for x in _build.SRC]):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_CParams)
        L.orc_lattice.argtypes = [C.POINTER(C.c_int32), dp]
        L.orc_hermite.argtypes = [C.c_int32] * 4
        L.orc_hermite.restype = C.c_double
        L.orc_isotropic_E.argtypes = [C.c_int32]
        L.orc_isotropic_E.restype = C.c_double
        L.orc_feq.argtypes = [C.c_int32, C.c_double, C.c_double, dp, dp]
        L.orc_feq_standard_cg.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_feq_li_original.argtypes = [C.c_double, C.c_double, dp, dp]
        L.orc_raw_moments.argtypes = [dp, dp]
        L.orc_central_moments.argtypes = [dp, dp, dp]
        L.orc_cm_to_f.argtypes = [dp, dp, dp]
        L.orc_moment_matrix.argtypes = [dp]
        L.orc_inverse_moment_matrix.argtypes = [dp]
        L.orc_collide.argtypes = [C.c_int32, C.c_int32, dp, C.c_double, dp, C.c_double,
                                  dp, dp, dp, dp]
        L.orc_recolour.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, C.c_double,
                                   dp, dp]
        L.orc_sound_speed2.argtypes = [C.c_double]
        L.orc_sound_speed2.restype = C.c_double
        L.orc_splitmix64.argtypes = [C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_noise.argtypes = [C.c_uint64, C.c_int32, C.c_int64, C.c_int32, C.c_double]
        L.orc_noise.restype = C.c_double
        L.orc_gradient.argtypes = [P, dp, dp]
        L.orc_fields.argtypes = [P, dp, dp]
        L.orc_init.argtypes = [P, dp, dp, dp, C.c_uint64, C.c_double, C.c_int32, dp]
        L.orc_init_window.argtypes = [P, dp, dp, dp, C.c_uint64, C.c_double, C.c_int32,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp]
        L.orc_step.argtypes = [P, dp, C.c_int32]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int32]
        L.orc_set_num_threads.restype = None
        for fn in ("orc_gradient", "orc_fields", "orc_init", "orc_init_window", "orc_step"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vec(v, n=3) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(n))
    return a


# ---- lattice and node-level pieces -------------------------------------------------

def lattice():
    c = np.zeros((NQ, 3), dtype=np.int32)
    w = np.zeros(NQ)
    lib().orc_lattice(c.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return c, w


def hermite(i, a, b, c) -> float:
    return lib().orc_hermite(i, a, b, c)


def isotropic_E() -> np.ndarray:
    return np.array([lib().orc_isotropic_E(i) for i in range(NQ)])


def feq(model, rho, p, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_feq(model, rho, p, _dp(_vec(u)), _dp(out))
    return out


def feq_standard_cg(rho, p, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_feq_standard_cg(rho, p, _dp(_vec(u)), _dp(out))
    return out


def feq_li_original(rho, p, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_feq_li_original(rho, p, _dp(_vec(u)), _dp(out))
    return out


def raw_moments(f) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_raw_moments(_dp(_vec(f, NQ)), _dp(out))
    return out


def central_moments(f, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_central_moments(_dp(_vec(f, NQ)), _dp(_vec(u)), _dp(out))
    return out


def cm_to_f(k, u) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_cm_to_f(_dp(_vec(k, NQ)), _dp(_vec(u)), _dp(out))
    return out


def moment_matrix() -> np.ndarray:
    out = np.zeros((NQ, NQ))
    lib().orc_moment_matrix(_dp(out))
    return out


def inverse_moment_matrix() -> np.ndarray:
    out = np.zeros((NQ, NQ))
    lib().orc_inverse_moment_matrix(_dp(out))
    return out


def collide(model, use_q, f, rho, u, p, F, Q, omega) -> np.ndarray:
    out = np.zeros(NQ)
    lib().orc_collide(model, use_q, _dp(_vec(f, NQ)), rho, _dp(_vec(u)), p, _dp(_vec(F)),
                      _dp(_vec(Q)), _dp(_vec(omega, 11)), _dp(out))
    return out


def recolour(fstar, rho_r, rho_b, p, n, beta):
    fr = np.zeros(NQ)
    fb = np.zeros(NQ)
    lib().orc_recolour(_dp(_vec(fstar, NQ)), rho_r, rho_b, p, _dp(_vec(n)), beta, _dp(fr),
                       _dp(fb))
    return fr, fb


def sound_speed2(alpha) -> float:
    return lib().orc_sound_speed2(alpha)


def splitmix64(state: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(state & 0xFFFFFFFFFFFFFFFF)))


def noise(seed, box, node, i, amp) -> float:
    return lib().orc_noise(C.c_uint64(seed), box, node, i, amp)


# ---- grid level --------------------------------------------------------------------

def gradient(P: Params, chi: np.ndarray) -> np.ndarray:
    chi = np.ascontiguousarray(chi, dtype=np.float64).reshape(P.shape)
    out = np.zeros((3,) + P.shape)
    cp = P.c()
    rc = lib().orc_gradient(C.byref(cp), _dp(chi), _dp(out))
    assert rc == 0
    return out


def fields(P: Params, f: np.ndarray) -> dict:
    out = np.zeros((len(FIELD_NAMES),) + P.shape)
    cp = P.c()
    rc = lib().orc_fields(C.byref(cp), _dp(f), _dp(out))
    if rc != 0:
        raise MemoryError("orc_fields failed")
    return {name: out[k] for k, name in enumerate(FIELD_NAMES)}


def init(P: Params, rho_r, rho_b, u, seed=0, amp=0.0, box=0) -> np.ndarray:
    rho_r = np.ascontiguousarray(rho_r, dtype=np.float64).reshape(P.shape)
    rho_b = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(P.shape)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + P.shape)
    f = np.zeros((2, NQ) + P.shape)
    cp = P.c()
    rc = lib().orc_init(C.byref(cp), _dp(rho_r), _dp(rho_b), _dp(u), C.c_uint64(seed), amp,
                        box, _dp(f))
    if rc != 0:
        raise ValueError("orc_init: non-positive total density")
    return f


def init_window(P: Params, rho_r, rho_b, u, global_dims, offset, seed=0, amp=0.0,
                box=0) -> np.ndarray:
    """Initial state of a window of a larger periodic box (noise keyed by the
    larger box's node index).  global_dims, offset: (x, y, z)."""
    rho_r = np.ascontiguousarray(rho_r, dtype=np.float64).reshape(P.shape)
    rho_b = np.ascontiguousarray(rho_b, dtype=np.float64).reshape(P.shape)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + P.shape)
    f = np.zeros((2, NQ) + P.shape)
    cp = P.c()
    gd = (C.c_int32 * 3)(*[int(v) for v in global_dims])
    go = (C.c_int32 * 3)(*[int(v) for v in offset])
    rc = lib().orc_init_window(C.byref(cp), _dp(rho_r), _dp(rho_b), _dp(u), C.c_uint64(seed),
                               amp, box, gd, go, _dp(f))
    if rc != 0:
        raise ValueError("orc_init_window: non-positive total density")
    return f


def step(P: Params, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
    """Advance the pre-collision state f in place by nsteps steps."""
    assert f.shape == (2, NQ) + P.shape
    cp = P.c()
    rc = lib().orc_step(C.byref(cp), _dp(f), nsteps)
    if rc != 0:
        raise MemoryError("orc_step failed")
    return f


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    lib().orc_set_num_threads(int(n))
