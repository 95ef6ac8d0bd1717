"""Python binding of the gfx950 colour-gradient LBM library (libcglbm.so).

Argument marshalling only: every step of the time update runs in the HIP
kernels behind the C ABI of ``include/cglbm.h``.  PyTorch provides device
memory and the stream.  There is no fallback: if the library is missing or
no GPU is present, the calls raise.

Layout of the concatenated node arrays: box b occupies nodes
``[offset(b), offset(b) + nx*ny*nz)`` with x fastest; gaps between boxes are
ignored by the library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcglbm.so")

CGLBM_OK = 0
ERRORS = {-1: "CGLBM_EINVAL", -2: "CGLBM_EHIP", -3: "CGLBM_EUNSUPPORTED",
          -4: "CGLBM_EUNSTABLE", -5: "CGLBM_ESTATE"}
FP32, FP16_SHIFT, BF16_SHIFT, FP32_EXACT, FP32_PAIRS, FP16_CSHIFT, BF16_CSHIFT = range(7)
STORAGE_NAMES = {FP32: "fp32", FP16_SHIFT: "fp16_shift", BF16_SHIFT: "bf16_shift",
                 FP32_EXACT: "fp32_exact", FP32_PAIRS: "fp32_pairs", FP16_CSHIFT: "fp16_cshift",
                 BF16_CSHIFT: "bf16_cshift"}
NDIAG = 13
DIAG_NAMES = ("M_r", "M_b", "Px", "Py", "Pz", "p_in", "p_out", "R_eff", "cx", "cy", "cz",
              "KE", "n_nonfinite")
FIELDS = ("rho_r", "rho_b", "phi", "p", "ux", "uy", "uz", "nx", "ny", "nz", "kappa",
          "Fx", "Fy", "Fz", "Qx", "Qy", "Qz")
KERNEL_KINDS = ("pull", "interface", "collide", "fused", "pull_first", "emit")

EXPORTED = ("cglbm_query_sizes", "cglbm_init", "cglbm_step", "cglbm_moments", "cglbm_reduce",
            "cglbm_box_offset", "cglbm_set_schedule", "cglbm_get_schedule", "cglbm_set_graph",
            "cglbm_num_variants",
            "cglbm_variant_info", "cglbm_set_variant", "cglbm_get_variant", "cglbm_autotune",
            "cglbm_profile_begin", "cglbm_profile_end", "cglbm_destroy",
            "cglbm_last_error", "cglbm_version", "cglbm_query_sizes_d2q9", "cglbm_init_d2q9",
            "cglbm_lattice", "cglbm_variant_info_d2q9", "cglbm_state_buffer",
            "cglbm_load_state", "cglbm_compact_variant", "cglbm_set_compact_variant",
            "cglbm_reduce_noalloc", "cglbm_set_wall_mode", "cglbm_get_wall_mode",
            "cglbm_set_resident", "cglbm_get_resident", "cglbm_sync_state")
# Lattices: the D3Q27 model of the paper's body and the D2Q9 model of App. A.
LATTICES = ("d3q27", "d2q9")
NUM_VARIANTS_D2Q9 = 4


class CglbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (ERRORS.get(code, str(code)), msg))
        self.code = code


class Phase(C.Structure):
    _fields_ = [("rho0", C.c_double), ("alpha", C.c_double), ("nu", C.c_double)]


class BoxParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("walls", C.c_uint32),
                ("red", Phase), ("blue", Phase), ("sigma", C.c_double), ("beta", C.c_double),
                ("omega_bulk", C.c_double), ("omega_hi", C.c_double * 9),
                ("body_force", C.c_double * 3), ("model", C.c_int32), ("q_correction", C.c_int32),
                ("gravity", C.c_double * 3), ("rho_ref", C.c_double)]


# equilibrium families of Table I (cglbm_model)
MODEL_A, MODEL_B, MODEL_C, MODEL_D = 0, 1, 2, 3


def box_params(nx, ny, nz, rho0_r, rho0_b, alpha_r, alpha_b, nu_r, nu_b, sigma, beta,
               omega_bulk=1.0, body_force=(0.0, 0.0, 0.0), walls=0, omega_hi=(1.0,) * 9,
               model=MODEL_D, q_correction=1, gravity=(0.0, 0.0, 0.0), rho_ref=0.0):
    p = BoxParams()
    p.model, p.q_correction = int(model), int(q_correction)
    p.gravity = (C.c_double * 3)(*[float(v) for v in gravity])
    p.rho_ref = float(rho_ref)
    p.nx, p.ny, p.nz, p.walls = int(nx), int(ny), int(nz), int(walls)
    p.red = Phase(float(rho0_r), float(alpha_r), float(nu_r))
    p.blue = Phase(float(rho0_b), float(alpha_b), float(nu_b))
    p.sigma, p.beta, p.omega_bulk = float(sigma), float(beta), float(omega_bulk)
    p.omega_hi = (C.c_double * 9)(*[float(v) for v in omega_hi])
    p.body_force = (C.c_double * 3)(*[float(v) for v in body_force])
    return p


def box_params_of(box) -> BoxParams:
    """BoxParams from any object with the attributes of a box description."""
    return box_params(box.nx, box.ny, box.nz, box.rho0_r, box.rho0_b, box.alpha_r, box.alpha_b,
                      box.nu_r, box.nu_b, box.sigma, box.beta, getattr(box, "omega_bulk", 1.0),
                      getattr(box, "body_force", (0.0, 0.0, 0.0)), getattr(box, "walls", 0),
                      omega_hi=getattr(box, "omega_hi", (1.0,) * 9),
                      model=getattr(box, "model", MODEL_D),
                      q_correction=getattr(box, "use_q", 1),
                      gravity=getattr(box, "gravity", (0.0, 0.0, 0.0)),
                      rho_ref=getattr(box, "rho_ref", 0.0))


_lib = None


def lib():
    """Load libcglbm.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcglbm.so is not built; run __graft_entry__.build() "
                              "or python paper_2309_07801_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32
        BP = C.POINTER(BoxParams)
        L.cglbm_query_sizes.argtypes = [i32, BP, i32, C.POINTER(C.c_size_t),
                                        C.POINTER(C.c_size_t), C.POINTER(i64)]
        L.cglbm_init.argtypes = [C.POINTER(vp), i32, BP, i32, vp, vp, vp, vp, vp, vp,
                                 C.c_uint64, C.c_double, vp]
        L.cglbm_query_sizes_d2q9.argtypes = L.cglbm_query_sizes.argtypes
        L.cglbm_init_d2q9.argtypes = L.cglbm_init.argtypes
        L.cglbm_lattice.argtypes = [vp]
        L.cglbm_variant_info_d2q9.argtypes = [i32, C.POINTER(i32)]
        L.cglbm_step.argtypes = [vp, i32, vp]
        L.cglbm_moments.argtypes = [vp, i32, u32, vp, vp]
        L.cglbm_reduce.argtypes = [vp, C.POINTER(C.c_double), vp, i32, vp]
        L.cglbm_reduce_noalloc.argtypes = [vp, vp, vp, vp]
        L.cglbm_box_offset.argtypes = [vp, i32]
        L.cglbm_box_offset.restype = i64
        L.cglbm_compact_variant.argtypes = [vp, C.POINTER(i32)]
        L.cglbm_set_compact_variant.argtypes = [vp, i32, vp]
        L.cglbm_state_buffer.argtypes = [vp]
        L.cglbm_state_buffer.restype = vp
        L.cglbm_load_state.argtypes = [vp, vp, vp]
        L.cglbm_set_schedule.argtypes = [vp, i32]
        L.cglbm_set_resident.argtypes = [vp, i32, vp]
        L.cglbm_get_resident.argtypes = [vp]
        L.cglbm_sync_state.argtypes = [vp, vp]
        L.cglbm_get_schedule.argtypes = [vp]
        L.cglbm_set_graph.argtypes = [vp, i32]
        L.cglbm_num_variants.argtypes = []
        L.cglbm_variant_info.argtypes = [i32, C.POINTER(i32)]
        L.cglbm_set_variant.argtypes = [vp, i32, vp]
        L.cglbm_get_variant.argtypes = [vp]
        L.cglbm_set_wall_mode.argtypes = [vp, i32, vp]
        L.cglbm_get_wall_mode.argtypes = [vp]
        L.cglbm_autotune.argtypes = [vp, i32, C.POINTER(C.c_double), vp]
        L.cglbm_profile_begin.argtypes = [vp, i32]
        L.cglbm_profile_end.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64), i32]
        L.cglbm_destroy.argtypes = [vp]
        L.cglbm_destroy.restype = None
        L.cglbm_last_error.restype = C.c_char_p
        L.cglbm_version.restype = C.c_char_p
        for fn in ("cglbm_query_sizes", "cglbm_init", "cglbm_query_sizes_d2q9", "cglbm_init_d2q9",
                   "cglbm_lattice", "cglbm_variant_info_d2q9", "cglbm_step", "cglbm_moments",
                   "cglbm_reduce", "cglbm_reduce_noalloc", "cglbm_set_schedule", "cglbm_get_schedule", "cglbm_set_graph",
                   "cglbm_num_variants",
                   "cglbm_variant_info", "cglbm_set_variant", "cglbm_get_variant",
                   "cglbm_set_wall_mode", "cglbm_get_wall_mode", "cglbm_autotune", "cglbm_profile_begin", "cglbm_profile_end"):
            getattr(L, fn).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != CGLBM_OK:
        raise CglbmError(rc, lib().cglbm_last_error().decode())


def query_sizes(params: Sequence[BoxParams], storage: int = FP32, lattice: str = "d3q27"):
    arr = (BoxParams * len(params))(*params)
    pop, aux, tot = C.c_size_t(), C.c_size_t(), C.c_int64()
    fn = lib().cglbm_query_sizes_d2q9 if _lattice_id(lattice) == 1 else lib().cglbm_query_sizes
    _check(fn(len(params), arr, storage, C.byref(pop), C.byref(aux), C.byref(tot)))
    return pop.value, aux.value, tot.value


def _lattice_id(lattice: str) -> int:
    if lattice not in LATTICES:
        raise ValueError("lattice must be one of %s" % (LATTICES,))
    return LATTICES.index(lattice)


def num_variants() -> int:
    return int(lib().cglbm_num_variants())


def variant_info(v: int, lattice: str = "d3q27"):
    info = (C.c_int32 * 4)()
    if _lattice_id(lattice) == 1:
        _check(lib().cglbm_variant_info_d2q9(int(v), info))
        return {"tx": info[0], "ty": info[1]}
    _check(lib().cglbm_variant_info(int(v), info))
    return {"tx": info[0], "ty": info[1], "zc": info[2], "min_waves": info[3]}


def _stream_ptr(stream) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Simulation:
    """A batch of independent boxes advanced together on one GPU.

    rho_r, rho_b: per-box float arrays of shape (nz, ny, nx); u: per-box
    (3, nz, ny, nx).  They are packed into the concatenated layout and copied
    to the device once for the initialisation.  lattice "d2q9" runs the
    two-dimensional model of App. A on boxes with nz = 1 (u may then have
    two components).  inplace=True keeps one population buffer (D3Q27 with
    unit higher-order rates; bitwise the same results).
    """

    def __init__(self, params: Sequence[BoxParams], rho_r: List[np.ndarray],
                 rho_b: List[np.ndarray], u: List[np.ndarray], seed: int = 0,
                 noise: float = 0.0, storage: int = FP32, device: int = 0, stream=None,
                 lattice: str = "d3q27", inplace: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the colour-gradient LBM library needs an MI355X")
        self.lattice = lattice
        lat = _lattice_id(lattice)
        self.params = list(params)
        self.nboxes = len(self.params)
        self.storage = storage
        self.device = torch.device("cuda", device)
        pop_bytes, aux_bytes, total = query_sizes(self.params, storage, lattice)
        self.total = total
        self.stream = stream
        dev = self.device
        self.inplace = bool(inplace)
        # zeroed, so that the padding between boxes (never read or written by
        # the kernels) is the same in every run and checkpoints compare bytewise
        self.pop_a = torch.zeros(pop_bytes, dtype=torch.uint8, device=dev)
        self.pop_b = None if self.inplace else torch.zeros(pop_bytes, dtype=torch.uint8, device=dev)
        self.aux = torch.empty(aux_bytes, dtype=torch.uint8, device=dev)
        self.offsets = self._offsets_host()
        rr = self.pack([np.asarray(a, np.float32) for a in rho_r])
        rb = self.pack([np.asarray(a, np.float32) for a in rho_b])
        uu = np.zeros((3, total), np.float32)
        for a in range(3):
            uu[a] = self.pack([np.asarray(x, np.float32)[a] if a < len(x) else
                               np.zeros(p.nx * p.ny * p.nz, np.float32)
                               for x, p in zip(u, self.params)])
        self._init_rr = torch.from_numpy(rr).to(dev)
        self._init_rb = torch.from_numpy(rb).to(dev)
        self._init_u = torch.from_numpy(uu).to(dev)
        arr = (BoxParams * self.nboxes)(*self.params)
        h = C.c_void_p()
        init = lib().cglbm_init_d2q9 if lat == 1 else lib().cglbm_init
        _check(init(C.byref(h), self.nboxes, arr, storage, self.pop_a.data_ptr(),
                                None if self.inplace else self.pop_b.data_ptr(), self.aux.data_ptr(),
                                self._init_rr.data_ptr(), self._init_rb.data_ptr(),
                                self._init_u.data_ptr(), C.c_uint64(seed), float(noise),
                                _stream_ptr(stream)))
        self.h = h
        self.steps_done = 0

    def _offsets_host(self):
        off, out = 0, []
        for p in self.params:
            out.append(off)
            n = p.nx * p.ny * p.nz
            off = (off + n + 63) // 64 * 64
        return out

    def pack(self, arrays: List[np.ndarray]) -> np.ndarray:
        out = np.zeros(self.total, np.float32)
        for b, a in enumerate(arrays):
            p = self.params[b]
            n = p.nx * p.ny * p.nz
            out[self.offsets[b]:self.offsets[b] + n] = np.asarray(a, np.float32).reshape(n)
        return out

    def box_offset(self, b: int) -> int:
        return int(lib().cglbm_box_offset(self.h, b))

    def state_tensor(self):
        """The population buffer that holds the current state (a view, valid
        until the next step); a resident compact state is stored first."""
        self.sync_state()
        ptr = lib().cglbm_state_buffer(self.h)
        if ptr == self.pop_a.data_ptr():
            return self.pop_a
        if self.pop_b is not None and ptr == self.pop_b.data_ptr():
            return self.pop_b
        raise CglbmError(-5, "state buffer is neither population buffer")

    def checkpoint(self):
        """A device copy of the current state (ordered on the simulation's
        stream after the work enqueued so far)."""
        import contextlib
        import torch
        ctx = torch.cuda.stream(self.stream) if self.stream is not None else contextlib.nullcontext()
        with ctx:
            return self.state_tensor().clone()

    def load_state(self, state):
        """Continue from a checkpoint taken on a simulation with the same
        boxes, storage and lattice."""
        if state.numel() != self.pop_a.numel() or state.device != self.device:
            raise ValueError("checkpoint size or device does not match this simulation")
        _check(lib().cglbm_load_state(self.h, state.data_ptr(), _stream_ptr(self.stream)))

    def step(self, n: int = 1):
        _check(lib().cglbm_step(self.h, int(n), _stream_ptr(self.stream)))
        self.steps_done += n

    def moments(self, box: int = 0, fields: Sequence[str] = FIELDS):
        import torch
        mask = 0
        for f in fields:
            mask |= 1 << FIELDS.index(f)
        names = [f for f in FIELDS if mask & (1 << FIELDS.index(f))]
        p = self.params[box]
        out = torch.empty((len(names), p.nz, p.ny, p.nx), dtype=torch.float32, device=self.device)
        _check(lib().cglbm_moments(self.h, box, mask, out.data_ptr(), _stream_ptr(self.stream)))
        return {n: out[k] for k, n in enumerate(names)}

    def reduce(self, centres: Optional[Sequence[Sequence[float]]] = None) -> np.ndarray:
        out = np.zeros((self.nboxes, NDIAG), np.float64)
        cptr = None
        if centres is not None:
            c = np.ascontiguousarray(np.asarray(centres, np.float64).reshape(self.nboxes, 3))
            cptr = c.ctypes.data_as(C.POINTER(C.c_double))
        rc = lib().cglbm_reduce(self.h, cptr, out.ctypes.data, 1, _stream_ptr(self.stream))
        if rc not in (CGLBM_OK, -4):
            _check(rc)
        self.last_reduce_unstable = (rc == -4)
        return out

    def reduce_device(self, centres: Optional[Sequence[Sequence[float]]] = None):
        """The diagnostics of reduce() into a new device tensor of shape
        (n_boxes, NDIAG), float64, enqueued on the simulation's stream with no
        host synchronization; column 12 holds the non-finite counts."""
        import torch
        out = torch.empty((self.nboxes, NDIAG), dtype=torch.float64, device=self.device)
        cptr = None
        if centres is not None:
            c = np.ascontiguousarray(np.asarray(centres, np.float64).reshape(self.nboxes, 3))
            cptr = c.ctypes.data_as(C.POINTER(C.c_double))
        _check(lib().cglbm_reduce(self.h, cptr, out.data_ptr(), 0, _stream_ptr(self.stream)))
        return out

    def reduce_noalloc(self, out, centres=None):
        """The diagnostics into the caller's device tensor `out` (n_boxes x
        NDIAG float64) through the allocation-free entry point (static
        scratch; usable under graph capture).  centres: device tensor of
        n_boxes x 3 doubles or None."""
        _check(lib().cglbm_reduce_noalloc(self.h, None if centres is None else centres.data_ptr(),
                                          out.data_ptr(), _stream_ptr(self.stream)))
        return out

    def profile_begin(self, max_launches: int):
        _check(lib().cglbm_profile_begin(self.h, int(max_launches)))

    def set_variant(self, v: int):
        _check(lib().cglbm_set_variant(self.h, int(v), _stream_ptr(self.stream)))

    def variant(self) -> int:
        return int(lib().cglbm_get_variant(self.h))

    def set_wall_mode(self, mode: int):
        """Wall mode of the tiled launches over boxes with walls: bit 0 short
        z-edge chunks, bit 1 the near-wall launch on a side stream."""
        _check(lib().cglbm_set_wall_mode(self.h, int(mode), _stream_ptr(self.stream)))

    def wall_mode(self) -> int:
        return int(lib().cglbm_get_wall_mode(self.h))

    def set_compact_variant(self, v: int):
        _check(lib().cglbm_set_compact_variant(self.h, int(v), _stream_ptr(self.stream)))

    def compact_variant(self):
        """Column tile and z chunk of the compact schedule's pull."""
        info = (C.c_int32 * 3)()
        v = int(lib().cglbm_compact_variant(self.h, info))
        return {"index": v, "tx": info[0], "ty": info[1], "zc": info[2]}

    def autotune(self, reps: int = 5):
        """Time every fused launch geometry and the three-kernel schedule and
        keep the fastest; returns the mean milliseconds per fused variant,
        then of the three-kernel schedule (D2Q9: per tile shape).  In the
        in-place layout the call advances the state by one step."""
        n = num_variants() + 1
        ms = (C.c_double * n)()
        _check(lib().cglbm_autotune(self.h, int(reps), ms, _stream_ptr(self.stream)))
        if self.inplace:
            self.steps_done += 1
        return list(ms)[:NUM_VARIANTS_D2Q9] if self.lattice == "d2q9" else list(ms)

    def set_schedule(self, schedule: int):
        _check(lib().cglbm_set_schedule(self.h, int(schedule)))

    def set_resident(self, enable: bool):
        """Keep the compact schedule's state resident between step calls
        (True) or store it as populations after each call (False, default)."""
        _check(lib().cglbm_set_resident(self.h, 1 if enable else 0, _stream_ptr(self.stream)))

    def resident(self) -> bool:
        return int(lib().cglbm_get_resident(self.h)) == 1

    def sync_state(self):
        """Store a resident compact state as populations in the state buffer."""
        _check(lib().cglbm_sync_state(self.h, _stream_ptr(self.stream)))

    def schedule(self) -> int:
        """Schedule in use: 0 fused, 1 three kernels, 2 compact."""
        return int(lib().cglbm_get_schedule(self.h))

    def set_graph(self, enable: bool):
        """Run pairs of steps as a captured HIP graph (default) or launch
        every kernel directly; results are bitwise identical."""
        _check(lib().cglbm_set_graph(self.h, int(bool(enable))))

    def profile_end(self):
        n = len(KERNEL_KINDS)
        ms = (C.c_double * n)()
        cnt = (C.c_int64 * n)()
        _check(lib().cglbm_profile_end(self.h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_KINDS)}

    def close(self):
        if getattr(self, "h", None):
            lib().cglbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
