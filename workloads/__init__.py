"""Seeded synthetic workloads for the colour-gradient LBM hot path.

This module builds *inputs only*: parameter sets expressed in the paper's
physical terms (reference densities, rest fractions alpha_k, kinematic
viscosities, sigma, beta, relaxation rates) and initial colour-density and
velocity fields (spheres of red fluid in blue fluid, uniform or sheared
carrier velocity).  It holds none of the method's update arithmetic and is
shared by the tests and the benchmark; the HIP path and the CPU oracle each
receive the same arrays and parameters.

Parameter conventions (readings of the paper where it leaves a choice):
  * the lighter phase takes alpha = 8/27, so its squared sound speed is 1/3
    (the bubble-rise set-up of Sec. IV uses this choice);
  * the heavier phase of density ratio g takes alpha = 1 - (19/27)/g, which
    makes the two ideal-gas pressures equal (Eq. 13 with xi = 9/19);
  * a relaxation time tau prescribed for a pure phase k sets its kinematic
    viscosity to (tau - 1/2) * xi * (1 - alpha_k) (Eq. 22 in a pure phase);
  * droplets are sharp: red density rho_r^0 where |x - x_c| <= R (periodic
    distance), blue density rho_b^0 elsewhere.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

XI = 9.0 / 19.0
ALPHA_LIGHT = 8.0 / 27.0


def alpha_heavy(gamma: float) -> float:
    """Rest fraction of the heavier phase for density ratio gamma >= 1."""
    return 1.0 - (19.0 / 27.0) / gamma


def sound2(alpha: float) -> float:
    return XI * (1.0 - alpha)


@dataclasses.dataclass
class Box:
    """One periodic (or walled) box and its physical parameters."""
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
    omega_bulk: float = 1.0
    body_force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    walls: int = 0
    model: int = 3        # equilibrium family of Table I: 0 A, 1 B, 2 C, 3 D
    use_q: int = 1        # correction term Q of Eq. (65)
    gravity: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # buoyancy -(rho - rho_ref) g
    rho_ref: float = 0.0
    omega_hi: Tuple[float, ...] = (1.0,) * 9   # omega_0, omega_3..omega_10 of Eq. (25)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nodes(self) -> int:
        return self.nx * self.ny * self.nz

    def fluid_nodes(self) -> int:
        ny = self.ny - 2 if (self.walls & 1) else self.ny
        nz = self.nz - 2 if (self.walls & 2) else self.nz
        return self.nx * ny * nz


@dataclasses.dataclass
class Workload:
    name: str
    box: Box
    rho_r: np.ndarray      # float32 [nz, ny, nx]
    rho_b: np.ndarray      # float32 [nz, ny, nx]
    u: np.ndarray          # float32 [3, nz, ny, nx]
    seed: int = 0
    noise: float = 0.0
    steps: int = 0
    centres: Optional[List[Tuple[float, float, float]]] = None
    radii: Optional[List[float]] = None


def two_phase_box(n: Sequence[int], gamma: float, rho_drop: float, tau: float,
                  sigma: float, beta: float, *, drop_is_heavy: bool = True,
                  visc_ratio_kin: Optional[float] = None, walls: int = 0,
                  omega_bulk: float = 1.0) -> Box:
    """Box with red droplet phase of density rho_drop and density ratio gamma.

    If ``visc_ratio_kin`` is None, tau is applied to both pure phases (equal
    dynamic viscosities); otherwise nu_r = tau-derived value of the red phase
    and nu_b = nu_r / visc_ratio_kin.
    """
    if gamma == 1.0:
        a_r = a_b = ALPHA_LIGHT
        rho_b = rho_drop
    elif drop_is_heavy:
        a_r, a_b = alpha_heavy(gamma), ALPHA_LIGHT
        rho_b = rho_drop / gamma
    else:
        a_r, a_b = ALPHA_LIGHT, alpha_heavy(gamma)
        rho_b = rho_drop * gamma
    nu_r = (tau - 0.5) * sound2(a_r)
    nu_b = (tau - 0.5) * sound2(a_b) if visc_ratio_kin is None else nu_r / visc_ratio_kin
    return Box(nx=n[0], ny=n[1], nz=n[2], rho0_r=rho_drop, rho0_b=rho_b, alpha_r=a_r,
               alpha_b=a_b, nu_r=nu_r, nu_b=nu_b, sigma=sigma, beta=beta,
               omega_bulk=omega_bulk, walls=walls)


def periodic_distance(shape_xyz, centre, walls=0):
    """Distance of every node to ``centre`` with periodic wrap on open axes."""
    nx, ny, nz = shape_xyz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    d = []
    for coord, c, n, periodic in ((x, centre[0], nx, True), (y, centre[1], ny, not (walls & 1)),
                                   (z, centre[2], nz, not (walls & 2))):
        dd = np.abs(coord - c)
        if periodic:
            dd = np.minimum(dd, n - dd)
        d.append(dd)
    return np.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)


def _sphere(box: Box, centre, r):
    """Nodes within distance r of centre, as index vectors (z, y, x) and a
    mask over their outer product.  Only the sphere's bounding box is
    visited; distances are formed as in periodic_distance."""
    axes = []
    for c, n, periodic in ((centre[0], box.nx, True), (centre[1], box.ny, not (box.walls & 1)),
                           (centre[2], box.nz, not (box.walls & 2))):
        lo, hi = int(math.floor(c - r)), int(math.ceil(c + r))
        if periodic:
            coord = np.arange(n) if hi - lo + 1 >= n else np.mod(np.arange(lo, hi + 1), n)
            dd = np.abs(coord - c)
            dd = np.minimum(dd, n - dd)
        else:
            coord = np.arange(max(lo, 0), min(hi, n - 1) + 1)
            dd = np.abs(coord - c)
        axes.append((coord, dd))
    (xc, dx), (yc, dy), (zc, dz) = axes
    d = np.sqrt(dx[None, None, :] ** 2 + dy[None, :, None] ** 2 + dz[:, None, None] ** 2)
    return (zc, yc, xc), d <= r


def droplet_fields(box: Box, centres, radii, u_drop=None, u_carrier=None):
    """Sharp droplets of red fluid in blue fluid; returns float32 arrays."""
    red = np.zeros(box.shape, dtype=bool)
    spheres = [_sphere(box, c, r) for c, r in zip(centres, radii)]
    for idx, m in spheres:
        sub = np.ix_(*idx)
        red[sub] |= m
    rho_r = np.where(red, box.rho0_r, 0.0).astype(np.float32)
    rho_b = np.where(red, 0.0, box.rho0_b).astype(np.float32)
    u = np.zeros((3,) + box.shape, dtype=np.float32)
    if u_carrier is not None:
        u[:] = np.asarray(u_carrier, dtype=np.float32).reshape(3, 1, 1, 1)
    if u_drop is not None:
        for (idx, m), ud in zip(spheres, u_drop):
            sub = np.ix_(*idx)
            for a in range(3):
                u[a][sub] = np.where(m, np.float32(ud[a]), u[a][sub])
    return rho_r, rho_b, u


# ---------------------------------------------------------------------------
# The five benchmark workloads and their reduced parity versions
# ---------------------------------------------------------------------------

def static_droplet(n: int = 32, R: float = 8.0, sigma: float = 0.01, tau: float = 1.0,
                   beta: float = 0.7, steps: int = 200) -> Workload:
    """Static droplet, density ratio 1, viscosity ratio 1 (Laplace-law case)."""
    box = two_phase_box((n, n, n), 1.0, 1.0, tau, sigma, beta)
    c = ((n - 1) / 2.0,) * 3
    rr, rb, u = droplet_fields(box, [c], [R])
    return Workload("static_droplet_%d" % n, box, rr, rb, u, steps=steps, centres=[c], radii=[R])


def translating_droplet(n: int = 256, R: float = 32.0, U: float = 0.05, gamma: float = 10.0,
                        omega_shear: float = 1.6, sigma: float = 0.005, beta: float = 0.7,
                        noise: float = 1e-6, seed: int = 2, steps: int = 5000) -> Workload:
    """Droplet translating with a uniform velocity U along x (Galilean case).

    Density ratio gamma (droplet heavier), equal dynamic viscosities, shear
    rate omega_shear in both pure phases, bulk rate 1."""
    tau = 1.0 / omega_shear
    box = two_phase_box((n, n, n), gamma, 1.0, tau, sigma, beta)
    c = ((n - 1) / 2.0,) * 3
    rr, rb, u = droplet_fields(box, [c], [R], u_carrier=(U, 0.0, 0.0))
    return Workload("translating_droplet_%d" % n, box, rr, rb, u, seed=seed, noise=noise,
                    steps=steps, centres=[c], radii=[R])


def place_droplets(n: int, count: int, rmin: float, rmax: float, gap: float, seed: int):
    """Rejection-sample non-overlapping droplets in a periodic cube."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres, radii = [], []
    tries = 0
    while len(centres) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place droplets")
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(0, n, size=3)
        ok = True
        for c2, r2 in zip(centres, radii):
            d = np.abs(c - np.asarray(c2))
            d = np.minimum(d, n - d)
            if np.sqrt((d ** 2).sum()) < r + r2 + gap:
                ok = False
                break
        if ok:
            centres.append(tuple(float(v) for v in c))
            radii.append(float(r))
    return centres, radii


def sheared_droplets(n: int = 512, count: int = 8, rmin: float = 20.0, rmax: float = 48.0,
                     gamma: float = 1000.0, U: float = 0.04, Re: float = 1000.0,
                     visc_ratio_dyn: float = 1000.0, sigma: float = 1e-4, beta: float = 0.2,
                     seed: int = 3, steps: int = 2000) -> Workload:
    """Several heavy droplets in a light carrier with a sinusoidal shear.

    Defaults: equal kinematic viscosities (dynamic ratio = density ratio) and
    sigma = 0.1 rho_light, the choices of the stationary-droplet tests at a
    density ratio of 1000 (Table II).  With a dynamic ratio of 10 (the heavy
    phase 100 times less viscous kinematically, relaxation time 1.1) or
    sigma = 0.005, the FP64 reference update diverges within a few tens of
    steps from sharp or tanh-smoothed droplets alike."""
    rho_r0, rho_b0 = 1.0, 1.0 / gamma
    nu_b = U * n / Re
    nu_r = visc_ratio_dyn * rho_b0 * nu_b / rho_r0
    box = Box(nx=n, ny=n, nz=n, rho0_r=rho_r0, rho0_b=rho_b0, alpha_r=alpha_heavy(gamma),
              alpha_b=ALPHA_LIGHT, nu_r=nu_r, nu_b=nu_b, sigma=sigma, beta=beta)
    centres, radii = place_droplets(n, count, rmin, rmax, 4.0, seed)
    rr, rb, u = droplet_fields(box, centres, radii)
    y = np.arange(n, dtype=np.float64)
    ux = U * np.sin(2.0 * np.pi * y / n)
    carrier = (rb > 0)
    u[0] = np.where(carrier, ux[None, :, None], 0.0).astype(np.float32)
    return Workload("sheared_droplets_%d" % n, box, rr, rb, u, seed=seed, steps=steps,
                    centres=centres, radii=radii)


def batched_boxes(count: int = 96, lmin: int = 24, lmax: int = 128, seed: int = 4,
                  steps: int = 1000) -> List[Workload]:
    """Independent periodic boxes of uneven size and parameters.

    The interfacial tension is drawn relative to the light-phase density,
    sigma = rho_light * U(0.01, 0.1), the span of the stationary-droplet
    parameters of Table II (there the light phase has unit density); at a
    density ratio of 100 a tension of 0.02 relative to the heavy phase is
    unstable in the FP64 reference update as well."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for b in range(count):
        L = rng.integers(lmin, lmax + 1, size=3)
        gamma = float(rng.choice([1.0, 10.0, 100.0]))
        sigma = float(rng.uniform(0.01, 0.1)) / gamma
        tau = float(rng.uniform(0.55, 1.2))
        box = two_phase_box((int(L[0]), int(L[1]), int(L[2])), gamma, 1.0, tau, sigma, 0.7)
        R = 0.25 * float(L.min())
        c = tuple((float(v) - 1) / 2.0 for v in L)
        rr, rb, u = droplet_fields(box, [c], [R])
        out.append(Workload("box%02d" % b, box, rr, rb, u, seed=seed, steps=steps,
                            centres=[c], radii=[R]))
    return out


def head_on_collision(nx: int = 768, ny: int = 384, nz: int = 384, R: float = 48.0,
                      U: float = 0.05, gamma: float = 10.0, Re: float = 5000.0,
                      We: float = 50.0, beta: float = 0.7, steps: int = 3000) -> Workload:
    """Two droplets moving toward each other between bounce-back walls."""
    rho_r0 = 1.0
    nu_r = 2 * U * (2 * R) / Re
    sigma = rho_r0 * (2 * U) ** 2 * (2 * R) / We
    box = Box(nx=nx, ny=ny, nz=nz, rho0_r=rho_r0, rho0_b=rho_r0 / gamma,
              alpha_r=alpha_heavy(gamma), alpha_b=ALPHA_LIGHT, nu_r=nu_r, nu_b=nu_r,
              sigma=sigma, beta=beta, walls=3)
    cy, cz = (ny - 1) / 2.0, (nz - 1) / 2.0
    cs = [(nx / 2.0 - 2 * R, cy, cz), (nx / 2.0 + 2 * R, cy, cz)]
    rr, rb, u = droplet_fields(box, cs, [R, R], u_drop=[(U, 0, 0), (-U, 0, 0)])
    return Workload("head_on_collision", box, rr, rb, u, steps=steps, centres=cs, radii=[R, R])


def rayleigh_taylor(W: int = 128, At: float = 0.5, Re: Optional[float] = 1024.0,
                    sqrt_wg: float = 0.04, beta: float = 0.7, model: int = 3,
                    steps: int = 16000) -> Workload:
    """Single-mode Rayleigh-Taylor instability in 3D (Sec. IV.E).

    W x W x 4W nodes, solid layers at z = 0 and z = 4W - 1, periodic in x and
    y.  Heavy (red) and light (blue) phases of Atwood number At (density
    ratio (1 + At)/(1 - At), light density 1), equal kinematic viscosities
    nu = sqrt(W g) W / Re (Re = None: nu = 0), no interfacial tension,
    buoyancy -(rho - (rho_r^0 + rho_b^0)/2) g with g = (0, 0, -g) and
    sqrt(W g) = sqrt_wg.  The interface lies at the mid-height plus
    h(x, y) = 0.05 W (cos 2 pi x / W + cos 2 pi y / W).  With g = (0, 0, -g)
    the printed force accelerates the heavy phase toward +z, so the heavy
    phase fills the side below the interface: the unstable arrangement.
    Time unit: sqrt(W / g) steps."""
    gamma = (1.0 + At) / (1.0 - At)
    rho_l, rho_h = 1.0, gamma
    g = sqrt_wg ** 2 / W
    nu = 0.0 if Re is None else sqrt_wg * W / Re
    nz = 4 * W
    box = Box(nx=W, ny=W, nz=nz, rho0_r=rho_h, rho0_b=rho_l, alpha_r=alpha_heavy(gamma),
              alpha_b=ALPHA_LIGHT, nu_r=nu, nu_b=nu, sigma=0.0, beta=beta, walls=2,
              model=model, gravity=(0.0, 0.0, -g), rho_ref=0.5 * (rho_h + rho_l))
    x = np.arange(W)
    h = 0.05 * W * (np.cos(2.0 * np.pi * x / W)[None, :] + np.cos(2.0 * np.pi * x / W)[:, None])
    zi = (nz - 1) / 2.0 + h                       # [y, x]
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    heavy = z < zi[None, :, :]
    rho_r = np.where(heavy, rho_h, 0.0).astype(np.float32)
    rho_b = np.where(heavy, 0.0, rho_l).astype(np.float32)
    u = np.zeros((3,) + box.shape, dtype=np.float32)
    return Workload("rayleigh_taylor_%d" % W, box, rho_r, rho_b, u, steps=steps)


def interface_height(phi: np.ndarray, x: int, y: int) -> float:
    """Height z of the phi = 0 crossing in column (x, y), the crossing nearest
    to the box's mid-height (linear interpolation)."""
    col = phi[:, y, x]
    nz = col.shape[0]
    s = np.sign(col)
    idx = np.nonzero(s[1:] * s[:-1] < 0)[0]
    if len(idx) == 0:
        return float("nan")
    k = idx[np.argmin(np.abs(idx - nz / 2.0))]
    return float(k + col[k] / (col[k] - col[k + 1]))


def layered_channel(case: str, a: int = 8, b: int = 16, nu: float = 0.02,
                    G: float = 1.5e-8, sigma: float = 0.002 / 4.5, beta: float = 0.7):
    """Layered two-phase channel flow between no-slip walls (Table III cases).

    Red occupies |y| <= a, blue a < |y| <= b; walls at |y| = b (bounce-back
    solid layers at y = 0 and y = 2b + 1).  The kinematic viscosities follow
    from the dynamic ratio M of Table III with the given nu for blue."""
    table = {"A": (0.1, 0.8, 0.9, 1.0 / 8.0),
             "B": (0.8, 0.1, 0.2, 8.0),
             "C": (0.008, 8.0, 0.9992, 1.0 / 40.0)}
    rho_r0, rho_b0, alpha_b, M = table[case]
    gamma = rho_r0 / rho_b0
    alpha_r = 1.0 - (1.0 - alpha_b) / gamma
    nu_b = nu
    nu_r = M * rho_b0 * nu_b / rho_r0
    ny = 2 * b + 2
    box = Box(nx=1, ny=ny, nz=1, rho0_r=rho_r0, rho0_b=rho_b0, alpha_r=alpha_r, alpha_b=alpha_b,
              nu_r=nu_r, nu_b=nu_b, sigma=sigma, beta=beta, body_force=(G, 0.0, 0.0), walls=1)
    y = np.arange(ny) - (ny - 1) / 2.0
    red = (np.abs(y) <= a)[None, :, None]
    rho_r = np.where(red, rho_r0, 0.0).astype(np.float32) * np.ones(box.shape, np.float32)
    rho_b = np.where(red, 0.0, rho_b0).astype(np.float32) * np.ones(box.shape, np.float32)
    u = np.zeros((3,) + box.shape, dtype=np.float32)
    return Workload("layered_%s" % case, box, rho_r, rho_b, u, centres=None, radii=None), M



# ---------------------------------------------------------------------------
# Two-dimensional cases (D2Q9 lattice of App. A): Boxes with nz = 1.
#   * xi = 3/5 (the rest fractions of Eq. 8 sum to one on D2Q9);
#   * the lighter phase takes alpha = 4/9 (squared sound speed 1/3), the
#     heavier alpha = 1 - (5/9)/g for density ratio g (equal pressures,
#     Eq. 13).
# ---------------------------------------------------------------------------

XI_2D = 3.0 / 5.0
ALPHA_LIGHT_2D = 4.0 / 9.0


def alpha_heavy_2d(gamma: float) -> float:
    return 1.0 - (5.0 / 9.0) / gamma


def stationary_droplet_2d(gamma: float = 1.0, sigma: float = 0.072, n: int = 100,
                          R: float = 25.0, nu: float = 1.0 / 6.0, beta: float = 0.7,
                          steps: int = 20000) -> Workload:
    """Table II's stationary droplet: a red circle of radius R (density
    gamma) in blue fluid of density 1, periodic n x n box, nu_r = nu_b = nu
    (Sec. IV.A)."""
    box = Box(nx=n, ny=n, nz=1, rho0_r=gamma, rho0_b=1.0, alpha_r=alpha_heavy_2d(gamma),
              alpha_b=ALPHA_LIGHT_2D, nu_r=nu, nu_b=nu, sigma=sigma, beta=beta)
    c = ((n - 1) / 2.0, (n - 1) / 2.0, 0.0)
    rr, rb, u = droplet_fields(box, [c], [R])
    return Workload("stationary_droplet_2d_g%g_s%g" % (gamma, sigma), box, rr, rb, u,
                    steps=steps, centres=[c], radii=[R])


def droplets_2d(n: int = 4096, per_side: int = 16, R: float = 48.0, gamma: float = 10.0,
                sigma: float = 0.01, nu: float = 0.05, U: float = 0.05, beta: float = 0.7,
                seed: int = 7, noise: float = 1e-4) -> Workload:
    """A periodic n x n field of per_side^2 circular droplets (radius R,
    density ratio gamma, centres on a jittered square grid) carried by a
    uniform flow U along x: the two-dimensional throughput case."""
    box = Box(nx=n, ny=n, nz=1, rho0_r=gamma, rho0_b=1.0, alpha_r=alpha_heavy_2d(gamma),
              alpha_b=ALPHA_LIGHT_2D, nu_r=nu, nu_b=nu, sigma=sigma, beta=beta)
    rng = np.random.Generator(np.random.PCG64(seed))
    pitch = n / per_side
    jit = max(pitch / 2.0 - R - 4.0, 0.0)
    centres = [((i + 0.5) * pitch + rng.uniform(-jit, jit),
                (j + 0.5) * pitch + rng.uniform(-jit, jit), 0.0)
               for j in range(per_side) for i in range(per_side)]
    rr, rb, u = droplet_fields(box, centres, [R] * len(centres), u_carrier=(U, 0.0, 0.0))
    return Workload("droplets_2d_%d" % n, box, rr, rb, u, seed=seed, noise=noise,
                    centres=centres, radii=[R] * len(centres))
