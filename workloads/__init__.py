"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the scattering method.  It only draws
particle clouds (centres, enclosing radii, truncation orders, boundary
conditions, shape labels, orientations), the material and frequency settings
of each named workload, and random coefficient vectors.  Everything is
deterministic given the seed (numpy PCG64).

Frame: the particles live in the half-space y < 0 of the paper's frame (the
interface is y = 0).  The workloads are described with a height coordinate
z > 0 measured from the interface; they are mapped with y = -z.  The medium
holding the particles is called the *host*; the other half-space is the
*substrate*.

Shape family of the paper's experiments (Section 7): r(t) = a1 + a2 cos(a3 t).
Labels used here: 0 circle (radius a), 1 ellipse (semi-axes a and a/2),
2 five-arm star r(t) = a (1 + 0.3 cos 5t).  The enclosing radius is a for the
first two and 1.3 a for the star.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SHAPE_CIRCLE, SHAPE_ELLIPSE, SHAPE_STAR, SHAPE_PEAR, SHAPE_STARFISH = 0, 1, 2, 3, 4
BC_RIGID, BC_TRACTION_FREE = 0, 1


@dataclasses.dataclass(frozen=True)
class Medium:
    lam: float
    mu: float
    rho: float


@dataclasses.dataclass
class Workload:
    """One particle cloud in the paper frame (y < 0) plus its physical settings."""

    name: str
    xy: np.ndarray          # [n, 2] centres, paper frame
    radius: np.ndarray      # [n] enclosing-disk radii
    a: np.ndarray           # [n] shape size parameter
    p: np.ndarray           # [n] truncation orders
    bc: np.ndarray          # [n] 0 rigid / 1 traction-free
    shape: np.ndarray       # [n] shape label
    theta0: np.ndarray      # [n] orientation angle
    host: Medium
    substrate: Medium
    omega: float
    incidence: list         # list of (wave, angle_rad): wave 0 = P, 1 = SV

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_coeff(self) -> int:
        """Complex unknowns per right-hand side: sum over particles of 2(2p+1)."""
        return int(np.sum(2 * (2 * self.p + 1)))

    def offsets(self) -> np.ndarray:
        """Start of each particle block in a coefficient vector ([n+1])."""
        sz = 2 * (2 * self.p.astype(np.int64) + 1)
        return np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx)
        return dataclasses.replace(
            self, name=f"{self.name}[sub{len(idx)}]", xy=self.xy[idx].copy(),
            radius=self.radius[idx].copy(), a=self.a[idx].copy(), p=self.p[idx].copy(),
            bc=self.bc[idx].copy(), shape=self.shape[idx].copy(),
            theta0=self.theta0[idx].copy())


# Materials of the benchmark workloads: host (particle side) lambda=2, mu=1,
# rho=1; substrate lambda=4, mu=2, rho=1.5.
HOST = Medium(2.0, 1.0, 1.0)
SUBSTRATE = Medium(4.0, 2.0, 1.5)
# Materials of the paper's numerical section (omega = 2 pi; lambda=1, mu=2 in
# the upper layer; lambda'=3, mu'=4 in the particle layer; rho = 1).
PAPER_UPPER = Medium(1.0, 2.0, 1.0)
PAPER_LOWER = Medium(3.0, 4.0, 1.0)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _uniform_gap_placement(rng, n, box, radius, min_centre_dist, max_tries=200000):
    """Rejection sampling: x then z uniform in the box, keep if far enough."""
    (x0, x1), (z0, z1) = box
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("placement did not converge")
        x = rng.uniform(x0, x1)
        z = rng.uniform(z0, z1)
        if all((x - q[0]) ** 2 + (z - q[1]) ** 2 >= min_centre_dist ** 2 for q in pts):
            pts.append((x, z))
    return np.array(pts)


def _dart_throwing(rng, radii, box, factor, min_z_clear=0.0, max_tries_per=20000):
    """Poisson-disk style dart throwing: |c_m - c_l| >= factor (R_m + R_l).

    Radii are placed in the given order.  A uniform cell grid keeps the
    neighbour test local.  Also keeps z - R >= min_z_clear.
    """
    (x0, x1), (z0, z1) = box
    rmax = float(np.max(radii))
    cell = 2.0 * factor * rmax
    nx = max(1, int(math.ceil((x1 - x0) / cell)))
    nz = max(1, int(math.ceil((z1 - z0) / cell)))
    grid: dict = {}
    out = np.zeros((len(radii), 2))
    for k, r in enumerate(radii):
        for _ in range(max_tries_per):
            x = rng.uniform(x0, x1)
            z = rng.uniform(z0, z1)
            if z - r < min_z_clear:
                continue
            cx = min(nx - 1, int((x - x0) / cell))
            cz = min(nz - 1, int((z - z0) / cell))
            ok = True
            for gx in range(cx - 1, cx + 2):
                for gz in range(cz - 1, cz + 2):
                    for j in grid.get((gx, gz), ()):
                        dx = x - out[j, 0]
                        dz = z - out[j, 1]
                        if dx * dx + dz * dz < (factor * (r + radii[j])) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                out[k] = (x, z)
                grid.setdefault((cx, cz), []).append(k)
                break
        else:
            raise RuntimeError(f"dart throwing jammed at particle {k}")
    return out


def c0_circles(seed: int = 0, p: int = 10) -> Workload:
    """16 rigid circles of radius 0.5 in [0,20]x[1,10] (height), gap >= 0.5.

    omega is chosen so that kp * a = 1 in the host: kp = 2, omega = 4.
    One P wave at 30 degrees from the interface normal.
    """
    rng = _rng(seed)
    n = 16
    xz = _uniform_gap_placement(rng, n, ((0.0, 20.0), (1.0, 10.0)), 0.5, 1.5)
    xy = np.stack([xz[:, 0], -xz[:, 1]], axis=1)
    rad = np.full(n, 0.5)
    host = HOST
    omega = 2.0 * math.sqrt((host.lam + 2 * host.mu) / host.rho)  # kp = 2
    return Workload("c0", xy, rad, rad.copy(), np.full(n, p, dtype=np.int32),
                    np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32),
                    np.zeros(n), host, SUBSTRATE, omega, [(0, math.radians(30.0))])


def cloud(n: int, box_x: float, box_z: tuple, seed: int, p: int | None = 15,
          omega: float = 8.0, shapes: bool = False, min_z_clear: float = 0.0,
          name: str = "cloud") -> Workload:
    """Random cloud as in the paper's large experiments, scaled up.

    a ~ U[0.3, 0.7]; half rigid and half traction-free (seeded permutation);
    shape labels split in thirds when ``shapes`` is set (else all circles);
    orientations U[0, 2 pi); dart throwing with the 10 % separation rule.
    ``p`` None selects p_i = ceil(ks a_i) + 8 with ks the host shear number.
    """
    rng = _rng(seed)
    a = rng.uniform(0.3, 0.7, size=n)
    perm = rng.permutation(n)
    bc = np.zeros(n, dtype=np.int32)
    bc[perm[: n // 2]] = BC_TRACTION_FREE
    shape = np.zeros(n, dtype=np.int32)
    if shapes:
        perm2 = rng.permutation(n)
        shape[perm2[: n // 3]] = SHAPE_ELLIPSE
        shape[perm2[n // 3: 2 * n // 3]] = SHAPE_STAR
    theta0 = rng.uniform(0.0, 2 * math.pi, size=n)
    theta0[shape == SHAPE_CIRCLE] = 0.0
    rad = np.where(shape == SHAPE_STAR, 1.3 * a, a)
    xz = _dart_throwing(rng, rad, ((0.0, box_x), box_z), 1.1, min_z_clear=min_z_clear)
    xy = np.stack([xz[:, 0], -xz[:, 1]], axis=1)
    host = HOST
    ks = omega * math.sqrt(host.rho / host.mu)
    if p is None:
        pv = (np.ceil(ks * a) + 8).astype(np.int32)
    else:
        pv = np.full(n, p, dtype=np.int32)
    return Workload(name, xy, rad, a, pv, bc, shape, theta0, host, SUBSTRATE, omega,
                    [(0, math.radians(30.0))])


def c1_cloud(shapes: bool = False) -> Workload:
    """2000 particles in [0,200] x [1,50], p = 15, omega = 8 (kp = 4)."""
    return cloud(2000, 200.0, (1.0, 50.0), seed=1, p=15, omega=8.0, shapes=shapes,
                 name="c1")


def c2_cloud(shapes: bool = False) -> Workload:
    """20000 particles in [0,600] x [1,150], p = 15, omega = 8 (kp = 4)."""
    return cloud(20000, 600.0, (1.0, 150.0), seed=2, p=15, omega=8.0, shapes=shapes,
                 name="c2")


def c3_cloud(freq: int) -> Workload:
    """The 20000-particle geometry with uneven orders p_i = ceil(ks a_i) + 8 at
    omega = 2, 4, 8 (kp a_mean = 0.5, 1, 2) for freq = 0, 1, 2, and 64
    incident directions linspace(-80, 80) degrees, even index P, odd SV."""
    omega = (2.0, 4.0, 8.0)[freq]
    w = cloud(20000, 600.0, (1.0, 150.0), seed=2, p=None, omega=omega, name=f"c3f{freq}")
    ang = np.radians(np.linspace(-80.0, 80.0, 64))
    w.incidence = [(k % 2, float(a)) for k, a in enumerate(ang)]
    return w


def c4_cloud() -> Workload:
    """5000 particles at the density of the 2000-particle cloud, [0,320] x [1,80]
    with z - R >= 0.6 (receivers at z = 0.5 stay outside every disk), p = 15,
    omega = 8; 32 P waves at linspace(-80, 80) degrees."""
    w = cloud(5000, 320.0, (1.0, 80.0), seed=4, p=15, omega=8.0, min_z_clear=0.6, name="c4")
    w.incidence = [(0, float(a)) for a in np.radians(np.linspace(-80.0, 80.0, 32))]
    return w


def c4_receivers(n: int = 1024, width: float = 320.0, z: float = 0.5) -> np.ndarray:
    """Receiver line in the paper frame: x equispaced over the box width, y = -z."""
    return np.stack([np.linspace(0.0, width, n), np.full(n, -z)], axis=1)


def c4_start(w: Workload, seed: int = 5, sigma: float = 0.05, lam_factor: float = 1.05,
             mu_factor: float = 0.95, z_clear: float = 0.55):
    """Perturbed start of the inverse problem: centres + N(0, sigma^2) per
    coordinate, substrate lambda and mu scaled.  A perturbation that would make
    two enclosing disks touch, or bring a disk within z_clear of the
    interface, is drawn again (up to 50 times, then the centre stays).
    Returns (workload, substrate)."""
    rng = _rng(seed)
    xy = w.xy.copy()
    R = w.radius
    cell = 4.0 * float(R.max()) + 1.0
    grid: dict = {}
    for i in range(w.n):
        grid.setdefault((int(xy[i, 0] // cell), int(xy[i, 1] // cell)), []).append(i)
    for i in range(w.n):
        for _ in range(50):
            c = w.xy[i] + rng.normal(0.0, sigma, size=2)
            if -c[1] - R[i] < z_clear:
                continue
            gx, gy = int(c[0] // cell), int(c[1] // cell)
            ok = True
            for ax in (gx - 1, gx, gx + 1):
                for ay in (gy - 1, gy, gy + 1):
                    for j in grid.get((ax, ay), ()):
                        if j != i and np.hypot(*(c - xy[j])) <= 1.001 * (R[i] + R[j]):
                            ok = False
            if ok:
                xy[i] = c
                break
    sub = Medium(w.substrate.lam * lam_factor, w.substrate.mu * mu_factor, w.substrate.rho)
    return dataclasses.replace(w, xy=xy, substrate=sub, name=w.name + "-start"), sub


def small_cloud(n: int, seed: int, p: int = 6, omega: float = 4.0, width: float = 30.0,
                depth: tuple = (1.0, 8.0), ragged: bool = False) -> Workload:
    """A small cloud for parity tests that the oracle finishes in seconds."""
    w = cloud(n, width, depth, seed=seed, p=p, omega=omega, name=f"small{n}s{seed}")
    if ragged:
        rng = _rng(seed + 777)
        w.p = rng.integers(max(1, p - 3), p + 1, size=n).astype(np.int32)
    return w


def random_coeffs(n_coeff: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """x ~ CN(0, 1) i.i.d., shape [nrhs, n_coeff] complex128."""
    rng = _rng(seed)
    re = rng.standard_normal((nrhs, n_coeff))
    im = rng.standard_normal((nrhs, n_coeff))
    return (re + 1j * im) / math.sqrt(2.0)


def random_smatrix_blocks(p: np.ndarray, seed: int, scale: float = 0.3) -> list:
    """Random dense complex blocks of size (4p+2)^2, one per particle."""
    rng = _rng(seed)
    out = []
    for pm in p:
        k = 4 * int(pm) + 2
        out.append(scale * (rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
                   / math.sqrt(2.0 * k))
    return out
