"""Scattering matrices of non-circular particles (Section 4.3).
TEST INFRASTRUCTURE ONLY: nothing in the product imports this module.

S maps the incoming coefficients (a_n, b_n) of grad(J_n(kp r) e^{i n th}) and
grad^perp(J_n(ks r) e^{i n th}) about the enclosing-disk centre to the outgoing
coefficients (alpha_n, beta_n) of grad(H_n(kp r) e^{i n th}) and
grad^perp(H_n(ks r) e^{i n th}) of the field the particle scatters (Section 4.1
definition, extended to any shape in Section 4.3).

Discretisation (the paper solves a boundary integral equation by a Nystrom
rule; here, method of fundamental solutions): the scattered field is a sum of
N compressional and N shear monopoles, phi = sum_j c_j H_0(kp |x - y_j|),
psi = sum_j d_j H_0(ks |x - y_j|), u = grad phi + grad^perp psi, with the
sources y_j on the boundary's parametrisation continued inward, z(t_j + i delta)
(t_j equispaced).  The boundary condition (u = -u_inc for a rigid particle,
traction sigma.nu = -sigma_inc.nu for a traction-free one) is collocated at the
N boundary points z(t_j): 2N equations for 2N unknowns per incident basis
field.  By Graf's addition theorem, for |x| > |y|,
  H_0(k |x - y|) = sum_l H_l(k |x|) e^{i l th_x} J_l(k |y|) e^{-i l th_y},
so alpha_l = sum_j c_j J_l(kp |y_j|) e^{-i l th_j} and beta_l likewise with
(d_j, ks).

Shapes (paper frame, about the centre, turned by theta0): 0 circle of radius a;
1 ellipse with semi-axes a and a/2; 2 five-arm star r(t) = a (1 + 0.3 cos 5t);
and the paper's own family r(t) = a1 + a2 cos(a3 t) (Section 7) with
a2 = a1/4: 3 pear (a3 = 3), 4 starfish (a3 = 5), a = a1.

Parity unpinned for the non-circular shapes: no closed form exists and the
GPU generator uses the same discretisation, so agreement with it shows two
implementations of one method agreeing.  What pins this module is the
closed-form disk (kind 0 against the mode-by-mode boundary conditions), and
for the other shapes only invariants: I + 2S unitary (lossless particles), the
boundary condition between the collocation points, the basis rotation of a
turned shape, and agreement between 256 and 320 collocation points.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .media import Media

DELTA = {0: 0.3, 1: 0.2, 2: 0.12, 3: 0.2, 4: 0.16}
# rose curves r = a (1 + eps cos(m t)): kind -> (m, eps)
ROSE = {2: (5, 0.3), 3: (3, 0.25), 4: (5, 0.25)}


def boundary(kind: int, a: float, t, delta: float = 0.0):
    """z(t + i delta) as a complex number (the point (Re, Im)) and dz/dt."""
    tt = np.asarray(t) + 1j * delta
    if kind == 0:
        z, dz = a * np.exp(1j * tt), 1j * a * np.exp(1j * tt)
    elif kind == 1:
        z = a * np.cos(tt) + 0.5j * a * np.sin(tt)
        dz = -a * np.sin(tt) + 0.5j * a * np.cos(tt)
    elif kind in ROSE:
        mm, eps = ROSE[kind]
        r = a * (1 + eps * np.cos(mm * tt))
        dr = -eps * mm * a * np.sin(mm * tt)
        z, dz = r * np.exp(1j * tt), (dr + 1j * r) * np.exp(1j * tt)
    else:
        raise ValueError("unknown shape")
    return z, dz


def _pot(kind: str, n: int, k: float, x, y):
    """(v, v_x, v_y, v_xx, v_xy, v_yy) of Z_n(k r) e^{i n th} by the Cartesian
    recurrences d_x v_n = (k/2)(v_{n-1} - v_{n+1}), d_y v_n = (i k/2)(v_{n-1} + v_{n+1})."""
    r = np.hypot(x, y)
    th = np.arctan2(y, x)

    def v(m):
        Z = special.jv(m, k * r) if kind == "J" else special.hankel1(m, k * r)
        return Z * np.exp(1j * m * th)

    def dx(f):
        return lambda m: 0.5 * k * (f(m - 1) - f(m + 1))

    def dy(f):
        return lambda m: 0.5j * k * (f(m - 1) + f(m + 1))
    return v(n), dx(v)(n), dy(v)(n), dx(dx(v))(n), dx(dy(v))(n), dy(dy(v))(n)


def _u_t(m: Media, phi, psi, nx, ny):
    """Displacement and traction sigma.nu of grad phi + grad^perp psi in the host."""
    lam, mu = m.lam_h, m.mu_h
    _, px, py, pxx, pxy, pyy = phi
    _, sx, sy, sxx, sxy, syy = psi
    u1, u2 = px - sy, py + sx
    u1x, u1y, u2x, u2y = pxx - sxy, pxy - syy, pxy + sxx, pyy + sxy
    div = u1x + u2y
    s11 = lam * div + 2 * mu * u1x
    s22 = lam * div + 2 * mu * u2y
    s12 = mu * (u1y + u2x)
    return np.stack([u1, u2]), np.stack([s11 * nx + s12 * ny, s12 * nx + s22 * ny])


def _system(m: Media, kind: int, a: float, p: int, bc: int, theta0: float, t, zs):
    """Collocation matrix (sources zs) and incident columns at boundary points z(t)."""
    kp, ks = m.kp, m.ks
    rot = np.exp(1j * theta0)
    zc, dz = boundary(kind, a, t)
    zc, dz = zc * rot, dz * rot
    nx, ny = dz.imag / np.abs(dz), -dz.real / np.abs(dz)
    xc, yc, xs, ys = zc.real, zc.imag, zs.real, zs.imag
    nc, ns_ = len(t), len(zs)
    zero = (np.zeros(nc),) * 6
    A = np.zeros((2 * nc, 2 * ns_), complex)
    for j in range(ns_):
        dx, dy = xc - xs[j], yc - ys[j]
        uP, tP = _u_t(m, _pot("H", 0, kp, dx, dy), zero, nx, ny)
        uS, tS = _u_t(m, zero, _pot("H", 0, ks, dx, dy), nx, ny)
        A[:, j] = (uP if bc == 0 else tP).reshape(-1)
        A[:, ns_ + j] = (uS if bc == 0 else tS).reshape(-1)
    ns = np.arange(-p, p + 1)
    B = np.zeros((2 * nc, 2 * len(ns)), complex)
    for c, n in enumerate(ns):
        uP, tP = _u_t(m, _pot("J", n, kp, xc, yc), zero, nx, ny)
        uS, tS = _u_t(m, zero, _pot("J", n, ks, xc, yc), nx, ny)
        B[:, c] = -(uP if bc == 0 else tP).reshape(-1)
        B[:, len(ns) + c] = -(uS if bc == 0 else tS).reshape(-1)
    return A, B


def smatrix(m: Media, kind: int, a: float, p: int, bc: int, theta0: float = 0.0,
            npts: int = 256, delta: float | None = None, residual: bool = False):
    """(4p+2) x (4p+2) S of one particle, columns (a_{-p..p}, b_{-p..p}).  With
    residual, also the relative boundary-condition residual of the monopole
    field at the points halfway between the collocation points."""
    kp, ks = m.kp, m.ks
    d = DELTA[kind] if delta is None else delta
    t = 2 * np.pi * np.arange(npts) / npts
    zs = boundary(kind, a, t, d)[0] * np.exp(1j * theta0)
    A, B = _system(m, kind, a, p, bc, theta0, t, zs)
    C = np.linalg.solve(A, B)   # a library primitive (LU with partial pivoting)
    ns = np.arange(-p, p + 1)
    rs, ths = np.abs(zs), np.angle(zs)
    Ep = special.jv(ns[:, None], kp * rs[None, :]) * np.exp(-1j * ns[:, None] * ths[None, :])
    Es = special.jv(ns[:, None], ks * rs[None, :]) * np.exp(-1j * ns[:, None] * ths[None, :])
    S = np.vstack([Ep @ C[:npts], Es @ C[npts:]])
    if not residual:
        return S
    Am, Bm = _system(m, kind, a, p, bc, theta0, t + np.pi / npts, zs)
    return S, float(np.linalg.norm(Am @ C - Bm) / np.linalg.norm(Bm))
