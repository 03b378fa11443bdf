"""Scattered displacement (Section 5, coupled representation): host points
(y < 0) and, transmitted through the interface, substrate points (y > 0).

u^sc(x) = sum_m sum_n alpha^m_n grad(H_n(kp r_m) e^{i n theta_m})
                  + beta^m_n grad^perp(H_n(ks r_m) e^{i n theta_m})
          + grad phi_R + grad^perp psi_R,
with phi_R = int e^{i xi x + s_p y} RP(xi) dxi and psi_R likewise with RS, the
reflected potentials of Section 5 (see ``sommerfeld``).

Derivatives of v_n = Z_n(k r) e^{i n theta} (standard cylinder-function
identities, the same structure as the density-to-coefficient formula of
Section 4.3):
  d_x v_n = (k/2)(v_{n-1} - v_{n+1}),  d_y v_n = (i k/2)(v_{n-1} + v_{n+1});
grad^perp = (-d_y, d_x).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, special

from . import interface, sommerfeld
from .media import Media


def cyl_wave(kind: str, n, k: float, dx, dy):
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    Z = special.hankel1(n, k * r) if kind == "H" else special.jv(n, k * r)
    return Z * np.exp(1j * n * th)


def grad_cyl(kind: str, n: int, k: float, dx, dy):
    """(d_x, d_y) of Z_n(k r) e^{i n theta} at offsets (dx, dy)."""
    vm = cyl_wave(kind, n - 1, k, dx, dy)
    vp = cyl_wave(kind, n + 1, k, dx, dy)
    return 0.5 * k * (vm - vp), 0.5j * k * (vm + vp)


def direct_part(w, m: Media, gamma: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Free-space outgoing fields of all particles at points [n, 2] -> [n, 2]."""
    kp, ks = m.kp, m.ks
    off = w.offsets()
    u = np.zeros((len(pts), 2), dtype=complex)
    for i in range(w.n):
        pm = int(w.p[i])
        N = 2 * pm + 1
        al = gamma[off[i]: off[i] + N]
        be = gamma[off[i] + N: off[i + 1]]
        dx = pts[:, 0] - w.xy[i, 0]
        dy = pts[:, 1] - w.xy[i, 1]
        for k_, n in enumerate(range(-pm, pm + 1)):
            gx, gy = grad_cyl("H", n, kp, dx, dy)
            u[:, 0] += al[k_] * gx
            u[:, 1] += al[k_] * gy
            hx, hy = grad_cyl("H", n, ks, dx, dy)
            u[:, 0] += -be[k_] * hy
            u[:, 1] += be[k_] * hx
    return u


def reflected_part(w, m: Media, gamma: np.ndarray, pts: np.ndarray, tol: float = 1e-13,
                   T: float | None = None, limit: int = 200000) -> np.ndarray:
    """grad phi_R + grad^perp psi_R at host points [n, 2] -> [n, 2]."""
    kp, ks = m.kp, m.ks
    off = w.offsets()
    groups = sommerfeld._Groups(w, range(w.n))
    coef = []
    for pv, sel, xs, ys, o in groups.items:
        Np = 2 * pv + 1
        c = gamma[o[:, None] + np.arange(2 * Np)[None, :]]
        coef.append((c[:, :Np], c[:, Np:]))
    px, py = pts[:, 0], pts[:, 1]
    npt = len(pts)

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        sp, ss = sv[0], sv[1]
        zp = (xi - sp) / kp
        zs = (xi - ss) / ks
        Ip = 0j
        Is = 0j
        for (pv, sel, xs, ys, o), (ca, cb) in zip(groups.items, coef):
            n = np.arange(-pv, pv + 1)
            Ip += np.sum(np.exp(sp * ys - 1j * xi * xs) * (ca @ ((-1j * zp) ** n)))
            Is += np.sum(np.exp(ss * ys - 1j * xi * xs) * (cb @ ((-1j * zs) ** n)))
        Ip /= 1j * math.pi * sp
        Is /= 1j * math.pi * ss
        R = interface.reflection(xi, m, sv)
        RP = R[0, 0] * Ip + R[0, 1] * Is
        RS = R[1, 0] * Ip + R[1, 1] * Is
        ep = np.exp(1j * xi * px + sp * py) * RP
        es = np.exp(1j * xi * px + ss * py) * RS
        ux = 1j * xi * ep - ss * es
        uy = sp * ep + 1j * xi * es
        v = np.concatenate([ux, uy])
        return np.concatenate([v.real, v.imag])

    if T is None:
        T = sommerfeld.tail_extent(w, m)
    pieces = sommerfeld._pieces(m, T)
    v, _, _ = sommerfeld._integrate(f, 2 * npt, pieces, tol, limit)
    return np.stack([v[:npt], v[npt:]], axis=1)


def transmitted_part(w, m: Media, gamma: np.ndarray, pts: np.ndarray, tol: float = 1e-13,
                     T: float | None = None, limit: int = 200000) -> np.ndarray:
    """Displacement at substrate points (y > 0) [n, 2] -> [n, 2]: the particles'
    upgoing potentials (the aggregate of ``reflected_part``) crossing the
    interface with the transmission T(xi) of ``interface.reflect_transmit``,
    phi_T = int e^{i xi x - s_pb y} TP(xi) dxi and psi_T likewise with TS, so
    grad -> (i xi, -s_pb) and grad^perp -> (s_sb, i xi)."""
    kp, ks = m.kp, m.ks
    groups = sommerfeld._Groups(w, range(w.n))
    coef = []
    for pv, sel, xs, ys, o in groups.items:
        Np = 2 * pv + 1
        c = gamma[o[:, None] + np.arange(2 * Np)[None, :]]
        coef.append((c[:, :Np], c[:, Np:]))
    px, py = pts[:, 0], pts[:, 1]
    npt = len(pts)

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        sp, ss, spb, ssb = sv
        zp = (xi - sp) / kp
        zs = (xi - ss) / ks
        Ip = 0j
        Is = 0j
        for (pv, sel, xs, ys, o), (ca, cb) in zip(groups.items, coef):
            n = np.arange(-pv, pv + 1)
            Ip += np.sum(np.exp(sp * ys - 1j * xi * xs) * (ca @ ((-1j * zp) ** n)))
            Is += np.sum(np.exp(ss * ys - 1j * xi * xs) * (cb @ ((-1j * zs) ** n)))
        Ip /= 1j * math.pi * sp
        Is /= 1j * math.pi * ss
        _, Tm = interface.reflect_transmit(xi, m, sv)
        TP = Tm[0, 0] * Ip + Tm[0, 1] * Is
        TS = Tm[1, 0] * Ip + Tm[1, 1] * Is
        ep = np.exp(1j * xi * px - spb * py) * TP
        es = np.exp(1j * xi * px - ssb * py) * TS
        ux = 1j * xi * ep + ssb * es
        uy = -spb * ep + 1j * xi * es
        v = np.concatenate([ux, uy])
        return np.concatenate([v.real, v.imag])

    if T is None:
        T = sommerfeld.tail_extent(w, m)
    pieces = sommerfeld._pieces(m, T)
    v, _, _ = sommerfeld._integrate(f, 2 * npt, pieces, tol, limit)
    return np.stack([v[:npt], v[npt:]], axis=1)


def scattered(w, m: Media, gamma: np.ndarray, pts: np.ndarray, tol: float = 1e-13) -> np.ndarray:
    """Host points (y < 0): direct + reflected; substrate points (y > 0): transmitted."""
    pts = np.asarray(pts, dtype=float)
    u = np.zeros((len(pts), 2), dtype=complex)
    host = pts[:, 1] < 0
    if host.any():
        ph = pts[host]
        u[host] = direct_part(w, m, gamma, ph) + reflected_part(w, m, gamma, ph, tol=tol)
    if (~host).any():
        u[~host] = transmitted_part(w, m, gamma, pts[~host], tol=tol)
    return u
