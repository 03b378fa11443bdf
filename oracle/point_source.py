"""Point-source incidence (Section 3.2; the point-source workload of Section 7).
TEST INFRASTRUCTURE ONLY: nothing in the product imports this module.

An elastic point source at x0 = (x0, y0), y0 > 0, in the substrate (the
paper's upper half-space; the particles live in the lower one, the host)
with polarisation alpha radiates u_inc = Phi(x, x0) alpha, Phi the Green's
tensor of the substrate's Navier operator,
  Phi = 1/(rho omega^2) (ks^2 g_ks I + grad grad^T (g_ks - g_kp)),  g_k = (i/4) H_0(k r)
(the paper writes it with rho = 1; the density is kept here as everywhere in
the oracle).  Its Sommerfeld form uses
  g~_k = 1/(4 pi) e^{-s |y - y0|} / s  e^{i xi (x - x0)},
so that Phi = int Phi~(xi) dxi with grad -> (i xi, -+ s) on the two sides of
the source.  The field scattered by the interface is u1 = int Phi~1 sigma_1
in the substrate (g~1 = e^{-s y}/s ...) and u2 = int Phi~2 sigma_2 in the host
(g~2 = e^{+s y}/s ..., host constants).  Continuity of displacement and of
the traction T_y u = (mu (d_y u1 + d_x u2), (lambda + 2 mu) d_y u2 + lambda d_x u1)
at y = 0, one xi at a time, gives the 4x4 system A_xi sigma = b_xi of the
paper; here it is assembled numerically from those definitions (each term's
displacement and traction at y = 0 as linear maps of its density), and the
tests compare it with the printed (aa) and b_xi at rho = 1.

The particles see u2.  Its Helmholtz split, per xi (grad -> (i xi, s)):
  P:  phi = -1/(rho omega^2) (i xi sigma_21 + s_p sigma_22) g~2_kp,
  S:  psi =  1/(rho omega^2) (s_s sigma_21 - i xi sigma_22) g~2_ks
(u = grad phi + grad^perp psi, grad^perp = (-d_y, d_x)), and Jacobi-Anger
(Section 5.3, (ja)) turns e^{i xi x + s y} into local coefficients about
(x_m, y_m): e^{i xi x_m + s y_m} (i (xi - s)/k)^n.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import interface, sommerfeld
from .media import Media


def _term(xi, q, k_s, rho, lam, mu, omega, c, G):
    """(u, t) at one height of 1/(rho omega^2) (ks^2 g_s c + grad grad^T (g_s - g_p) c)
    with g_k = G[k] e^{q[k] y} e^{i xi x} at that height (G, q, s indexed 'p', 's')."""
    Dp = np.array([1j * xi, q["p"]])
    Ds = np.array([1j * xi, q["s"]])
    us = (k_s ** 2 * c + Ds * (Ds @ c)) * G["s"] / (rho * omega ** 2)
    up = -Dp * (Dp @ c) * G["p"] / (rho * omega ** 2)

    def trac(v, b):
        return np.array([mu * (b * v[0] + 1j * xi * v[1]), (lam + 2 * mu) * b * v[1] + lam * 1j * xi * v[0]])
    return us + up, trac(us, q["s"]) + trac(up, q["p"])


def system(xi, m: Media, y0: float, alpha, svals=None):
    """(A, b) of A sigma = b at one real xi: rows (u1, u2, t1, t2) continuity,
    sigma = (sigma_11, sigma_12, sigma_21, sigma_22); the common factor
    e^{i xi (x - x0)} is left out."""
    sp, ss, spb, ssb = svals if svals is not None else interface.s_values(xi, m)
    w = m.omega
    sub = dict(rho=m.rho_b, lam=m.lam_b, mu=m.mu_b, k_s=m.ksb)
    hos = dict(rho=m.rho_h, lam=m.lam_h, mu=m.mu_h, k_s=m.ks)
    A = np.zeros((4, 4), dtype=complex)
    for col in range(2):
        c = np.zeros(2, dtype=complex)
        c[col] = 1.0
        # upper field at y = 0: g~1 = e^{-s y}/(4 pi s)
        u1, t1 = _term(xi, {"p": -spb, "s": -ssb}, omega=w, c=c,
                       G={"p": 1 / (4 * math.pi * spb), "s": 1 / (4 * math.pi * ssb)}, **sub)
        # lower field at y = 0: g~2 = e^{+s y}/(4 pi s), host constants
        u2, t2 = _term(xi, {"p": sp, "s": ss}, omega=w, c=c,
                       G={"p": 1 / (4 * math.pi * sp), "s": 1 / (4 * math.pi * ss)}, **hos)
        A[:, col] = np.concatenate([u1, t1])
        A[:, 2 + col] = -np.concatenate([u2, t2])
    # incident field at y = 0 (below the source: e^{-s (y0 - y)})
    ui, ti = _term(xi, {"p": spb, "s": ssb}, omega=w, c=np.asarray(alpha, dtype=complex),
                   G={"p": np.exp(-spb * y0) / (4 * math.pi * spb),
                      "s": np.exp(-ssb * y0) / (4 * math.pi * ssb)}, **sub)
    b = -np.concatenate([ui, ti])
    return A, b


def densities(xi, m: Media, y0: float, alpha, svals=None):
    A, b = system(xi, m, y0, alpha, svals)
    return np.linalg.solve(A, b)


def greens_tensor(m: Media, x0, pts: np.ndarray) -> np.ndarray:
    """Phi(x, x0) of the substrate, closed form, [n, 2, 2] (derivatives of
    H_0 by the chain rule: d_i d_j H_0(k r) = k^2 [H_0'' r_i r_j / r^2 + H_0'/(k r) (delta_ij - r_i r_j / r^2)],
    H_0' = -H_1, H_0'' = -H_0 + H_1 / (k r))."""
    d = pts - np.asarray(x0)[None, :]
    r = np.hypot(d[:, 0], d[:, 1])
    e = d / r[:, None]
    I2 = np.eye(2)[None]
    ee = e[:, :, None] * e[:, None, :]

    def hess_g(k):
        z = k * r
        h0, h1 = special.hankel1(0, z), special.hankel1(1, z)
        d1 = -h1
        d2 = -h0 + h1 / z
        return 0.25j * k * k * (d2[:, None, None] * ee + (d1 / z)[:, None, None] * (I2 - ee))

    gs = 0.25j * special.hankel1(0, m.ksb * r)
    return (m.ksb ** 2 * gs[:, None, None] * I2 + hess_g(m.ksb) - hess_g(m.kpb)) / (m.rho_b * m.omega ** 2)


def _tail(m: Media, y0: float, dmin: float, p: int, drop: float = 1e-18) -> float:
    kmin = min(m.kp, m.ks)
    kmax = max(m.kp, m.ks, m.kpb, m.ksb)
    t = np.linspace(0.0, 5000.0, 500001)
    logb = -t * (y0 + dmin) + p * np.log(2.0 * t / kmin + 1.0)
    ok = np.nonzero((logb < float(np.max(logb)) + math.log(drop)) & (t > kmax + 2.0))[0]
    return float(t[ok[0]])


def transmitted_field(m: Media, x0, alpha, pts: np.ndarray, tol: float = 1e-13) -> np.ndarray:
    """u2 = int Phi~2 sigma_2 dxi at host points [n, 2] -> [n, 2]."""
    x0 = np.asarray(x0, dtype=float)
    px, py = pts[:, 0], pts[:, 1]
    npt = len(pts)

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        sp, ss = sv[0], sv[1]
        sig = densities(xi, m, x0[1], alpha, sv)
        c = sig[2:]
        ph = np.exp(1j * xi * (px - x0[0]))
        Gp = np.exp(sp * py) / (4 * math.pi * sp) * ph
        Gs = np.exp(ss * py) / (4 * math.pi * ss) * ph
        Dp = np.array([1j * xi, sp])
        Ds = np.array([1j * xi, ss])
        u = ((m.ks ** 2 * c + Ds * (Ds @ c))[:, None] * Gs[None, :]
             - (Dp * (Dp @ c))[:, None] * Gp[None, :]) / (m.rho_h * m.omega ** 2)
        v = np.concatenate([u[0], u[1]])
        return np.concatenate([v.real, v.imag])

    T = _tail(m, x0[1], float(np.min(-py)), 0)
    v, _, _ = sommerfeld._integrate(f, 2 * npt, sommerfeld._pieces(m, T), tol, 200000)
    return np.stack([v[:npt], v[npt:]], axis=1)


def upper_field(m: Media, x0, alpha, pts: np.ndarray, tol: float = 1e-13) -> np.ndarray:
    """u_inc + u1 at substrate points below the source (0 < y < y0)."""
    x0 = np.asarray(x0, dtype=float)
    px, py = pts[:, 0], pts[:, 1]
    npt = len(pts)

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        spb, ssb = sv[2], sv[3]
        c = densities(xi, m, x0[1], alpha, sv)[:2]
        ph = np.exp(1j * xi * (px - x0[0]))
        Gp = np.exp(-spb * py) / (4 * math.pi * spb) * ph
        Gs = np.exp(-ssb * py) / (4 * math.pi * ssb) * ph
        Dp = np.array([1j * xi, -spb])
        Ds = np.array([1j * xi, -ssb])
        u = ((m.ksb ** 2 * c + Ds * (Ds @ c))[:, None] * Gs[None, :]
             - (Dp * (Dp @ c))[:, None] * Gp[None, :]) / (m.rho_b * m.omega ** 2)
        v = np.concatenate([u[0], u[1]])
        return np.concatenate([v.real, v.imag])

    T = _tail(m, x0[1], float(np.min(py)), 0)
    v, _, _ = sommerfeld._integrate(f, 2 * npt, sommerfeld._pieces(m, T), tol, 200000)
    u1 = np.stack([v[:npt], v[npt:]], axis=1)
    return u1 + greens_tensor(m, x0, pts) @ np.asarray(alpha, dtype=complex)


def local_coefficients(w, m: Media, x0, alpha, tol: float = 1e-13) -> np.ndarray:
    """(a0, b0) of u2 about every particle centre, layout [a, b] per particle."""
    x0 = np.asarray(x0, dtype=float)
    off = w.offsets()
    n_coef = int(off[-1])
    idx = []
    for i in range(w.n):
        pm = int(w.p[i])
        idx.append((i, pm, np.arange(-pm, pm + 1)))

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        sp, ss = sv[0], sv[1]
        sig = densities(xi, m, x0[1], alpha, sv)
        s21, s22 = sig[2], sig[3]
        ph = np.exp(-1j * xi * x0[0]) / (m.rho_h * m.omega ** 2)
        phi = -(1j * xi * s21 + sp * s22) / (4 * math.pi * sp) * ph
        psi = (ss * s21 - 1j * xi * s22) / (4 * math.pi * ss) * ph
        out = np.zeros(n_coef, dtype=complex)
        for i, pm, n in idx:
            xm, ym = w.xy[i]
            a = phi * np.exp(1j * xi * xm + sp * ym) * (1j * (xi - sp) / m.kp) ** n
            b = psi * np.exp(1j * xi * xm + ss * ym) * (1j * (xi - ss) / m.ks) ** n
            out[off[i]: off[i + 1]] = np.concatenate([a, b])
        return np.concatenate([out.real, out.imag])

    T = _tail(m, x0[1], float(np.min(-w.xy[:, 1])), int(np.max(w.p)))
    v, _, _ = sommerfeld._integrate(f, n_coef, sommerfeld._pieces(m, T), tol, 200000)
    return v


def rhs(w, m: Media, S_blocks, x0, alpha, tol: float = 1e-13) -> np.ndarray:
    """S_m (a0^m, b0^m) for every particle."""
    c = local_coefficients(w, m, x0, alpha, tol)
    off = w.offsets()
    out = np.zeros_like(c)
    for i in range(w.n):
        out[off[i]: off[i + 1]] = S_blocks[i] @ c[off[i]: off[i + 1]]
    return out
