"""Receiver-misfit gradient by forward-mode (tangent) differentiation.

TEST INFRASTRUCTURE ONLY: a plain dense computation for small clouds.

Misfit J = 1/2 sum_r sum_rcv |u_r(x_rcv) - u_obs,r|^2 with u_r = F gamma_r,
A gamma_r = b_r the Schur system of Sections 4.2 and 5.2 (A = I - S (T_free +
T_refl), b = S a0 with a0 the background local coefficients, Section 7.3),
F the scattered-field map (Section 5, coupled representation).  Parameters:
every centre coordinate and the substrate's (lambda_b, mu_b).  For each
parameter theta the tangent gamma' = A^{-1} (b' - A' gamma) gives
  dJ/dtheta = Re sum_r res_r^H (F' gamma_r + F gamma'_r),
with every derivative taken from its definition:
  * Graf blocks: chain rule on H_nu(k r) e^{-i nu (th - pi)} in polar
    coordinates of X = x_m - x_l (d r = (cos, sin) . dX, d th = (-sin, cos) . dX / r);
  * reflected operator and field: derivative of the plane-wave factors under
    the integral, -i xi / s on a source's e^{s y - i xi x}, i xi / s on a
    target's e^{i xi x + s y}, and dR(xi) for the Lame parameters;
  * outgoing fields at the receivers: Hessian of H_n(k r) e^{i n th} from the
    polar chain rule and Bessel's equation;
  * background coefficients: i xi0 and -+s on the down-/up-going plane waves,
    dR(xi0) for the reflected one.
dR comes from differentiating the interface system M X = rhs of Section 3.2:
dX = -M^{-1} (dM) X, only the substrate columns depending on (lambda_b, mu_b)
(explicitly and through s_pb, s_sb).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import linalg, special

from . import graf, interface, smatrix, sommerfeld
from .media import Media


# ---------------------------------------------------------------------------
# interface derivative

def _dcols(xi, q, dq, lam, mu, which):
    """d/dtheta of the P and S potential columns (theta = lambda (0) or mu (1))."""
    dP = np.array([0.0, dq, 2 * mu * 1j * xi * dq, 2 * (lam + 2 * mu) * q * dq], dtype=complex)
    dS = np.array([-dq, 0.0, -2 * mu * q * dq, 2 * mu * 1j * xi * dq], dtype=complex)
    if which == 0:
        dP[3] += q * q - xi * xi
    else:
        dP[2] += 2j * xi * q
        dP[3] += 2 * q * q
        dS[2] += -(q * q + xi * xi)
        dS[3] += 2j * xi * q
    return dP, dS


def reflection_tangent(xi, m: Media, svals=None):
    """(R, dR/dlambda_b, dR/dmu_b), each 2x2."""
    sv = svals if svals is not None else interface.s_values(xi, m)
    M, rhs = interface.system(xi, m, sv)
    X = np.linalg.solve(M, rhs)
    spb, ssb = sv[2], sv[3]
    lp = m.lam_b + 2 * m.mu_b
    out = [X[:2, :]]
    for which in (0, 1):
        dspb = (1.0 if which == 0 else 2.0) * m.kpb ** 2 / (2 * spb * lp)
        dssb = 0.0 if which == 0 else m.ksb ** 2 / (2 * ssb * m.mu_b)
        dPt, _ = _dcols(xi, -spb, -dspb, m.lam_b, m.mu_b, which)
        _, dSt = _dcols(xi, -ssb, -dssb, m.lam_b, m.mu_b, which)
        dM = np.zeros((4, 4), dtype=complex)
        dM[:, 2] = -dPt
        dM[:, 3] = -dSt
        dX = np.linalg.solve(M, -dM @ X)
        out.append(dX[:2, :])
    return out


# ---------------------------------------------------------------------------
# free part

def graf_block_tangent(k, xm, xl, pm, pl):
    """(T, dT/dX_x, dT/dX_y) of one Graf block, X = x_m - x_l."""
    d = np.asarray(xm, float) - np.asarray(xl, float)
    r = float(np.hypot(d[0], d[1]))
    th = float(np.arctan2(d[1], d[0]))
    c, s = math.cos(th), math.sin(th)
    nu = np.arange(-pm, pm + 1)[:, None] - np.arange(-pl, pl + 1)[None, :]
    E = np.exp(-1j * nu * (th - np.pi))
    H = special.hankel1(nu, k * r)
    Hp = special.h1vp(nu, k * r)
    dr = k * Hp * E
    dth = H * (-1j * nu) * E
    return H * E, dr * c - dth * s / r, dr * s + dth * c / r


def free_tangent(w, m: Media):
    """Dense T_free and its derivatives, list over particles q of (dT/dx_q, dT/dy_q)."""
    off = w.offsets()
    nc = int(off[-1])
    T = np.zeros((nc, nc), dtype=complex)
    dT = [[np.zeros((nc, nc), dtype=complex), np.zeros((nc, nc), dtype=complex)] for _ in range(w.n)]
    for a in range(w.n):
        for b in range(w.n):
            if a == b:
                continue
            pa, pb = int(w.p[a]), int(w.p[b])
            Na, Nb = 2 * pa + 1, 2 * pb + 1
            for wv, k in enumerate((m.kp, m.ks)):
                B, Bx, By = graf_block_tangent(k, w.xy[a], w.xy[b], pa, pb)
                ra = slice(off[a] + wv * Na, off[a] + (wv + 1) * Na)
                cb = slice(off[b] + wv * Nb, off[b] + (wv + 1) * Nb)
                T[ra, cb] = B
                dT[a][0][ra, cb] += Bx
                dT[a][1][ra, cb] += By
                dT[b][0][ra, cb] -= Bx
                dT[b][1][ra, cb] -= By
    return T, dT


# ---------------------------------------------------------------------------
# outgoing fields at receivers

def _hess_cyl(n, k, dx, dy):
    """(f, f_x, f_y, f_xx, f_xy, f_yy) of f = H_n(k r) e^{i n th}."""
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    c, s = np.cos(th), np.sin(th)
    z = k * r
    E = np.exp(1j * n * th)
    Z = special.hankel1(n, z)
    Zp = special.h1vp(n, z)
    Zpp = -Zp / z - (1.0 - n * n / (z * z)) * Z       # Bessel's equation
    f = Z * E
    fr = k * Zp * E
    frr = k * k * Zpp * E
    ft = 1j * n * f
    frt = 1j * n * fr
    ftt = -n * n * f
    fx = c * fr - s / r * ft
    fy = s * fr + c / r * ft
    fxx = c * c * frr - 2 * c * s / r * frt + s * s / r * fr + 2 * c * s / r ** 2 * ft + s * s / r ** 2 * ftt
    fyy = s * s * frr + 2 * c * s / r * frt + c * c / r * fr - 2 * c * s / r ** 2 * ft + c * c / r ** 2 * ftt
    fxy = (c * s * frr + (c * c - s * s) / r * frt - c * s / r * fr
           - (c * c - s * s) / r ** 2 * ft - c * s / r ** 2 * ftt)
    return f, fx, fy, fxx, fxy, fyy


def direct_field_tangent(w, m: Media, pts):
    """Dense F_direct [2 npts, nc] (rows x-components then y-components) and
    dF/dx_q, dF/dy_q per particle."""
    off = w.offsets()
    nc = int(off[-1])
    npt = len(pts)
    F = np.zeros((2 * npt, nc), dtype=complex)
    dF = [[np.zeros((2 * npt, nc), dtype=complex), np.zeros((2 * npt, nc), dtype=complex)]
          for _ in range(w.n)]
    for i in range(w.n):
        pm = int(w.p[i])
        N = 2 * pm + 1
        dx = pts[:, 0] - w.xy[i, 0]
        dy = pts[:, 1] - w.xy[i, 1]
        for kk, n in enumerate(range(-pm, pm + 1)):
            _, fx, fy, fxx, fxy, fyy = _hess_cyl(n, m.kp, dx, dy)
            ca = off[i] + kk
            F[:npt, ca], F[npt:, ca] = fx, fy
            # moving the centre: d/dx_i = -d/dx of the field
            dF[i][0][:npt, ca], dF[i][0][npt:, ca] = -fxx, -fxy
            dF[i][1][:npt, ca], dF[i][1][npt:, ca] = -fxy, -fyy
            _, gx, gy, gxx, gxy, gyy = _hess_cyl(n, m.ks, dx, dy)
            cb = off[i] + N + kk
            F[:npt, cb], F[npt:, cb] = -gy, gx
            dF[i][0][:npt, cb], dF[i][0][npt:, cb] = gxy, -gxx
            dF[i][1][:npt, cb], dF[i][1][npt:, cb] = gyy, -gxy
    return F, dF


# ---------------------------------------------------------------------------
# reflected operator and field (one stacked matrix-valued Sommerfeld integral)

def _tail(w, m: Media, pts, drop=1e-18, extra=2):
    """Where the slowest integrand envelope exp(-|xi| D) (2|xi|/k_min + 1)^P has
    fallen by ``drop``; D from the shallowest particle and receiver."""
    kmin = min(m.kp, m.ks)
    kmax = max(m.kp, m.ks, m.kpb, m.ksb)
    dpart = float(np.min(-w.xy[:, 1]))
    D = 2 * dpart
    if pts is not None and len(pts):
        D = min(D, dpart + float(np.min(-pts[:, 1])))
    P = 2 * int(np.max(w.p)) + extra
    t = np.linspace(0.0, 20000.0, 2000001)
    logb = -t * D + P * np.log(2.0 * t / kmin + 1.0)
    peak = float(np.max(logb))
    ok = np.nonzero((logb < peak + math.log(drop)) & (t > kmax + 2.0))[0]
    return float(t[ok[0]])


def refl_tangent(w, m: Media, pts, tol=1e-13, limit=200000, derivs=True):
    """Dense T_refl [nc, nc] and F_refl [2 npts, nc] and, with ``derivs``, their
    derivatives: lists over particles of (d/dx_q, d/dy_q) and (d/dlambda_b, d/dmu_b)."""
    off = w.offsets()
    nc = int(off[-1])
    npt = 0 if pts is None else len(pts)
    n = w.n
    nmat = 1 + (2 * n + 2 if derivs else 0)
    size_T = nc * nc
    size_F = 2 * npt * nc
    out_len = nmat * (size_T + size_F)
    kp, ks = m.kp, m.ks
    rows_w = np.zeros(nc, dtype=int)
    part = np.zeros(nc, dtype=int)
    modes = np.zeros(nc, dtype=int)
    for i in range(n):
        N = 2 * int(w.p[i]) + 1
        part[off[i]:off[i + 1]] = i
        rows_w[off[i] + N:off[i + 1]] = 1
        modes[off[i]:off[i + 1]] = np.concatenate([np.arange(-w.p[i], w.p[i] + 1)] * 2)
    xs, ys = w.xy[part, 0], w.xy[part, 1]

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        sp, ss = sv[0], sv[1]
        s_of = np.where(rows_w == 0, sp, ss)
        k_of = np.where(rows_w == 0, kp, ks)
        z = (xi - s_of) / k_of
        # B: 2 x nc (row w only on its wave's columns); C: nc x 2
        bval = np.exp(s_of * ys - 1j * xi * xs) * (-1j * z) ** modes / (1j * math.pi * s_of)
        cval = np.exp(1j * xi * xs + s_of * ys) * (1j * z) ** modes
        B = np.zeros((2, nc), dtype=complex)
        C = np.zeros((nc, 2), dtype=complex)
        B[rows_w, np.arange(nc)] = bval
        C[np.arange(nc), rows_w] = cval
        if derivs:
            R, dRl, dRm = reflection_tangent(xi, m, sv)
        else:
            R = interface.reflection(xi, m, sv)
        mats_T = [C @ R @ B]
        if npt:
            ep = np.exp(1j * xi * pts[:, 0] + sp * pts[:, 1])
            es = np.exp(1j * xi * pts[:, 0] + ss * pts[:, 1])
            G = np.zeros((2 * npt, 2), dtype=complex)
            G[:npt, 0], G[:npt, 1] = 1j * xi * ep, -ss * es
            G[npt:, 0], G[npt:, 1] = sp * ep, 1j * xi * es
            mats_F = [G @ R @ B]
        else:
            mats_F = [np.zeros((0, nc))]
        if derivs:
            CR = C @ R
            RB = R @ B
            for q in range(n):
                sel = part == q
                for fac_src, fac_tgt in ((-1j * xi, 1j * xi), (s_of, s_of)):
                    fs = np.where(sel, fac_src, 0.0)
                    ft = np.where(sel, fac_tgt, 0.0)
                    Bq = B * fs[None, :]
                    Cq = C * ft[:, None]
                    mats_T.append(Cq @ RB + CR @ Bq)
                    mats_F.append(G @ R @ Bq if npt else np.zeros((0, nc)))
            for dR in (dRl, dRm):
                mats_T.append(C @ dR @ B)
                mats_F.append(G @ dR @ B if npt else np.zeros((0, nc)))
        v = np.concatenate([np.concatenate([a.ravel() for a in mats_T]),
                            np.concatenate([a.ravel() for a in mats_F])])
        return np.concatenate([v.real, v.imag])

    T = _tail(w, m, pts, extra=4 if derivs else 2)
    pieces = sommerfeld._pieces(m, T)
    v, _, _ = sommerfeld._integrate(f, out_len, pieces, tol, limit)
    vt, vf = v[:nmat * size_T], v[nmat * size_T:]
    Ts = [vt[k * size_T:(k + 1) * size_T].reshape(nc, nc) for k in range(nmat)]
    Fs = [vf[k * size_F:(k + 1) * size_F].reshape(2 * npt, nc) for k in range(nmat)]
    if not derivs:
        return Ts[0], Fs[0]
    dT = [[Ts[1 + 2 * q], Ts[2 + 2 * q]] for q in range(n)]
    dF = [[Fs[1 + 2 * q], Fs[2 + 2 * q]] for q in range(n)]
    return Ts[0], Fs[0], dT, dF, [Ts[-2], Ts[-1]], [Fs[-2], Fs[-1]]


# ---------------------------------------------------------------------------
# background coefficients

def background_tangent(w, m: Media, wave: int, angle: float):
    """a0 and its derivatives: list over particles of (d/dx_q, d/dy_q), and (d/dlambda_b, d/dmu_b)."""
    kp, ks = m.kp, m.ks
    k = kp if wave == 0 else ks
    xi0 = k * math.sin(angle)
    A = 1.0 / (1j * k)
    amp_in = np.array([A, 0.0]) if wave == 0 else np.array([0.0, A])
    R, dRl, dRm = reflection_tangent(xi0, m)
    sp = complex(interface.branch_s(xi0, kp))
    ss = complex(interface.branch_s(xi0, ks))
    off = w.offsets()
    nc = int(off[-1])
    a0 = np.zeros(nc, dtype=complex)
    d = [[np.zeros(nc, dtype=complex), np.zeros(nc, dtype=complex)] for _ in range(w.n)]
    dl = [np.zeros(nc, dtype=complex), np.zeros(nc, dtype=complex)]
    for i in range(w.n):
        pm = int(w.p[i])
        n = np.arange(-pm, pm + 1)
        x0, y0 = w.xy[i]
        sl = slice(off[i], off[i + 1])
        parts = []
        for wv, (s, kk) in enumerate(((sp, kp), (ss, ks))):
            up = np.exp(1j * xi0 * x0 + s * y0) * (1j * (xi0 - s) / kk) ** n      # reflected
            dn = np.exp(1j * xi0 * x0 - s * y0) * (1j * (xi0 + s) / kk) ** n      # incident
            parts.append((up, dn, s))
        val = []
        dx = []
        dy = []
        dlam = [[], []]
        for wv, (up, dn, s) in enumerate(parts):
            ar = (R @ amp_in)[wv]
            ai = amp_in[wv]
            val.append(ar * up + ai * dn)
            dx.append(1j * xi0 * (ar * up + ai * dn))
            dy.append(s * ar * up - s * ai * dn)
            for t, dR in enumerate((dRl, dRm)):
                dlam[t].append((dR @ amp_in)[wv] * up)
        a0[sl] = np.concatenate(val)
        d[i][0][sl] = np.concatenate(dx)
        d[i][1][sl] = np.concatenate(dy)
        dl[0][sl] = np.concatenate(dlam[0])
        dl[1][sl] = np.concatenate(dlam[1])
    return a0, d, dl


# ---------------------------------------------------------------------------
# misfit and gradient

def _s_matrix(w, S_blocks):
    off = w.offsets()
    nc = int(off[-1])
    S = np.zeros((nc, nc), dtype=complex)
    for i in range(w.n):
        S[off[i]:off[i + 1], off[i]:off[i + 1]] = S_blocks[i]
    return S


def misfit(w, m: Media, S_blocks, waves, pts, u_obs, tol=1e-13):
    """J, the solutions gamma [nw, nc] and the fields u [nw, npts, 2]."""
    S = _s_matrix(w, S_blocks)
    Tf, _ = free_tangent(w, m)
    Tr, Fr = refl_tangent(w, m, pts, tol=tol, derivs=False)
    Fd, _ = direct_field_tangent(w, m, pts)
    A = np.eye(S.shape[0]) - S @ (Tf + Tr)
    F = Fd + Fr
    npt = len(pts)
    J = 0.0
    gams, us = [], []
    for r, (wave, ang) in enumerate(waves):
        a0, _, _ = background_tangent(w, m, wave, ang)
        g = np.linalg.solve(A, S @ a0)
        u = F @ g
        u2 = np.stack([u[:npt], u[npt:]], axis=1)
        J += 0.5 * float(np.sum(np.abs(u2 - u_obs[r]) ** 2))
        gams.append(g)
        us.append(u2)
    return J, np.array(gams), np.array(us)


def gradient(w, m: Media, S_blocks, waves, pts, u_obs, tol=1e-13):
    """(J, dJ/dxy [n, 2], (dJ/dlambda_b, dJ/dmu_b)) by forward-mode tangents."""
    S = _s_matrix(w, S_blocks)
    Tf, dTf = free_tangent(w, m)
    Tr, Fr, dTr, dFr, dTl, dFl = refl_tangent(w, m, pts, tol=tol, derivs=True)
    Fd, dFd = direct_field_tangent(w, m, pts)
    nc = S.shape[0]
    A = np.eye(nc) - S @ (Tf + Tr)
    F = Fd + Fr
    lu = linalg.lu_factor(A)
    npt = len(pts)
    n = w.n
    J = 0.0
    gxy = np.zeros((n, 2))
    glame = np.zeros(2)
    for r, (wave, ang) in enumerate(waves):
        a0, da0, da0l = background_tangent(w, m, wave, ang)
        g = linalg.lu_solve(lu, S @ a0)
        u = F @ g
        res = u - np.concatenate([u_obs[r][:, 0], u_obs[r][:, 1]])
        J += 0.5 * float(np.vdot(res, res).real)

        def dJ(dA, db, dF):
            gt = linalg.lu_solve(lu, db - dA @ g)
            return float(np.vdot(res, dF @ g + F @ gt).real)

        for q in range(n):
            for c in range(2):
                dA = -S @ (dTf[q][c] + dTr[q][c])
                gxy[q, c] += dJ(dA, S @ da0[q][c], dFd[q][c] + dFr[q][c])
        for t in range(2):
            glame[t] += dJ(-S @ dTl[t], S @ da0l[t], dFl[t])
    return J, gxy, glame


def perturbed(w, m: Media, dxy=None, dlame=(0.0, 0.0)):
    """(workload, media) with centres moved by dxy [n, 2] and (lambda_b, mu_b) shifted."""
    w2 = w if dxy is None else dataclasses.replace(w, xy=w.xy + dxy)
    m2 = dataclasses.replace(m, lam_b=m.lam_b + dlame[0], mu_b=m.mu_b + dlame[1])
    return w2, m2


def smatrix_blocks(w, m: Media):
    return smatrix.workload_blocks(w, m)
