"""Layered reflected part of the operator by Sommerfeld integrals (Section 5).

Multipole-to-Sommerfeld (Section 5.4, Lemma): for y > y_m,
  H_n(k r) e^{i n theta} = ((-1)^n / (i pi)) int e^{s (y_m - y)} / s
                            e^{i xi (x - x_m)} ((s - xi)/(i k))^n dxi,
with s = sqrt(xi^2 - k^2).  Since (-1)^n ((s - xi)/(i k))^n = (-i zeta)^n with
zeta = (xi - s)/k, the upgoing P potential of all particles is
  int I_p(xi) e^{i xi x - s_p y} dxi,
  I_p(xi) = sum_m e^{s_p y_m - i xi x_m} / (i pi s_p) sum_n alpha^m_n (-i zeta_p)^n,
and the S potential the same with (beta, ks).

Reflection (Section 3.2 per mode; the Schur complement of Section 5.2 applies
A^{-1} node by node): [RP; RS] = R(xi) [I_p; I_s] are the amplitudes of the
reflected potentials e^{i xi x + s y} in the host.

Sommerfeld-to-local (Section 5.3, Jacobi-Anger): e^{i xi x + s y} =
e^{i xi x_l + s y_l} sum_n (i zeta)^n J_n(k r_l) e^{i n theta_l}, hence
  a^l_n = int e^{i xi x_l + s_p y_l} (i zeta_p)^n RP(xi) dxi,
  b^l_n = int e^{i xi x_l + s_s y_l} (i zeta_s)^n RS(xi) dxi,
for every particle l, the particle itself included (the Schur complement
couples every pair through the interface).

The oracle integrates on the real xi axis (the paper's contour is a
deformation of it, Section 5.1) with adaptive Gauss-Kronrod quadrature
(scipy.integrate.quad_vec, a library primitive), breaking at every branch point
+-kp, +-ks, +-kpb, +-ksb and substituting xi = k +- u^2 on a short piece next to
each branch point so that the 1/sqrt singularities become smooth.  The tails
stop where exp(-|xi| D_min) (2|xi|/k_min)^(2 p_max) has fallen by 1e-18 from
its peak.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from . import interface
from .media import Media


class _Groups:
    """Particles grouped by truncation order, for vectorised evaluation."""

    def __init__(self, w, idx):
        self.items = []
        off = w.offsets()
        for pv in np.unique(w.p[idx]):
            sel = np.asarray([i for i in idx if w.p[i] == pv], dtype=int)
            self.items.append((int(pv), sel, w.xy[sel, 0].copy(), w.xy[sel, 1].copy(),
                               off[sel].copy()))


def _integrand_factory(w, m: Media, x: np.ndarray, targets, S_blocks, R_fun):
    kp, ks = m.kp, m.ks
    off = w.offsets()
    src = _Groups(w, range(w.n))
    tgt = _Groups(w, list(targets))
    src_coef = []
    for pv, sel, xs, ys, o in src.items:
        N = 2 * pv + 1
        idx = o[:, None] + np.arange(2 * N)[None, :]
        c = x[idx]
        src_coef.append((c[:, :N], c[:, N:]))
    out_len = int(sum(2 * (2 * pv + 1) * len(sel) for pv, sel, *_ in tgt.items))

    def f(xi: float, bp=None, d=None) -> np.ndarray:
        sv = interface.s_values(xi, m, bp, d)
        sp, ss = sv[0], sv[1]
        zp = (xi - sp) / kp
        zs = (xi - ss) / ks
        Ip = 0j
        Is = 0j
        for (pv, sel, xs, ys, o), (ca, cb) in zip(src.items, src_coef):
            n = np.arange(-pv, pv + 1)
            Ep = np.exp(sp * ys - 1j * xi * xs)
            Es = np.exp(ss * ys - 1j * xi * xs)
            Ip += np.sum(Ep * (ca @ ((-1j * zp) ** n)))
            Is += np.sum(Es * (cb @ ((-1j * zs) ** n)))
        Ip /= 1j * math.pi * sp
        Is /= 1j * math.pi * ss
        R = R_fun(xi, sv)
        RP = R[0, 0] * Ip + R[0, 1] * Is
        RS = R[1, 0] * Ip + R[1, 1] * Is
        parts = []
        for pv, sel, xt, yt, o in tgt.items:
            n = np.arange(-pv, pv + 1)
            ea = np.exp(1j * xi * xt + sp * yt)[:, None] * ((1j * zp) ** n)[None, :] * RP
            eb = np.exp(1j * xi * xt + ss * yt)[:, None] * ((1j * zs) ** n)[None, :] * RS
            blk = np.concatenate([ea, eb], axis=1)           # [L, 4pv+2]
            if S_blocks is not None:
                blk = np.stack([S_blocks[l] @ blk[k] for k, l in enumerate(sel)])
            parts.append(blk.ravel())
        v = np.concatenate(parts)
        return np.concatenate([v.real, v.imag])

    return f, out_len, tgt


def tail_extent(w, m: Media, drop: float = 1e-18) -> float:
    """Where exp(-|xi| D_min) (2|xi|/k_min + 1)^(2 p_max) has decayed by ``drop``."""
    kmin = min(m.kp, m.ks)
    kmax = max(m.kp, m.ks, m.kpb, m.ksb)
    dmin = 2.0 * float(np.min(-w.xy[:, 1]))
    pm = 2 * int(np.max(w.p))
    t = np.linspace(0.0, 5000.0, 500001)
    logb = -t * dmin + pm * np.log(2.0 * t / kmin + 1.0)
    peak = float(np.max(logb))
    ok = np.nonzero((logb < peak + math.log(drop)) & (t > kmax + 2.0))[0]
    return float(t[ok[0]])


def _pieces(m: Media, T: float, sub_len: float = 0.5):
    """Real-axis pieces: (kind, a, b) where kind 0 plain, +1 xi = a + u^2, -1 xi = b - u^2."""
    ks_ = sorted(set([m.kp, m.ks, m.kpb, m.ksb]))
    bps = sorted([-k for k in ks_] + ks_)
    edges = [-T] + bps + [T]
    pieces = []
    for a, b in zip(edges[:-1], edges[1:]):
        left_sing = a in bps
        right_sing = b in bps
        L = b - a
        la = min(sub_len, L / 2) if left_sing else 0.0
        lb = min(sub_len, L / 2) if right_sing else 0.0
        if la > 0:
            pieces.append((+1, a, a + la))
        if b - lb > a + la:
            pieces.append((0, a + la, b - lb))
        if lb > 0:
            pieces.append((-1, b - lb, b))
    return pieces


def _integrate(f, out_len, pieces, tol, limit, floor=0.0):
    """Sum of adaptive integrals over the pieces, real-valued output vector."""
    def wrap(kind, a, b):
        # on a substituted piece the exact offset u^2 from the branch point is
        # passed along, so s = sqrt(d (2 bp + d)) loses nothing to cancellation
        if kind == 0:
            return (lambda t: f(t)), a, b
        if kind == +1:
            return (lambda u: f(a + u * u, a, u * u) * (2.0 * u)), 0.0, math.sqrt(b - a)
        return (lambda u: f(b - u * u, b, -u * u) * (2.0 * u)), 0.0, math.sqrt(b - a)

    # coarse pass to set the absolute error scale
    coarse = np.zeros(2 * out_len)
    for kind, a, b in pieces:
        g, lo, hi = wrap(kind, a, b)
        r, _ = integrate.quad_vec(g, lo, hi, epsrel=1e-6, epsabs=0.0, norm="2", limit=limit)
        coarse += r
    scale = float(np.linalg.norm(coarse))
    total = np.zeros(2 * out_len)
    err_tot = 0.0
    eabs = tol * max(scale, floor, 1e-300) / math.sqrt(len(pieces))
    for kind, a, b in pieces:
        g, lo, hi = wrap(kind, a, b)
        r, e = integrate.quad_vec(g, lo, hi, epsrel=0.0, epsabs=eabs, norm="2", limit=limit)
        total += r
        err_tot += e * e
    v = total[:out_len] + 1j * total[out_len:]
    return v, math.sqrt(err_tot), scale


def apply_refl(w, m: Media, x: np.ndarray, targets=None, S_blocks=None, R_fun=None,
               tol: float = 1e-13, limit: int = 200000, T: float | None = None,
               return_info: bool = False, floor: float = 0.0):
    """T_refl x (or S T_refl x when S_blocks is given), rows of ``targets`` only.

    Returns a full-length vector with zeros on the rows not requested.
    ``R_fun`` replaces the interface reflection (xi -> 2x2), e.g. a constant
    diagonal for the image-source check.  ``floor`` is a lower bound on the
    norm used for the absolute error target (for results that vanish).
    """
    if targets is None:
        targets = list(range(w.n))
    if R_fun is None:
        R_fun = lambda xi, sv: interface.reflection(xi, m, sv)  # noqa: E731
    else:
        user_R = R_fun
        R_fun = lambda xi, sv: user_R(xi)  # noqa: E731
    f0, out_len, tgt = _integrand_factory(w, m, np.asarray(x, complex), targets, S_blocks, R_fun)
    neval = [0]

    def f(*a):
        neval[0] += 1
        return f0(*a)

    if T is None:
        T = tail_extent(w, m)
    pieces = _pieces(m, T)
    v, err, scale = _integrate(f, out_len, pieces, tol, limit, floor)
    y = np.zeros(len(x), dtype=complex)
    off = w.offsets()
    pos = 0
    for pv, sel, *_ in tgt.items:
        blk = 2 * (2 * pv + 1)
        for l in sel:
            y[off[l]: off[l] + blk] = v[pos: pos + blk]
            pos += blk
    if return_info:
        return y, {"err": err, "scale": scale, "T": T, "pieces": len(pieces), "neval": neval[0]}
    return y

