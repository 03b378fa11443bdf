"""Closed-form scattering matrices of a disk and basis rotation.

Section 4.1: the incoming field near a particle is sum_n a_n grad u_n^{kp} +
b_n grad^perp u_n^{ks} with u_n^k = J_n(k r) e^{i n theta}; the scattered field
is sum_n alpha_n grad v_n^{kp} + beta_n grad^perp v_n^{ks} with
v_n^k = H_n^{(1)}(k r) e^{i n theta}; S maps (a, b) to (alpha, beta).  For a disk
the boundary condition is imposed mode by mode (the paper cites the derivation;
it is written out here).

Polar components, with f(r) e^{i n theta}:
  grad      -> ( f'          ,  (i n / r) f )       in (r_hat, theta_hat)
  grad^perp -> ( -(i n / r) f,  f'          )

Rigid (u = 0 on r = a): M_Z = [[kp Z_n'(kp a), -(i n/a) Z_n(ks a)],
                                [(i n/a) Z_n(kp a), ks Z_n'(ks a)]]
and [alpha; beta] = -M_H^{-1} M_J [a; b].  M_H is the matrix of the paper's
direct projection formula (Section 4.3, remark on EBCM / projection).

Traction-free (sigma . r_hat = 0 on r = a): columns (sigma_rr, sigma_rtheta) of
the P potential f = Z_n(kp r) and of the S potential g = Z_n(ks r):
  P: sigma_rr = -lambda kp^2 f + 2 mu f'',  sigma_rt = 2 mu (i n / r)(f' - f / r)
  S: sigma_rr = -2 mu (i n / r)(g' - g / r), sigma_rt = mu (g'' - g'/r + n^2 g / r^2)
and [alpha; beta] = -N_H^{-1} N_J [a; b].

Coefficient layout of one particle: [alpha_{-p..p}, beta_{-p..p}] (Section 4.2,
truncation remark and the matrix form of the MS system).  S is (4p+2)^2.

Rotation (Section 4.3: rotated copies by a rotation of the basis): a particle
turned by theta0 has S_rot[n, n'] = e^{-i n theta0} S[n, n'] e^{i n' theta0} on
each of the four (2p+1)^2 sub-blocks.
"""
from __future__ import annotations

import numpy as np
from scipy import special

from .media import Media


def _zfuncs(kind: str, n: int, z: float):
    """Z_n(z), Z_n'(z), Z_n''(z) with Z = J or H^{(1)}; derivatives w.r.t. z."""
    if kind == "J":
        f0 = special.jv(n, z)
        f1 = special.jvp(n, z, 1)
    else:
        f0 = special.hankel1(n, z)
        f1 = special.h1vp(n, z, 1)
    # Bessel's equation: Z'' = -Z'/z - (1 - n^2/z^2) Z
    f2 = -f1 / z - (1.0 - n * n / (z * z)) * f0
    return f0, f1, f2


def _bc_matrix(kind: str, n: int, a: float, m: Media, bc: int) -> np.ndarray:
    kp, ks = m.kp, m.ks
    fp0, fp1, fp2 = _zfuncs(kind, n, kp * a)
    fs0, fs1, fs2 = _zfuncs(kind, n, ks * a)
    # radial derivatives of f(r) = Z_n(k r)
    f, df, d2f = fp0, kp * fp1, kp * kp * fp2
    g, dg, d2g = fs0, ks * fs1, ks * ks * fs2
    if bc == 0:
        return np.array([[df, -(1j * n / a) * g],
                         [(1j * n / a) * f, dg]], dtype=complex)
    lam, mu = m.lam_h, m.mu_h
    s_rr_p = -lam * kp * kp * f + 2 * mu * d2f
    s_rt_p = 2 * mu * (1j * n / a) * (df - f / a)
    s_rr_s = -2 * mu * (1j * n / a) * (dg - g / a)
    s_rt_s = mu * (d2g - dg / a + n * n * g / (a * a))
    return np.array([[s_rr_p, s_rr_s], [s_rt_p, s_rt_s]], dtype=complex)


def disk(m: Media, a: float, p: int, bc: int) -> np.ndarray:
    """(4p+2)x(4p+2) scattering matrix of a disk of radius a (bc 0 rigid, 1 free)."""
    N = 2 * p + 1
    S = np.zeros((2 * N, 2 * N), dtype=complex)
    for n in range(-p, p + 1):
        MJ = _bc_matrix("J", n, a, m, bc)
        MH = _bc_matrix("H", n, a, m, bc)
        blk = -np.linalg.solve(MH, MJ)
        k = n + p
        S[k, k] = blk[0, 0]
        S[k, N + k] = blk[0, 1]
        S[N + k, k] = blk[1, 0]
        S[N + k, N + k] = blk[1, 1]
    return S


def rotate(S: np.ndarray, p: int, theta0: float) -> np.ndarray:
    """Basis rotation of a prototype S by theta0."""
    n = np.arange(-p, p + 1)
    ph = np.exp(-1j * n * theta0)
    d = np.concatenate([ph, ph])
    return d[:, None] * S * np.conj(d)[None, :]


def projection_matrix(m: Media, R: float, n: int) -> np.ndarray:
    """M_H of the direct projection formula (Section 4.3 remark)."""
    kp, ks = m.kp, m.ks
    return np.array([[kp * special.h1vp(n, kp * R), -(1j * n / R) * special.hankel1(n, ks * R)],
                     [(1j * n / R) * special.hankel1(n, kp * R), ks * special.h1vp(n, ks * R)]])


def workload_blocks(w, m: Media | None = None) -> list:
    """Per-particle S blocks of a workload whose particles are all circles."""
    if m is None:
        m = Media.from_workload(w)
    if np.any(w.shape != 0):
        raise ValueError("the oracle has closed-form S only for circles")
    cache = {}
    out = []
    for a, pm, bc in zip(w.radius, w.p, w.bc):
        key = (float(a), int(pm), int(bc))
        if key not in cache:
            cache[key] = disk(m, float(a), int(pm), int(bc))
        out.append(cache[key])
    return out
