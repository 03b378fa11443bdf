"""Welded-interface reflection of plane-wave potentials, one Fourier mode at a time.

Section 3.2: the Sommerfeld representation diagonalises the tangential
variable, so continuity of displacement and traction T_y across y = 0 is
imposed per mode xi (the paper's 4x4 system A_xi sigma = b_xi, written there
with rho = 1 for densities on the interface).  The oracle writes the same four
conditions for potentials (density kept):

A potential e^{i xi x + q y} in a medium (lambda, mu, rho) gives
(u1, u2, t1, t2) with t = T_y u = (mu(d_y u1 + d_x u2), (lambda+2mu) d_y u2 + lambda d_x u1):
  P (u = grad phi):        (i xi, q, 2 mu i xi q, (lambda + 2 mu) q^2 - lambda xi^2)
  S (u = grad^perp psi):   (-q, i xi, -mu (q^2 + xi^2), 2 mu i xi q)

Branch (the paper asks only for decay away from the interface): s(xi; k) =
-i sqrt(k^2 - xi^2) with the principal root; on the real axis s > 0 for
|xi| > k and s = -i sqrt(k^2 - xi^2) for |xi| < k, chosen by cases.
In the host (y < 0) the wave going up to the interface is e^{i xi x - s y},
the reflected one e^{i xi x + s y}; in the substrate the transmitted one is
e^{i xi x - s_b y}.

R(xi) is the top 2x2 block of X in
  [P_h(+s_p), S_h(+s_s), -P_b(-s_pb), -S_b(-s_sb)] X = -[P_h(-s_p), S_h(-s_s)],
column 0 answering a unit upgoing P potential, column 1 a unit S potential.
The bottom 2x2 block is the transmission T(xi).
"""
from __future__ import annotations

import math

import numpy as np

from .media import Media


def branch_s(xi, k: float):
    """s(xi; k) = sqrt(xi^2 - k^2) with Re s >= 0 (decaying branch).

    Real xi is split by cases; complex xi with Im(k^2 - xi^2) >= 0 uses the
    principal root of k^2 - xi^2.
    """
    xi = np.asarray(xi)
    if np.isrealobj(xi):
        xr = xi.astype(float)
        out = np.where(np.abs(xr) > k, np.sqrt(np.maximum(xr * xr - k * k, 0.0)) + 0j,
                       -1j * np.sqrt(np.maximum(k * k - xr * xr, 0.0)))
        return out
    return -1j * np.sqrt(k * k - xi * xi)


def branch_s_offset(bp: float, d: float, k: float):
    """s at xi = bp + d exactly, bp = +-k: xi^2 - k^2 = d (2 bp + d), no cancellation."""
    v = d * (2.0 * bp + d)
    return math.sqrt(v) + 0j if v > 0 else -1j * math.sqrt(max(-v, 0.0))


def s_values(xi, m: Media, bp=None, d=None):
    """(s_p, s_s, s_pb, s_sb) at xi; with (bp, d) the wavenumber equal to |bp| uses the offset."""
    out = []
    for k in (m.kp, m.ks, m.kpb, m.ksb):
        if bp is not None and abs(abs(bp) - k) <= 1e-14 * k:
            out.append(branch_s_offset(bp, d, k))
        else:
            out.append(complex(branch_s(xi, k)))
    return out


def _cols(xi, q, lam, mu):
    P = np.array([1j * xi, q, 2 * mu * 1j * xi * q, (lam + 2 * mu) * q * q - lam * xi * xi])
    S = np.array([-q, 1j * xi, -mu * (q * q + xi * xi), 2 * mu * 1j * xi * q])
    return P, S


def system(xi, m: Media, svals=None):
    """The 4x4 matrix and 4x2 right-hand side at one xi."""
    sp, ss, spb, ssb = svals if svals is not None else s_values(xi, m)
    Pr, _ = _cols(xi, +sp, m.lam_h, m.mu_h)
    _, Sr = _cols(xi, +ss, m.lam_h, m.mu_h)
    Pi, _ = _cols(xi, -sp, m.lam_h, m.mu_h)
    _, Si = _cols(xi, -ss, m.lam_h, m.mu_h)
    Pt, _ = _cols(xi, -spb, m.lam_b, m.mu_b)
    _, St = _cols(xi, -ssb, m.lam_b, m.mu_b)
    M = np.stack([Pr, Sr, -Pt, -St], axis=1)
    rhs = -np.stack([Pi, Si], axis=1)
    return M, rhs


def reflect_transmit(xi, m: Media, svals=None):
    """(R, T), each 2x2, at one scalar xi."""
    M, rhs = system(xi, m, svals)
    X = np.linalg.solve(M, rhs)
    return X[:2, :], X[2:, :]


def from_substrate(xi, m: Media, svals=None):
    """(Td, Rb), each 2x2, for waves sent from the substrate (Section 7.3's
    plane-wave setup): a unit downgoing potential e^{i xi x + s_b y} (column
    0 P, column 1 S) meets the same four continuity conditions with the
    unknowns host downgoing (Td, e^{i xi x + s y}) and substrate upgoing (Rb,
    e^{i xi x - s_b y}):
      [P_h(+s_p), S_h(+s_s), -P_b(-s_pb), -S_b(-s_sb)] X = [P_b(+s_pb), S_b(+s_sb)].
    """
    sp, ss, spb, ssb = svals if svals is not None else s_values(xi, m)
    M, _ = system(xi, m, (sp, ss, spb, ssb))
    Pd, _ = _cols(xi, +spb, m.lam_b, m.mu_b)
    _, Sd = _cols(xi, +ssb, m.lam_b, m.mu_b)
    X = np.linalg.solve(M, np.stack([Pd, Sd], axis=1))
    return X[:2, :], X[2:, :]


def reflection(xi, m: Media, svals=None) -> np.ndarray:
    return reflect_transmit(xi, m, svals)[0]


def reflection_many(xis, m: Media) -> np.ndarray:
    """R at many real xi: array [len(xis), 2, 2]."""
    return np.stack([reflection(float(x) if np.isrealobj(x) else x, m) for x in np.asarray(xis)])
