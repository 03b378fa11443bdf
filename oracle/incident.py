"""Plane-wave right-hand side (Section 6.3 and the preconditioned system of Section 3.2).

The background field in the host is the incident plane wave plus its
interface reflection (Section 2: total = background + scattered; Section 6.3:
reflected and transmitted fields of a plane wave are plane waves).  Waves are
sent from the particle side towards the interface: paper-frame direction
d = (sin th, cos th).  A P wave of unit displacement d e^{i kp d.x} is grad of
phi = A e^{i xi0 x - s_p(xi0) y}, A = 1/(i kp), xi0 = kp sin th; an SV wave
d_perp e^{i ks d.x} (d_perp = (-d2, d1)) is grad^perp of A e^{i xi0 x - s_s y},
A = 1/(i ks), xi0 = ks sin th.  The reflected potentials are R(xi0) times the
incident ones.

Local (Jacobi-Anger) coefficients of the plane wave e^{i xi x - s y} about a
centre (x_m, y_m): e^{i xi x_m - s y_m} (i (xi + s)/k)^n; of e^{i xi x + s y}:
e^{i xi x_m + s y_m} (i (xi - s)/k)^n.  The right-hand side of the
S-preconditioned system is S_m (a0, b0) for every particle.
"""
from __future__ import annotations

import math

import numpy as np

from . import interface
from .media import Media


def local_coefficients(w, m: Media, wave: int, angle: float) -> np.ndarray:
    """(a0, b0) of the background field at every particle, layout [a, b] per particle."""
    kp, ks = m.kp, m.ks
    k = kp if wave == 0 else ks
    xi0 = k * math.sin(angle)
    A = 1.0 / (1j * k)
    amp_in = np.array([A, 0.0]) if wave == 0 else np.array([0.0, A])
    R = interface.reflection(xi0, m)
    amp_r = R @ amp_in
    sp = complex(interface.branch_s(xi0, kp))
    ss = complex(interface.branch_s(xi0, ks))
    off = w.offsets()
    out = np.zeros(int(off[-1]), dtype=complex)
    for i in range(w.n):
        pm = int(w.p[i])
        n = np.arange(-pm, pm + 1)
        x0, y0 = w.xy[i]
        a = amp_r[0] * np.exp(1j * xi0 * x0 + sp * y0) * (1j * (xi0 - sp) / kp) ** n
        b = amp_r[1] * np.exp(1j * xi0 * x0 + ss * y0) * (1j * (xi0 - ss) / ks) ** n
        if wave == 0:
            a = a + amp_in[0] * np.exp(1j * xi0 * x0 - sp * y0) * (1j * (xi0 + sp) / kp) ** n
        else:
            b = b + amp_in[1] * np.exp(1j * xi0 * x0 - ss * y0) * (1j * (xi0 + ss) / ks) ** n
        out[off[i]: off[i + 1]] = np.concatenate([a, b])
    return out


def rhs(w, m: Media, S_blocks, wave: int, angle: float) -> np.ndarray:
    """S_m (a0^m, b0^m) for every particle."""
    c = local_coefficients(w, m, wave, angle)
    off = w.offsets()
    out = np.zeros_like(c)
    for i in range(w.n):
        out[off[i]: off[i + 1]] = S_blocks[i] @ c[off[i]: off[i + 1]]
    return out


def background_field(m: Media, wave: int, angle: float, pts: np.ndarray) -> np.ndarray:
    """Displacement of incident + reflected plane waves at host points [n, 2] -> [n, 2]."""
    kp, ks = m.kp, m.ks
    k = kp if wave == 0 else ks
    xi0 = k * math.sin(angle)
    A = 1.0 / (1j * k)
    amp_in = np.array([A, 0.0]) if wave == 0 else np.array([0.0, A])
    amp_r = interface.reflection(xi0, m) @ amp_in
    sp = complex(interface.branch_s(xi0, kp))
    ss = complex(interface.branch_s(xi0, ks))
    x, y = pts[:, 0], pts[:, 1]
    u = np.zeros((len(pts), 2), dtype=complex)
    # grad of e^{i xi x + q y} = (i xi, q) e^{...}; grad^perp = (-q, i xi) e^{...}
    for amp, q in ((amp_in[0], -sp), (amp_r[0], sp)):
        e = amp * np.exp(1j * xi0 * x + q * y)
        u[:, 0] += 1j * xi0 * e
        u[:, 1] += q * e
    for amp, q in ((amp_in[1], -ss), (amp_r[1], ss)):
        e = amp * np.exp(1j * xi0 * x + q * y)
        u[:, 0] += -q * e
        u[:, 1] += 1j * xi0 * e
    return u
