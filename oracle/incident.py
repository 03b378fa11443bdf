"""Plane-wave right-hand side (Section 7.3 and the preconditioned system of Section 4.2).

The background field in the host is the incident plane wave plus its
interface reflection (Section 2: total = background + scattered; Section 7.3:
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

Waves sent from the substrate (Section 7.3's own setup, (bplan)): direction
(sin th, -cos th), unit displacement, potential A e^{i xi0 x + s_b y} with A =
1/(i k_b), xi0 = k_b sin th; the host sees the transmitted potentials Td A
(``interface.from_substrate``), the substrate the incident and reflected ones.
"""
from __future__ import annotations

import math

import numpy as np

from . import interface
from .media import Media


def _waves(m: Media, wave: int, angle: float):
    """(xi0, [(layer, kind, A, q)]) of the background field of one plane wave:
    potentials A e^{i xi0 x + q y}, layer 0 host (y < 0) / 1 substrate, kind 0
    P (grad) / 1 S (grad^perp).  Waves 0, 1 come from the host side (Section
    7.3 reading: towards the interface, direction (sin th, cos th)); waves 2,
    3 from the substrate (direction (sin th, -cos th)) and reach the
    particles transmitted."""
    k = (m.kp, m.ks, m.kpb, m.ksb)[wave]
    xi0 = k * math.sin(angle)
    A = 1.0 / (1j * k)
    sp, ss, spb, ssb = (complex(interface.branch_s(xi0, kk)) for kk in (m.kp, m.ks, m.kpb, m.ksb))
    if wave < 2:
        c = wave
        R, T = interface.reflect_transmit(xi0, m)
        return xi0, [(0, c, A, -(sp, ss)[c]),
                     (0, 0, R[0, c] * A, sp), (0, 1, R[1, c] * A, ss),
                     (1, 0, T[0, c] * A, -spb), (1, 1, T[1, c] * A, -ssb)]
    c = wave - 2
    Td, Rb = interface.from_substrate(xi0, m)
    return xi0, [(1, c, A, (spb, ssb)[c]),
                 (1, 0, Rb[0, c] * A, -spb), (1, 1, Rb[1, c] * A, -ssb),
                 (0, 0, Td[0, c] * A, sp), (0, 1, Td[1, c] * A, ss)]


def local_coefficients(w, m: Media, wave: int, angle: float) -> np.ndarray:
    """(a0, b0) of the background field at every particle, layout [a, b] per particle."""
    kp, ks = m.kp, m.ks
    xi0, parts = _waves(m, wave, angle)
    off = w.offsets()
    out = np.zeros(int(off[-1]), dtype=complex)
    for i in range(w.n):
        pm = int(w.p[i])
        n = np.arange(-pm, pm + 1)
        x0, y0 = w.xy[i]
        ab = [np.zeros(2 * pm + 1, complex), np.zeros(2 * pm + 1, complex)]
        for layer, kind, A, q in parts:
            if layer != 0:
                continue
            k = (kp, ks)[kind]
            # e^{i xi x + q y} about (x0, y0): e^{i xi x0 + q y0} (i (xi - q)/k)^n
            ab[kind] = ab[kind] + A * np.exp(1j * xi0 * x0 + q * y0) * (1j * (xi0 - q) / k) ** n
        out[off[i]: off[i + 1]] = np.concatenate(ab)
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
    """Background displacement at points [n, 2] of either layer -> [n, 2]."""
    xi0, parts = _waves(m, wave, angle)
    x, y = pts[:, 0], pts[:, 1]
    layer_of = np.where(y < 0, 0, 1)
    u = np.zeros((len(pts), 2), dtype=complex)
    # grad of e^{i xi x + q y} = (i xi, q) e^{...}; grad^perp = (-q, i xi) e^{...}
    for layer, kind, A, q in parts:
        e = np.where(layer_of == layer, A * np.exp(1j * xi0 * x + q * y), 0.0)
        if kind == 0:
            u[:, 0] += 1j * xi0 * e
            u[:, 1] += q * e
        else:
            u[:, 0] += -q * e
            u[:, 1] += 1j * xi0 * e
    return u
