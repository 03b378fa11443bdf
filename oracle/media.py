"""Material constants and wavenumbers.

Section 2: Navier equation with Lame parameters and density; the Helmholtz
split gives compressional and shear numbers kp = omega / sqrt(lambda + 2 mu)
and ks = omega / sqrt(mu) when rho = 1.  The paper normalises rho to one; the
oracle keeps rho, so kp = omega sqrt(rho / (lambda + 2 mu)),
ks = omega sqrt(rho / mu).
"""
from __future__ import annotations

import dataclasses
import math


@dataclasses.dataclass(frozen=True)
class Media:
    """Host = half-space y < 0 holding the particles; substrate = y > 0."""

    lam_h: float
    mu_h: float
    rho_h: float
    lam_b: float
    mu_b: float
    rho_b: float
    omega: float

    @property
    def kp(self) -> float:
        return wavenumbers(self.omega, self.lam_h, self.mu_h, self.rho_h)[0]

    @property
    def ks(self) -> float:
        return wavenumbers(self.omega, self.lam_h, self.mu_h, self.rho_h)[1]

    @property
    def kpb(self) -> float:
        return wavenumbers(self.omega, self.lam_b, self.mu_b, self.rho_b)[0]

    @property
    def ksb(self) -> float:
        return wavenumbers(self.omega, self.lam_b, self.mu_b, self.rho_b)[1]

    @staticmethod
    def from_workload(w) -> "Media":
        return Media(w.host.lam, w.host.mu, w.host.rho,
                     w.substrate.lam, w.substrate.mu, w.substrate.rho, w.omega)


def wavenumbers(omega: float, lam: float, mu: float, rho: float = 1.0):
    """(kp, ks) of a homogeneous isotropic medium."""
    return omega * math.sqrt(rho / (lam + 2.0 * mu)), omega * math.sqrt(rho / mu)
