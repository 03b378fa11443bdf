"""Pins of the oracle's scattering matrices of non-circular particles
(Section 4.3; method of fundamental solutions, see oracle/shapes.py), on the
CPU:

* circles reproduce the closed-form S of the disk (mode-by-mode boundary
  conditions, a different construction);
* energy: for a rigid or traction-free (lossless) particle, I + 2S is unitary
  (an incident regular wave is half incoming, half outgoing; the flux of every
  potential mode is the same per |amplitude|^2);
* the boundary condition holds between the collocation points;
* a turned particle's S is the basis rotation of the unturned one (Section 4.3,
  rotated copies);
* the discretisation has converged at the paper-like 256 points.
"""
import math

import numpy as np
import pytest

from oracle import media, shapes, smatrix

M0 = media.Media(2.0, 1.0, 1.0, 4.0, 2.0, 1.5, 8.0)   # omega = 8: kp = 4, ks = 8
P = 15


@pytest.mark.parametrize("bc,a", [(0, 0.6), (1, 0.6), (0, 0.3), (1, 0.45)])
def test_circle_matches_closed_form(bc, a):
    S = shapes.smatrix(M0, 0, a, P, bc, npts=160)
    Sd = smatrix.disk(M0, a, P, bc)
    e = np.abs(S - Sd).max() / np.abs(Sd).max()
    print("circle", bc, a, e)
    assert e < (1e-12 if bc == 0 else 1e-8)


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", [0, 1])
def test_unitarity_residual_and_convergence(kind, bc):
    S, res = shapes.smatrix(M0, kind, 0.6, P, bc, residual=True)
    U = np.eye(len(S)) + 2 * S
    eu = np.abs(U.conj().T @ U - np.eye(len(S))).max()
    S2 = shapes.smatrix(M0, kind, 0.6, P, bc, npts=320)
    ec = np.abs(S - S2).max() / np.abs(S2).max()
    print("shape", kind, bc, "unitarity", eu, "midpoint residual", res, "256 vs 320", ec)
    assert eu < 1e-8 and ec < 1e-8 and res < 1e-4


@pytest.mark.parametrize("kind,bc", [(1, 0), (2, 1), (3, 1), (4, 0)])
def test_turned_particle_is_basis_rotation(kind, bc):
    th = 0.7
    S0 = shapes.smatrix(M0, kind, 0.5, P, bc)
    St = shapes.smatrix(M0, kind, 0.5, P, bc, theta0=th)
    e = np.abs(St - smatrix.rotate(S0, P, th)).max() / np.abs(St).max()
    print("rotation", kind, bc, e)
    assert e < 1e-8
