"""Pins of the oracle's misfit gradient (forward-mode tangents).

Each derivative the oracle takes from its definition is checked against a
central difference of the oracle's own undifferentiated function, and the
assembled gradient against central differences of the misfit J itself
(steps 1e-5 to 1e-6: truncation error O(h^2) ~ 1e-11, rounding and
quadrature noise ~ 1e-13 / h).  The dense free and reflected operators it
assembles agree with the oracle's operator applies.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import graf, interface, media, smatrix, sommerfeld
from oracle import gradient as G


def _cloud():
    w = W.small_cloud(3, seed=21, p=3, omega=4.0, width=6.0, depth=(1.0, 3.0), ragged=True)
    m = media.Media.from_workload(w)
    return w, m


@pytest.mark.parametrize("xi", [0.7, 3.1, 5.4, 9.0, 2.0 + 0.3j])
def test_reflection_tangent_matches_differences(xi):
    w, m = _cloud()
    R, dRl, dRm = G.reflection_tangent(xi, m)
    assert np.allclose(R, interface.reflection(xi, m), atol=1e-14)
    h = 1e-6
    for dR, sh in ((dRl, (h, 0.0)), (dRm, (0.0, h))):
        _, mp = G.perturbed(w, m, None, sh)
        _, mm = G.perturbed(w, m, None, (-sh[0], -sh[1]))
        fd = (interface.reflection(xi, mp) - interface.reflection(xi, mm)) / (2 * h)
        assert np.abs(fd - dR).max() <= 1e-7 * max(1.0, np.abs(dR).max())


def test_graf_block_tangent_matches_differences():
    xm, xl = np.array([1.3, -2.0]), np.array([-0.4, -1.1])
    B, Bx, By = G.graf_block_tangent(3.0, xm, xl, 4, 2)
    assert np.allclose(B, graf.translation_block(3.0, xm, xl, 4, 2), atol=1e-14)
    h = 1e-6
    for D, e in ((Bx, np.array([h, 0.0])), (By, np.array([0.0, h]))):
        fd = (graf.translation_block(3.0, xm + e, xl, 4, 2)
              - graf.translation_block(3.0, xm - e, xl, 4, 2)) / (2 * h)
        assert np.abs(fd - D).max() <= 1e-7 * np.abs(D).max()


def test_outgoing_hessian_matches_differences():
    from oracle import field
    dx, dy = np.array([0.9, -1.7, 2.2]), np.array([-0.8, -0.5, 1.9])
    h = 1e-6
    for n in (-3, 0, 2, 5):
        _, fx, fy, fxx, fxy, fyy = G._hess_cyl(n, 2.5, dx, dy)
        gx, gy = field.grad_cyl("H", n, 2.5, dx, dy)
        assert np.allclose(fx, gx, rtol=1e-12) and np.allclose(fy, gy, rtol=1e-12)
        px, py = field.grad_cyl("H", n, 2.5, dx + h, dy)
        mx, my = field.grad_cyl("H", n, 2.5, dx - h, dy)
        assert np.abs((px - mx) / (2 * h) - fxx).max() <= 1e-7 * np.abs(fxx).max()
        assert np.abs((py - my) / (2 * h) - fxy).max() <= 1e-7 * np.abs(fxy).max()
        px, py = field.grad_cyl("H", n, 2.5, dx, dy + h)
        mx, my = field.grad_cyl("H", n, 2.5, dx, dy - h)
        assert np.abs((py - my) / (2 * h) - fyy).max() <= 1e-7 * np.abs(fyy).max()


def test_dense_operators_match_oracle_applies():
    w, m = _cloud()
    x = W.random_coeffs(w.n_coeff, 5)[0]
    Tf, _ = G.free_tangent(w, m)
    Tr, _ = G.refl_tangent(w, m, None, derivs=False)
    assert np.linalg.norm(Tf @ x - graf.apply_free(w, m, x)) <= 1e-13 * np.linalg.norm(Tf @ x)
    yr = sommerfeld.apply_refl(w, m, x)
    assert np.linalg.norm(Tr @ x - yr) <= 1e-12 * np.linalg.norm(yr)


def test_gradient_matches_misfit_differences():
    w, m = _cloud()
    S = smatrix.workload_blocks(w, m)
    pts = np.stack([np.linspace(-1, 7, 6), np.full(6, -0.4)], 1)
    waves = [(0, math.radians(25)), (1, math.radians(-40))]
    rng = np.random.default_rng(3)
    u_obs = (rng.normal(size=(2, 6, 2)) + 1j * rng.normal(size=(2, 6, 2))) * 0.1
    J, gxy, gl = G.gradient(w, m, S, waves, pts, u_obs)
    J2, _, _ = G.misfit(w, m, S, waves, pts, u_obs)
    assert abs(J - J2) <= 1e-12 * J
    h = 1e-5
    for q in range(w.n):
        for c in range(2):
            d = np.zeros((w.n, 2))
            d[q, c] = h
            Jp = G.misfit(*G.perturbed(w, m, d), S, waves, pts, u_obs)[0]
            Jm = G.misfit(*G.perturbed(w, m, -d), S, waves, pts, u_obs)[0]
            assert abs((Jp - Jm) / (2 * h) - gxy[q, c]) <= 1e-7 * np.abs(gxy).max()
    for t in range(2):
        sh = [0.0, 0.0]
        sh[t] = h
        Jp = G.misfit(*G.perturbed(w, m, None, sh), S, waves, pts, u_obs)[0]
        Jm = G.misfit(*G.perturbed(w, m, None, [-v for v in sh]), S, waves, pts, u_obs)[0]
        assert abs((Jp - Jm) / (2 * h) - gl[t]) <= 1e-7 * max(np.abs(gl).max(), 1e-3)
