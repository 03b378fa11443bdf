"""Pins of the oracle's waves sent from the substrate (Section 7.3's plane-wave
setup, (bplan)) and of its transmitted field, checked on the CPU against what
the physics fixes independently of the oracle's formulas:

* identical layers: nothing is reflected and everything is transmitted;
* energy flux: for propagating waves the vertical flux of the incident wave
  equals the reflected plus transmitted fluxes;
* continuity: displacement and traction T_y u = (mu (d_y u1 + d_x u2),
  (lambda + 2 mu) d_y u2 + lambda d_x u1) of the background field, and of the
  scattered field of a small cloud (direct + reflected below, transmitted
  above), agree across y = 0.  Derivatives are central differences of the
  displacement and both sides are extrapolated to y = 0 from inside their
  layer, so the check never uses the oracle's potential-to-traction columns;
* the incident component is the unit-displacement wave d e^{i k d.x} of the
  stated direction.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import field, incident, interface, media
from tests.helpers import at_interface as _at_interface

M0 = media.Media(2.0, 1.0, 1.0, 4.0, 2.0, 1.5, 4.0)


def test_identical_layers_transmit_everything():
    m = media.Media(2.0, 1.0, 1.0, 2.0, 1.0, 1.0, 4.0)
    for xi in (0.3, 1.7, 2.5, 5.0):
        Td, Rb = interface.from_substrate(xi, m)
        assert np.abs(Rb).max() < 1e-13 and np.abs(Td - np.eye(2)).max() < 1e-13
        R, T = interface.reflect_transmit(xi, m)
        assert np.abs(R).max() < 1e-13 and np.abs(T - np.eye(2)).max() < 1e-13


@pytest.mark.parametrize("xi", [0.0, 0.4, -1.1, 1.6])
def test_substrate_incidence_conserves_energy_flux(xi):
    """rho |A|^2 k_y (the vertical flux of a potential plane wave up to
    omega^3 / 2) of the incident wave = reflected + transmitted."""
    m = M0
    assert abs(xi) < min(m.kp, m.ks, m.kpb, m.ksb)
    Td, Rb = interface.from_substrate(xi, m)
    ky = lambda k: math.sqrt(k * k - xi * xi)  # noqa: E731
    for inc in (0, 1):
        flux_in = m.rho_b * ky(m.kpb if inc == 0 else m.ksb)
        out = (m.rho_b * (abs(Rb[0, inc]) ** 2 * ky(m.kpb) + abs(Rb[1, inc]) ** 2 * ky(m.ksb))
               + m.rho_h * (abs(Td[0, inc]) ** 2 * ky(m.kp) + abs(Td[1, inc]) ** 2 * ky(m.ks)))
        assert abs(out - flux_in) < 1e-12 * flux_in


@pytest.mark.parametrize("wave,angle", [(0, 0.3), (1, -0.6), (2, 0.2), (2, 1.2), (3, 0.5),
                                        (3, -1.3)])
def test_background_field_continuous_across_interface(wave, angle):
    m = M0
    x = np.linspace(-3.0, 4.0, 9)
    uf = lambda X, Y: incident.background_field(m, wave, angle, np.stack([X, Y], 1))  # noqa: E731
    u_h, t_h = _at_interface(uf, x, -1, m.lam_h, m.mu_h)
    u_b, t_b = _at_interface(uf, x, +1, m.lam_b, m.mu_b)
    su, st = np.abs(u_h).max(), np.abs(t_h).max()
    assert np.abs(u_h - u_b).max() < 1e-8 * su
    assert np.abs(t_h - t_b).max() < 1e-7 * st


@pytest.mark.parametrize("wave,angle", [(0, 0.4), (1, -0.2), (2, 0.7), (3, -0.9)])
def test_incident_component_is_unit_plane_wave(wave, angle):
    m = M0
    xi0, parts = incident._waves(m, wave, angle)
    layer, kind, A, q = parts[0]
    k = (m.kp, m.ks, m.kpb, m.ksb)[wave]
    d = np.array([math.sin(angle), math.cos(angle) if wave < 2 else -math.cos(angle)])
    X = np.array([0.7, -1.3]) if wave < 2 else np.array([0.7, 1.3])
    e = A * np.exp(1j * xi0 * X[0] + q * X[1])
    u = np.array([1j * xi0 * e, q * e]) if kind == 0 else np.array([-q * e, 1j * xi0 * e])
    want_dir = d if kind == 0 else np.array([-d[1], d[0]])
    assert np.allclose(u, want_dir * np.exp(1j * k * d @ X), atol=1e-14)


def test_scattered_field_continuous_across_interface():
    """Direct + reflected below, transmitted above: the scattered field of a
    small cloud with random coefficients satisfies both continuity
    conditions at y = 0."""
    m = M0
    w = W.small_cloud(3, seed=4, p=3, omega=4.0, width=6.0, depth=(1.0, 2.5))
    mw = media.Media.from_workload(w)
    rng = np.random.default_rng(5)
    g = rng.standard_normal(w.n_coeff) + 1j * rng.standard_normal(w.n_coeff)
    x = np.linspace(-1.0, 7.0, 5)
    uf = lambda X, Y: field.scattered(w, mw, g, np.stack([X, Y], 1), tol=1e-13)  # noqa: E731
    u_h, t_h = _at_interface(uf, x, -1, mw.lam_h, mw.mu_h)
    u_b, t_b = _at_interface(uf, x, +1, mw.lam_b, mw.mu_b)
    su, st = np.abs(u_h).max(), np.abs(t_h).max()
    print("scattered continuity", np.abs(u_h - u_b).max() / su, np.abs(t_h - t_b).max() / st)
    assert np.abs(u_h - u_b).max() < 1e-7 * su
    assert np.abs(t_h - t_b).max() < 1e-6 * st
    del m
