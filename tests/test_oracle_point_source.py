"""Pins of the oracle's point-source incidence (Section 3.2), on the CPU.

* The 4x4 system assembled from the definitions of the three Sommerfeld
  fields equals the paper's printed A_xi (aa) and b_xi at rho = 1, up to the
  row scale 1/(4 pi omega^2) — with one entry of (aa) moved: the second row
  as printed puts the sigma_22 coefficient in the sigma_21 column, but
  continuity of u_2 has no sigma_21 term (its two contributions cancel), so
  the entry belongs to the sigma_22 column (reading recorded with the design
  notes).
* The Sommerfeld form of the incident field (the same spectral term the
  system uses) integrates to the closed-form Green's tensor with Hankel
  functions.
* The Green's tensor carries a unit point force: the traction on a small
  circle around the source sums to -alpha (this fixes its normalisation,
  density included).
* The total field is continuous across the interface: displacement and
  traction of u_inc + u1 above and u2 below agree at y = 0 (finite
  differences, extrapolated to y = 0 from each side).
* The local coefficients reproduce u2 near a particle through the regular
  wave expansion sum a_n grad(J_n e^{i n th}) + b_n grad^perp(J_n e^{i n th}).
"""
import math

import numpy as np
import pytest
from scipy import special

import workloads as W
from oracle import interface, media, point_source, sommerfeld
from tests.helpers import at_interface

M0 = media.Media(2.0, 1.0, 1.0, 4.0, 2.0, 1.5, 4.0)
ALPHA = np.array([math.cos(math.pi / 4), math.sin(math.pi / 4)])   # the paper's polarisation


def _printed_aa_b(xi, m, y0, alpha):
    """(aa) and b_xi as printed, paper notation: unprimed = upper layer (here
    the substrate), primed = lower layer (the host); rho = 1."""
    lam, mu, lam2, mu2 = m.lam_b, m.mu_b, m.lam_h, m.mu_h
    kp, ks, kp2, ks2 = m.kpb, m.ksb, m.kp, m.ks
    sv = interface.s_values(xi, m)
    lp2, ls2, lp, ls = sv
    I = 1j
    A = np.array([
        [ks**2 / ls - xi**2 / ls + xi**2 / lp, 0, xi**2 / ls2 - ks2**2 / ls2 - xi**2 / lp2, 0],
        [0, ks**2 / ls + ls - lp, 0, lp2 - ks2**2 / ls2 - ls2],
        [-mu * ks**2, I * mu * xi * (ks**2 / ls + 2 * ls - 2 * lp), -mu2 * ks2**2,
         I * mu2 * xi * (2 * lp2 - 2 * ls2 - ks2**2 / ls2)],
        [I * xi * (2 * mu * (ls - lp) + lam * kp**2 / lp), -(lam + 2 * mu) * kp**2,
         I * xi * (2 * mu2 * (lp2 - ls2) - lam2 * kp2**2 / lp2), -(lam2 + 2 * mu2) * kp2**2]])
    es, ep = np.exp(-ls * y0), np.exp(-lp * y0)
    a1, a2 = alpha
    b = -np.array([
        (-ls * es + xi**2 * ep / lp) * a1 + I * xi * (es - ep) * a2,
        I * xi * (es - ep) * a1 + (xi**2 * es / ls - ep * lp) * a2,
        mu * (ks**2 * es - 2 * xi**2 * es + 2 * xi**2 * ep) * a1
        + I * mu * xi * (ks**2 * es / ls + 2 * es * ls - 2 * ep * lp) * a2,
        I * xi * (2 * mu * (ls * es - lp * ep) + lam * kp**2 * ep / lp) * a1
        + (2 * mu * xi**2 * (es - ep) + (lam + 2 * mu) * kp**2 * ep) * a2])
    return A, b


@pytest.mark.parametrize("xi", [0.3, -1.7, 2.9, 4.6, -9.0])
def test_system_matches_printed_aa_and_b(xi):
    m = media.Media(2.0, 1.0, 1.0, 4.0, 2.0, 1.0, 4.0)  # rho = 1 in both layers
    y0 = 1.3
    A, b = point_source.system(xi, m, y0, ALPHA)
    Ap, bp = _printed_aa_b(xi, m, y0, ALPHA)
    sc = 4 * math.pi * m.omega ** 2
    assert np.abs(A * sc - Ap).max() < 1e-12 * np.abs(Ap).max()
    assert np.abs(b * sc - bp).max() < 1e-12 * np.abs(bp).max()


def test_sommerfeld_form_of_incident_field_is_greens_tensor():
    m = M0
    x0 = np.array([0.4, 2.0])
    pts = np.array([[0.0, 1.2], [1.5, 0.4], [-2.0, 0.9]])    # below the source
    alpha = np.array([0.3, -0.8])

    def f(xi, bp=None, d=None):
        sv = interface.s_values(xi, m, bp, d)
        spb, ssb = sv[2], sv[3]
        out = []
        for x, y in pts:
            u, _ = point_source._term(xi, {"p": spb, "s": ssb}, k_s=m.ksb, rho=m.rho_b,
                                      lam=m.lam_b, mu=m.mu_b, omega=m.omega, c=alpha.astype(complex),
                                      G={"p": np.exp(-spb * (x0[1] - y)) / (4 * math.pi * spb),
                                         "s": np.exp(-ssb * (x0[1] - y)) / (4 * math.pi * ssb)})
            out.append(u * np.exp(1j * xi * (x - x0[0])))
        v = np.concatenate(out)
        return np.concatenate([v.real, v.imag])

    # adaptive Gauss-Kronrod on the real axis with xi = k +- u^2 next to each
    # branch point (the oracle's own integration primitive)
    v, _, _ = sommerfeld._integrate(f, 6, sommerfeld._pieces(m, 60.0), 1e-13, 200000)
    total = np.concatenate([v.real, v.imag])
    got = (total[:6] + 1j * total[6:]).reshape(3, 2)
    want = point_source.greens_tensor(m, x0, pts) @ alpha
    assert np.abs(got - want).max() < 1e-8 * np.abs(want).max()


def test_greens_tensor_carries_unit_point_force():
    m = M0
    x0 = np.array([0.0, 3.0])
    alpha = np.array([0.6, -0.8])
    r, h = 2e-3, 1e-6
    th = np.linspace(0, 2 * np.pi, 400, endpoint=False)
    n = np.stack([np.cos(th), np.sin(th)], 1)
    P = x0 + r * n
    u = lambda Q: point_source.greens_tensor(m, x0, Q) @ alpha  # noqa: E731
    ux = (u(P + [h, 0]) - u(P - [h, 0])) / (2 * h)
    uy = (u(P + [0, h]) - u(P - [0, h])) / (2 * h)
    div = ux[:, 0] + uy[:, 1]
    s11 = m.lam_b * div + 2 * m.mu_b * ux[:, 0]
    s22 = m.lam_b * div + 2 * m.mu_b * uy[:, 1]
    s12 = m.mu_b * (uy[:, 0] + ux[:, 1])
    t = np.stack([s11 * n[:, 0] + s12 * n[:, 1], s12 * n[:, 0] + s22 * n[:, 1]], 1)
    force = t.sum(0) * r * (2 * np.pi / len(th))
    assert np.abs(force + alpha).max() < 1e-3


def test_total_field_continuous_across_interface():
    m = M0
    x0 = np.array([0.5, 1.5])
    x = np.linspace(-2.0, 3.0, 5)
    up = lambda X, Y: point_source.upper_field(m, x0, ALPHA, np.stack([X, Y], 1))  # noqa: E731
    dn = lambda X, Y: point_source.transmitted_field(m, x0, ALPHA, np.stack([X, Y], 1))  # noqa: E731
    u_h, t_h = at_interface(dn, x, -1, m.lam_h, m.mu_h)
    u_b, t_b = at_interface(up, x, +1, m.lam_b, m.mu_b)
    eu = np.abs(u_h - u_b).max() / np.abs(u_h).max()
    et = np.abs(t_h - t_b).max() / np.abs(t_h).max()
    print("point-source continuity", eu, et)
    assert eu < 1e-7 and et < 1e-6


def test_local_coefficients_reproduce_transmitted_field():
    w = W.small_cloud(3, seed=8, p=12, omega=4.0, width=6.0, depth=(1.0, 3.0))
    m = media.Media.from_workload(w)
    x0 = np.array([2.0, 1.2])
    c = point_source.local_coefficients(w, m, x0, ALPHA)
    off = w.offsets()
    for i in range(w.n):
        pm = int(w.p[i])
        a = c[off[i]: off[i] + 2 * pm + 1]
        b = c[off[i] + 2 * pm + 1: off[i + 1]]
        th = np.linspace(0, 2 * np.pi, 24, endpoint=False)
        rr = 0.3
        dx, dy = rr * np.cos(th), rr * np.sin(th)
        pts = w.xy[i] + np.stack([dx, dy], 1)
        u = np.zeros((len(th), 2), dtype=complex)
        r = np.hypot(dx, dy)
        ang = np.arctan2(dy, dx)
        for k_, nn in enumerate(range(-pm, pm + 1)):
            for kind, kk, coef in ((0, m.kp, a[k_]), (1, m.ks, b[k_])):
                # grad of J_n(k r) e^{i n th}: d_x = (k/2)(v_{n-1} - v_{n+1}), d_y = (i k/2)(v_{n-1} + v_{n+1})
                vm = special.jv(nn - 1, kk * r) * np.exp(1j * (nn - 1) * ang)
                vp = special.jv(nn + 1, kk * r) * np.exp(1j * (nn + 1) * ang)
                gx, gy = 0.5 * kk * (vm - vp), 0.5j * kk * (vm + vp)
                if kind == 0:
                    u[:, 0] += coef * gx
                    u[:, 1] += coef * gy
                else:
                    u[:, 0] += -coef * gy
                    u[:, 1] += coef * gx
        ref = point_source.transmitted_field(m, x0, ALPHA, pts)
        e = np.abs(u - ref).max() / np.abs(ref).max()
        print("particle", i, "local expansion vs field", e)
        assert e < 1e-9
