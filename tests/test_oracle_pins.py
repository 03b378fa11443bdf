"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks one oracle part against something other than itself:
closed forms (Graf addition theorem, the Sommerfeld identity and the Lemma of
Section 5.4, Jacobi-Anger), brute-force boundary conditions evaluated with
Cartesian derivative identities, invariants (reciprocity, energy flux of the
interface, identical media), values the paper prints (Section 7 wavenumbers),
an image-source closed form for the reflected part, and spectral convergence
of the solved field on a particle boundary.  A plausible slip anywhere (a
dropped term, a sign, a transposed index) fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import workloads as W
from oracle import field, gmres, graf, incident, interface, media, operator, smatrix, sommerfeld

HERE = os.path.dirname(__file__)
M0 = media.Media(2.0, 1.0, 1.0, 4.0, 2.0, 1.5, 4.0)


# ---- helpers written independently of the oracle's polar formulas ----------

def cw(kind, n, k, dx, dy):
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    Z = special.hankel1(n, k * r) if kind == "H" else special.jv(n, k * r)
    return Z * np.exp(1j * n * th)


def grad_cw(kind, n, k, dx, dy):
    return (0.5 * k * (cw(kind, n - 1, k, dx, dy) - cw(kind, n + 1, k, dx, dy)),
            0.5j * k * (cw(kind, n - 1, k, dx, dy) + cw(kind, n + 1, k, dx, dy)))


def field_and_jacobian(kind, n, k, wave, dx, dy):
    """u and d_j u_i of grad (wave 0) or grad^perp (wave 1) of Z_n(kr)e^{in th}."""
    gm = grad_cw(kind, n - 1, k, dx, dy)
    gp = grad_cw(kind, n + 1, k, dx, dy)
    gx, gy = grad_cw(kind, n, k, dx, dy)
    hxx = 0.5 * k * (gm[0] - gp[0])
    hxy = 0.5 * k * (gm[1] - gp[1])
    hyy = 0.5j * k * (gm[1] + gp[1])
    if wave == 0:
        return (gx, gy), ((hxx, hxy), (hxy, hyy))
    return (-gy, gx), ((-hxy, -hyy), (hxx, hxy))


def real_axis_integral(f, m, T, tol=1e-13):
    """Integrate a real-vector f over the real axis with the oracle's piece layout."""
    tot = 0.0
    for kind, a, b in sommerfeld._pieces(m, T):
        if kind == 0:
            g, lo, hi = f, a, b
        elif kind == 1:
            g, lo, hi = (lambda a_: (lambda u: f(a_ + u * u) * 2 * u))(a), 0.0, math.sqrt(b - a)
        else:
            g, lo, hi = (lambda b_: (lambda u: f(b_ - u * u) * 2 * u))(b), 0.0, math.sqrt(b - a)
        r, _ = integrate.quad_vec(g, lo, hi, epsabs=1e-16, epsrel=tol, limit=20000)
        tot = tot + r
    return tot


# ---- wavenumbers: values printed in Section 7 ------------------------------

def test_paper_wavenumbers():
    g = json.load(open(os.path.join(HERE, "golden", "paper_wavenumbers.json")))
    for side in ("upper", "lower"):
        kp, ks = media.wavenumbers(g["omega"], g[side]["lam"], g[side]["mu"], 1.0)
        assert abs(kp - g[side]["kp"]) < 1e-13
        assert abs(ks - g[side]["ks"]) < 1e-13


# ---- disk scattering matrices ------------------------------------------------

@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("a", [0.3, 0.5, 0.7])
def test_disk_smatrix_boundary_condition(bc, a):
    """Incident mode + S-predicted scattered field meets the particle BC on 64 points."""
    p = 8
    S = smatrix.disk(M0, a, p, bc)
    N = 2 * p + 1
    th = np.linspace(0, 2 * np.pi, 64, endpoint=False)
    dx, dy = a * np.cos(th), a * np.sin(th)
    lam, mu = M0.lam_h, M0.mu_h
    for col in range(2 * N):
        wave = 0 if col < N else 1
        n = (col if col < N else col - N) - p
        k = M0.kp if wave == 0 else M0.ks
        u, J = field_and_jacobian("J", n, k, wave, dx, dy)
        u = [u[0].copy(), u[1].copy()]
        J = [[J[0][0].copy(), J[0][1].copy()], [J[1][0].copy(), J[1][1].copy()]]
        for row in range(2 * N):
            c = S[row, col]
            if c == 0:
                continue
            ww = 0 if row < N else 1
            nn = (row if row < N else row - N) - p
            us, Js = field_and_jacobian("H", nn, M0.kp if ww == 0 else M0.ks, ww, dx, dy)
            for i in range(2):
                u[i] = u[i] + c * us[i]
                for j in range(2):
                    J[i][j] = J[i][j] + c * Js[i][j]
        if bc == 0:
            assert np.max(np.abs(u[0])) + np.max(np.abs(u[1])) < 1e-13 * k
        else:
            div = J[0][0] + J[1][1]
            sxx = lam * div + 2 * mu * J[0][0]
            syy = lam * div + 2 * mu * J[1][1]
            sxy = mu * (J[0][1] + J[1][0])
            tx = sxx * np.cos(th) + sxy * np.sin(th)
            ty = sxy * np.cos(th) + syy * np.sin(th)
            assert np.max(np.abs(tx)) + np.max(np.abs(ty)) < 1e-13 * (lam + 2 * mu) * k * k


def test_projection_formula_recovers_outgoing_coefficients():
    """Section 4.3 remark: (1/2 pi R) M_H^{-1} [int u.e^{il th} r_hat; int u.e^{il th} th_hat]."""
    rng = np.random.default_rng(4)
    p = 5
    al = rng.standard_normal(2 * p + 1) + 1j * rng.standard_normal(2 * p + 1)
    be = rng.standard_normal(2 * p + 1) + 1j * rng.standard_normal(2 * p + 1)
    R = 0.9
    th = np.linspace(0, 2 * np.pi, 128, endpoint=False)
    dx, dy = R * np.cos(th), R * np.sin(th)
    ux = np.zeros_like(th, dtype=complex)
    uy = np.zeros_like(th, dtype=complex)
    for k_, n in enumerate(range(-p, p + 1)):
        (gx, gy), _ = field_and_jacobian("H", n, M0.kp, 0, dx, dy)
        (hx, hy), _ = field_and_jacobian("H", n, M0.ks, 1, dx, dy)
        ux += al[k_] * gx + be[k_] * hx
        uy += al[k_] * gy + be[k_] * hy
    ur = ux * np.cos(th) + uy * np.sin(th)
    ut = -ux * np.sin(th) + uy * np.cos(th)
    for k_, l in enumerate(range(-p, p + 1)):
        # the projection integrates against e^{-i l th} so that mode l is picked out
        ds = R * (2 * np.pi / len(th))
        proj = np.array([np.sum(ur * np.exp(-1j * l * th)) * ds, np.sum(ut * np.exp(-1j * l * th)) * ds])
        got = np.linalg.solve(smatrix.projection_matrix(M0, R, l), proj) / (2 * np.pi * R)
        assert abs(got[0] - al[k_]) < 1e-12 * (1 + abs(al[k_]))
        assert abs(got[1] - be[k_]) < 1e-12 * (1 + abs(be[k_]))


def test_rotation_composes_and_fixes_disk():
    rng = np.random.default_rng(1)
    p = 4
    S = rng.standard_normal((4 * p + 2, 4 * p + 2)) + 1j * rng.standard_normal((4 * p + 2, 4 * p + 2))
    a, b = 0.7, -1.9
    assert np.allclose(smatrix.rotate(smatrix.rotate(S, p, a), p, b), smatrix.rotate(S, p, a + b), atol=1e-13)
    D = smatrix.disk(M0, 0.5, p, 1)
    assert np.allclose(smatrix.rotate(D, p, 1.234), D, atol=1e-15)


def test_rotation_matches_rotated_field():
    """A field rotated by theta0 about the centre has coefficients c_n e^{-i n theta0}."""
    rng = np.random.default_rng(2)
    p, th0 = 4, 0.83
    c = rng.standard_normal(2 * p + 1) + 1j * rng.standard_normal(2 * p + 1)
    pt = np.array([1.3, -0.4])
    rot = np.array([[math.cos(th0), -math.sin(th0)], [math.sin(th0), math.cos(th0)]])
    q = rot.T @ pt            # field rotated by th0: value at pt = original at R^{-1} pt
    lhs = sum(c[k] * cw("H", n, 2.0, q[0], q[1]) for k, n in enumerate(range(-p, p + 1)))
    c_rot = c * np.exp(-1j * np.arange(-p, p + 1) * th0)
    rhs = sum(c_rot[k] * cw("H", n, 2.0, pt[0], pt[1]) for k, n in enumerate(range(-p, p + 1)))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    # the oracle's rotate() applies exactly these phases on the outgoing side
    S = np.eye(4 * p + 2, dtype=complex)
    assert np.allclose(np.diag(smatrix.rotate(S, p, th0)), 1.0)


# ---- Graf translations -------------------------------------------------------

@pytest.mark.parametrize("k", [2.0, 4.0, 7.5])
def test_graf_identity(k):
    """DLMF 10.23.7: outgoing field of l near m equals the T^{ml} local expansion."""
    rng = np.random.default_rng(0)
    xl = np.array([0.3, -2.0])
    xm = np.array([2.1, -3.3])
    pl, pm = 6, 40
    al = rng.standard_normal(2 * pl + 1) + 1j * rng.standard_normal(2 * pl + 1)
    a = graf.translation_block(k, xm, xl, pm, pl) @ al
    for off in ([0.2, 0.15], [-0.3, 0.1], [0.05, -0.25]):
        pt = xm + np.array(off)
        direct = sum(al[j + pl] * cw("H", j, k, pt[0] - xl[0], pt[1] - xl[1]) for j in range(-pl, pl + 1))
        local = sum(a[i + pm] * cw("J", i, k, pt[0] - xm[0], pt[1] - xm[1]) for i in range(-pm, pm + 1))
        assert abs(direct - local) < 1e-12 * abs(direct)


def test_graf_reciprocity():
    """(T^{lm})^T = P T^{ml} P with P = diag((-1)^n) composed with n -> -n."""
    xm, xl = np.array([1.0, -2.0]), np.array([-0.7, -4.1])
    p = 7
    Tml = graf.translation_block(3.0, xm, xl, p, p)
    Tlm = graf.translation_block(3.0, xl, xm, p, p)
    n = np.arange(-p, p + 1)
    P = np.diag((-1.0) ** n)[::-1]
    assert np.allclose(Tlm.T, P @ Tml @ P, rtol=1e-13, atol=1e-13)


def test_apply_free_matches_blocks():
    w = W.small_cloud(5, seed=2, p=3, ragged=True)
    x = W.random_coeffs(w.n_coeff, 3)[0]
    y = graf.apply_free(w, M0, x)
    off = w.offsets()
    for mm in range(w.n):
        pm = int(w.p[mm])
        acc_a = np.zeros(2 * pm + 1, complex)
        acc_b = np.zeros(2 * pm + 1, complex)
        for ll in range(w.n):
            if ll == mm:
                continue
            pl = int(w.p[ll])
            acc_a += graf.translation_block(M0.kp, w.xy[mm], w.xy[ll], pm, pl) @ x[off[ll]: off[ll] + 2 * pl + 1]
            acc_b += graf.translation_block(M0.ks, w.xy[mm], w.xy[ll], pm, pl) @ x[off[ll] + 2 * pl + 1: off[ll + 1]]
        assert np.allclose(y[off[mm]: off[mm + 1]], np.concatenate([acc_a, acc_b]), rtol=1e-13, atol=1e-12)


# ---- Sommerfeld primitives ---------------------------------------------------

def test_sommerfeld_identity_h0():
    """(i/4) H0(k|x - x0|) = (1/4 pi) int e^{-s |y - y0|} / s e^{i xi (x - x0)} dxi."""
    k = 2.0
    for X, Y in ((0.7, 1.9), (-2.3, 0.8), (4.0, 2.5)):
        def f(xi):
            s = complex(interface.branch_s(xi, k))
            v = np.exp(-s * abs(Y) + 1j * xi * X) / s / (4 * math.pi)
            return np.array([v.real, v.imag])
        r = real_axis_integral(f, M0, 40.0)
        ex = 0.25j * special.hankel1(0, k * math.hypot(X, Y))
        assert abs(r[0] + 1j * r[1] - ex) < 1e-12 * abs(ex)


@pytest.mark.parametrize("n", [-7, -2, 0, 1, 5, 9])
def test_multipole_to_sommerfeld_lemma(n):
    """Section 5.4 Lemma with the oracle's (-i zeta)^n form, for y > y_m."""
    k = M0.ks
    X, Y = 1.1, 1.6
    def f(xi):
        s = complex(interface.branch_s(xi, k))
        z = (xi - s) / k
        v = np.exp(-s * Y + 1j * xi * X) / s * (-1j * z) ** n / (1j * math.pi)
        return np.array([v.real, v.imag])
    r = real_axis_integral(f, M0, 60.0)
    ex = cw("H", n, k, X, Y)
    assert abs(r[0] + 1j * r[1] - ex) < 1e-11 * abs(ex)


@pytest.mark.parametrize("xi", [0.3, -1.7, 3.9, 6.5, -9.0])
def test_jacobi_anger_local_expansion(xi):
    """Section 5.3: e^{i xi x + s y} = e^{i xi x_l + s y_l} sum (i zeta)^n J_n e^{i n th}."""
    k = 4.0
    s = complex(interface.branch_s(xi, k))
    z = (xi - s) / k
    c = np.array([0.4, -2.0])
    pt = c + np.array([0.3, -0.2])
    lhs = np.exp(1j * xi * pt[0] + s * pt[1])
    rhs = np.exp(1j * xi * c[0] + s * c[1]) * sum(
        (1j * z) ** n * cw("J", n, k, pt[0] - c[0], pt[1] - c[1]) for n in range(-60, 61))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ---- interface reflection --------------------------------------------------

def test_plane_wave_columns_by_finite_differences():
    """Displacement and traction columns of potentials, checked by Cartesian FD."""
    lam, mu = 2.0, 1.0
    xi, q = 0.8, 1.3 - 0.4j
    h = 1e-5
    for wave in (0, 1):
        def phi(x, y):
            return np.exp(1j * xi * x + q * y)
        def u(x, y):
            dx = (phi(x + h, y) - phi(x - h, y)) / (2 * h)
            dy = (phi(x, y + h) - phi(x, y - h)) / (2 * h)
            return np.array([dx, dy]) if wave == 0 else np.array([-dy, dx])
        hh = 1e-3
        ux = (u(hh, 0) - u(-hh, 0)) / (2 * hh)
        uy = (u(0, hh) - u(0, -hh)) / (2 * hh)
        t1 = mu * (uy[0] + ux[1])
        t2 = (lam + 2 * mu) * uy[1] + lam * ux[0]
        P, S = interface._cols(xi, q, lam, mu)
        col = P if wave == 0 else S
        assert np.allclose(col, np.array([*u(0, 0), t1, t2]), rtol=1e-5, atol=1e-5)


def test_reflection_identical_media_vanishes():
    mi = media.Media(2.0, 1.0, 1.0, 2.0, 1.0, 1.0, 4.0)
    for xi in (0.0, 0.7, 1.99, 3.5, -6.0, 25.0):
        R, T = interface.reflect_transmit(xi, mi)
        assert np.max(np.abs(R)) < 1e-13
        assert np.allclose(T, np.eye(2), atol=1e-13)


@pytest.mark.parametrize("xi", [0.0, 0.4, -0.9, 1.2, 1.6])
def test_reflection_conserves_energy_flux(xi):
    """Propagating |xi| below every wavenumber: rho |A|^2 Re k_y summed out = in.

    For a potential plane wave of amplitude A the time-averaged vertical energy
    flux is (omega^3 / 2) rho |A|^2 k_y for both P and S (|u| = k |A|).
    """
    m = M0
    assert abs(xi) < min(m.kp, m.ks, m.kpb, m.ksb)
    R, T = interface.reflect_transmit(xi, m)
    ky = lambda k: math.sqrt(k * k - xi * xi)  # noqa: E731
    for inc in (0, 1):
        flux_in = m.rho_h * ky(m.kp if inc == 0 else m.ks)
        out = (m.rho_h * (abs(R[0, inc]) ** 2 * ky(m.kp) + abs(R[1, inc]) ** 2 * ky(m.ks))
               + m.rho_b * (abs(T[0, inc]) ** 2 * ky(m.kpb) + abs(T[1, inc]) ** 2 * ky(m.ksb)))
        assert abs(out - flux_in) < 1e-12 * flux_in


def test_reflection_free_surface_limit_rayleigh_pole():
    """Substrate -> vacuum: |R| blows up at the Rayleigh number, root of
    (2 xi^2 - ks^2)^2 - 4 xi^2 sqrt(xi^2 - kp^2) sqrt(xi^2 - ks^2) (textbook)."""
    from scipy.optimize import brentq
    kp, ks = M0.kp, M0.ks
    ray = lambda x: (2 * x * x - ks * ks) ** 2 - 4 * x * x * math.sqrt(x * x - kp * kp) * math.sqrt(x * x - ks * ks)  # noqa: E731
    xr = brentq(ray, ks * 1.0001, ks * 1.5)
    mv = media.Media(2.0, 1.0, 1.0, 2e-9, 1e-9, 1e-9, 4.0)
    near = np.max(np.abs(interface.reflection(xr * (1 + 1e-7), mv)))
    away = np.max(np.abs(interface.reflection(xr * 1.1, mv)))
    assert near > 1e4 * away
    # and at normal incidence a free surface reflects a P potential with |R_pp| = 1
    R = interface.reflection(0.0, mv)
    assert abs(abs(R[0, 0]) - 1.0) < 1e-6 and abs(R[1, 0]) < 1e-6


# ---- reflected operator: image-source closed form ------------------------------

def test_reflected_part_image_source():
    """R = diag(rp, rs): T_refl equals Graf from mirror sources (x_m, -y_m)
    with coefficients (-1)^j c_{-j}, self pair included (Lemma with y -> -y)."""
    w = W.small_cloud(4, seed=3, p=5, omega=4.0, width=8.0, depth=(1.0, 4.0), ragged=True)
    rp, rs = 0.7 - 0.2j, -0.4 + 0.5j
    x = W.random_coeffs(w.n_coeff, 11)[0]
    yr = sommerfeld.apply_refl(w, M0, x, R_fun=lambda xi: np.array([[rp, 0], [0, rs]]), tol=1e-14)
    off = w.offsets()
    yi = np.zeros_like(x)
    for l in range(w.n):
        pl = int(w.p[l])
        Nl = 2 * pl + 1
        for mm in range(w.n):
            pm = int(w.p[mm])
            N = 2 * pm + 1
            j = np.arange(-pm, pm + 1)
            als = ((-1.0) ** j) * x[off[mm]: off[mm] + N][::-1]
            bes = ((-1.0) ** j) * x[off[mm] + N: off[mm + 1]][::-1]
            src = np.array([w.xy[mm, 0], -w.xy[mm, 1]])
            yi[off[l]: off[l] + Nl] += rp * graf.translation_block(M0.kp, w.xy[l], src, pl, pm) @ als
            yi[off[l] + Nl: off[l + 1]] += rs * graf.translation_block(M0.ks, w.xy[l], src, pl, pm) @ bes
    assert np.linalg.norm(yr - yi) < 1e-12 * np.linalg.norm(yi)


# ---- right-hand side ------------------------------------------------------------

@pytest.mark.parametrize("wave", [0, 1])
def test_incident_local_expansion_reproduces_background(wave):
    m = M0
    w = W.small_cloud(2, seed=4, p=18)
    ang = math.radians(35.0)
    c = incident.local_coefficients(w, m, wave, ang)
    off = w.offsets()
    th = np.linspace(0, 2 * np.pi, 9, endpoint=False)
    for i in range(w.n):
        pts = w.xy[i] + 0.3 * np.stack([np.cos(th), np.sin(th)], 1)
        ub = incident.background_field(m, wave, ang, pts)
        p = int(w.p[i])
        N = 2 * p + 1
        u = np.zeros_like(ub)
        dx, dy = pts[:, 0] - w.xy[i, 0], pts[:, 1] - w.xy[i, 1]
        for k_, n in enumerate(range(-p, p + 1)):
            (gx, gy), _ = field_and_jacobian("J", n, m.kp, 0, dx, dy)
            (hx, hy), _ = field_and_jacobian("J", n, m.ks, 1, dx, dy)
            u[:, 0] += c[off[i] + k_] * gx + c[off[i] + N + k_] * hx
            u[:, 1] += c[off[i] + k_] * gy + c[off[i] + N + k_] * hy
        assert np.max(np.abs(u - ub)) < 1e-12


def test_plane_wave_is_unit_displacement():
    m = M0
    ang = math.radians(30.0)
    d = np.array([math.sin(ang), math.cos(ang)])
    mi = media.Media(2.0, 1.0, 1.0, 2.0, 1.0, 1.0, 4.0)   # no reflection
    pts = np.array([[0.3, -1.0], [2.0, -0.4]])
    up = incident.background_field(mi, 0, ang, pts)
    us = incident.background_field(mi, 1, ang, pts)
    for q, x in enumerate(pts):
        assert np.allclose(up[q], d * np.exp(1j * m.kp * d @ x), atol=1e-14)
        assert np.allclose(us[q], np.array([-d[1], d[0]]) * np.exp(1j * m.ks * d @ x), atol=1e-14)


# ---- GMRES ---------------------------------------------------------------------

def test_gmres_matches_dense_solve():
    rng = np.random.default_rng(7)
    n = 60
    A = np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / math.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = gmres.gmres(lambda v: A @ v, b, tol=1e-13, maxit=n)
    assert info["relres"] <= 1e-13
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-11 * np.linalg.norm(x)


def test_operator_gmres_vs_dense_lu_tiny():
    """N = 2 particles: GMRES on the operator equals LU of the assembled matrix."""
    w = W.small_cloud(2, seed=9, p=2, omega=3.0, width=5.0, depth=(1.0, 2.5))
    m = media.Media.from_workload(w)
    S = smatrix.workload_blocks(w, m)
    A = operator.dense_matrix(w, m, S, tol=1e-13)
    b = incident.rhs(w, m, S, 0, math.radians(30.0))
    x, info = gmres.gmres(lambda v: operator.apply(w, m, S, v, tol=1e-13), b, tol=1e-13, maxit=40)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)


# ---- whole chain: the solved field meets the particle boundary condition -------------

@pytest.mark.slow
def test_solved_field_spectral_convergence_rigid():
    """Three rigid disks, SV incidence: the boundary residual of the total field
    (background + all outgoing fields + reflected field) decays spectrally in p."""
    res = []
    for p in (4, 8, 12):
        w = W.small_cloud(3, seed=5, p=p, omega=2.0, width=6.0, depth=(1.0, 3.0))
        w.radius[:] = 0.4
        w.a[:] = 0.4
        w.bc[:] = 0
        m = media.Media.from_workload(w)
        S = smatrix.workload_blocks(w, m)
        ang = math.radians(20.0)
        b = incident.rhs(w, m, S, 1, ang)
        x, _ = gmres.gmres(lambda v: operator.apply(w, m, S, v, tol=1e-13), b, tol=1e-13, maxit=100)
        th = np.linspace(0, 2 * np.pi, 16, endpoint=False)
        r = 0.0
        for q in range(w.n):
            pts = w.xy[q] + 0.4 * np.stack([np.cos(th), np.sin(th)], 1)
            u = incident.background_field(m, 1, ang, pts) + field.scattered(w, m, x, pts, tol=1e-13)
            r = max(r, float(np.abs(u).max()))
        res.append(r)
    assert res[0] > 30 * res[1] > 900 * res[2]
    assert res[2] < 1e-6
