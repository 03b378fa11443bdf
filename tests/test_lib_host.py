"""Host-side checks of the HIP library that need no GPU.

* the shared library loads and exports every symbol include/ems.h declares;
* argument and geometry validation return the documented codes;
* host set-up code (closed-form disk S, per-node interface reflection) agrees
  with the oracle;
* the library's Sommerfeld node rules integrate the Sommerfeld identity and
  the multipole-to-Sommerfeld lemma (closed forms, Sections 3.1 and 5.4) to
  near machine precision, i.e. the quadrature the kernels consume is pinned
  on the CPU.
"""
import math
import os
import re

import numpy as np
import pytest
from scipy import special

import paper_2608_26875_amd as E
import workloads as W
from oracle import interface, media, smatrix

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ems.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ems_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(E.lib(), s), s
    assert set(syms) == set(E.EXPORTED)


def test_create_and_validation_without_gpu():
    import ctypes
    lib = E.lib()
    h = ctypes.c_void_p()
    assert lib.ems_create(ctypes.byref(h)) == 0
    m = E.make_media((2, 1, 1), (4, 2, 1.5), 4.0)
    assert lib.ems_set_media(h, ctypes.byref(m)) == 0
    xy = np.array([[0.0, -2.0], [0.5, -2.0]])
    R = np.array([0.4, 0.4])
    p = np.array([3, 3], dtype=np.int32)
    assert lib.ems_set_particles(h, 2, xy.ctypes.data, R.ctypes.data, p.ctypes.data) == 0
    # build before S -> state error
    assert lib.ems_build(h, None) == -5
    S = np.zeros(2 * 14 * 14, complex)
    off = np.array([0, 196, 392], dtype=np.int64)
    assert lib.ems_set_smatrices(h, S.ctypes.data, off.ctypes.data) == 0
    assert lib.ems_build(h, None) == -2                 # overlapping enclosing disks
    assert b"overlap" in lib.ems_last_error(h)
    xy2 = np.array([[0.0, -0.3], [3.0, -2.0]])
    assert lib.ems_set_particles(h, 2, xy2.ctypes.data, R.ctypes.data, p.ctypes.data) == 0
    assert lib.ems_set_smatrices(h, S.ctypes.data, off.ctypes.data) == 0
    assert lib.ems_build(h, None) == -2                 # disk reaches the interface
    bad = np.array([0, 99], dtype=np.int32)
    assert lib.ems_set_particles(h, 2, xy2.ctypes.data, R.ctypes.data, bad.ctypes.data) == -7
    nanxy = np.array([[np.nan, -2.0], [3.0, -2.0]])
    assert lib.ems_set_particles(h, 2, nanxy.ctypes.data, R.ctypes.data, p.ctypes.data) == -6
    neg = E.make_media((2, -1, 1), (4, 2, 1.5), 4.0)
    assert lib.ems_set_media(h, ctypes.byref(neg)) == -1
    lib.ems_destroy(h)


@pytest.mark.parametrize("bc", [0, 1])
def test_disk_smatrix_matches_oracle(bc):
    Em = E.make_media((2, 1, 1), (4, 2, 1.5), 8.0)
    mo = media.Media(2, 1, 1, 4, 2, 1.5, 8.0)
    for a in (0.3, 0.55, 0.7):
        for p in (1, 7, 15):
            Sg = E.smatrix_disk(Em, a, p, bc)
            So = smatrix.disk(mo, a, p, bc)
            assert np.linalg.norm(Sg - So) <= 1e-13 * np.linalg.norm(So)


def test_reflection_matches_oracle():
    Em = E.make_media((2, 1, 1), (4, 2, 1.5), 4.0)
    mo = media.Media(2, 1, 1, 4, 2, 1.5, 4.0)
    for xi in (0.0, 0.3, -1.1, 1.9, 2.7, -3.9, 5.0, 17.0, -40.0, 0.7 - 0.3j, -3.0 + 0.45j):
        Rg = E.reflection(Em, xi)
        Ro = interface.reflection(xi if isinstance(xi, complex) else float(xi), mo)
        assert np.allclose(Rg, Ro, rtol=1e-12, atol=1e-13), xi


def _nodes_for(w, **kw):
    Em = E.make_media(w.host, w.substrate, w.omega)
    return E.sommerfeld_nodes(Em, w.xy, w.p, **kw)


def _s_of(nodes, k):
    xi = nodes[:, 0] + 1j * nodes[:, 1]
    out = np.empty(len(xi), complex)
    for j, z in enumerate(xi):
        bp, d = nodes[j, 4], nodes[j, 5]
        if bp != 0 and abs(abs(bp) - k) <= 1e-14 * k:
            out[j] = interface.branch_s_offset(bp, d, k)
        elif z.imag == 0:
            out[j] = complex(interface.branch_s(z.real, k))
        else:
            out[j] = complex(interface.branch_s(z, k))
    return xi, out


@pytest.mark.parametrize("kind", [1, 0])
def test_node_rule_integrates_sommerfeld_identity(kind):
    """(i/4) H0(k r) = (1/4pi) int e^{-s|Y|}/s e^{i xi X} dxi on the library's nodes,
    over the horizontal span and depths of a C0-like cloud."""
    w = W.c0_circles()
    kw = dict(kind=1) if kind == 1 else dict(kind=0, q=1024)
    nodes, _ = _nodes_for(w, **kw)
    wt = nodes[:, 2] + 1j * nodes[:, 3]
    for k in (2.0, 4.0):
        xi, s = _s_of(nodes, k)
        for X, Y in ((0.0, 2.0), (19.0, 2.0), (-13.5, 5.5), (7.0, 18.0)):
            val = np.sum(wt * np.exp(-s * Y + 1j * xi * X) / s) / (4 * math.pi)
            ex = 0.25j * special.hankel1(0, k * math.hypot(X, Y))
            tol = 1e-13 if kind == 1 else 1e-10
            assert abs(val - ex) <= tol * max(abs(ex), 1e-3), (k, X, Y, abs(val - ex))


@pytest.mark.parametrize("case", [(40, 10, 8.0, 80.0), (16, 10, 4.0, 20.0), (30, 5, 6.0, 100.0),
                                  (40, 15, 8.0, 300.0)])
def test_node_rule_integrates_lemma_high_order(case):
    """Section 5.4 Lemma for n = -2p..2p at the horizontal spreads and depth
    sums the cloud produces.  The sum of many large terms has a rounding floor
    of about eps * sum |terms| (the same for any quadrature of this integral),
    so the bound is 1e-12 |exact| + 64 eps sum |terms|."""
    nn, p, om, width = case
    w = W.small_cloud(nn, seed=3, p=p, omega=om, width=width, depth=(1.0, 10.0))
    dmin, dmax = 2 * np.min(-w.xy[:, 1]), 2 * np.max(-w.xy[:, 1])
    X = float(np.ptp(w.xy[:, 0]))
    nodes, T = _nodes_for(w, kind=1)
    wt = nodes[:, 2] + 1j * nodes[:, 3]
    eps = np.finfo(float).eps
    for k in (om / 2, om):
        xi, s = _s_of(nodes, k)
        z = (xi - s) / k
        for Xv, Y in ((0.0, dmin), (X, dmin), (-X / 2, (dmin + dmax) / 2), (3.0, dmax),
                      (0.77 * X, 1.3 * dmin)):
            for n in (-2 * p, -p, 0, 1, p, 2 * p):
                terms = wt * np.exp(-s * Y + 1j * xi * Xv) / s * (-1j * z) ** n / (1j * math.pi)
                val = np.sum(terms)
                r, th = math.hypot(Xv, Y), math.atan2(Y, Xv)
                ex = special.hankel1(n, k * r) * np.exp(1j * n * th)
                bound = 1e-12 * abs(ex) + 64 * eps * np.sum(np.abs(terms))
                assert abs(val - ex) <= bound, (k, Xv, Y, n, abs(val - ex) / bound)


def test_rotated_prototypes_validation_without_gpu():
    import ctypes
    lib = E.lib()
    h = ctypes.c_void_p()
    assert lib.ems_create(ctypes.byref(h)) == 0
    m = E.make_media((2, 1, 1), (4, 2, 1.5), 4.0)
    assert lib.ems_set_media(h, ctypes.byref(m)) == 0
    xy = np.array([[0.0, -2.0], [3.0, -2.0], [6.0, -2.0]])
    R = np.full(3, 0.4)
    p = np.array([3, 3, 2], dtype=np.int32)
    assert lib.ems_set_particles(h, 3, xy.ctypes.data, R.ctypes.data, p.ctypes.data) == 0
    protos = np.zeros(14 * 14 + 10 * 10, complex)           # orders 3 and 2
    off = np.array([0, 196, 296], dtype=np.int64)
    th = np.array([0.1, 0.2, 0.3])
    ok = np.array([0, 0, 1], dtype=np.int32)
    assert lib.ems_set_smatrices_rotated(h, 2, protos.ctypes.data, off.ctypes.data,
                                         ok.ctypes.data, th.ctypes.data) == 0
    wrong_size = np.array([0, 1, 1], dtype=np.int32)          # order-2 prototype on p = 3
    assert lib.ems_set_smatrices_rotated(h, 2, protos.ctypes.data, off.ctypes.data,
                                         wrong_size.ctypes.data, th.ctypes.data) == -1
    assert b"prototype size" in lib.ems_last_error(h)
    out_of_range = np.array([0, 0, 2], dtype=np.int32)
    assert lib.ems_set_smatrices_rotated(h, 2, protos.ctypes.data, off.ctypes.data,
                                         out_of_range.ctypes.data, th.ctypes.data) == -1
    nan_th = np.array([0.1, np.nan, 0.3])
    assert lib.ems_set_smatrices_rotated(h, 2, protos.ctypes.data, off.ctypes.data,
                                         ok.ctypes.data, nan_th.ctypes.data) == -6
    lib.ems_destroy(h)


def test_rejected_particles_leave_no_valid_state():
    """A rejected ems_set_particles (order out of range) must not leave the
    handle marked as holding particles from an earlier successful call: the
    S-matrices and the build that follow are refused, not run on a mix of
    old and new data."""
    import ctypes
    lib = E.lib()
    h = ctypes.c_void_p()
    assert lib.ems_create(ctypes.byref(h)) == 0
    m = E.make_media((2, 1, 1), (4, 2, 1.5), 4.0)
    assert lib.ems_set_media(h, ctypes.byref(m)) == 0
    xy = np.array([[0.0, -2.0], [3.0, -2.0]])
    R = np.array([0.4, 0.4])
    p = np.array([3, 3], dtype=np.int32)
    assert lib.ems_set_particles(h, 2, xy.ctypes.data, R.ctypes.data, p.ctypes.data) == 0
    bad = np.array([3, 20], dtype=np.int32)
    assert lib.ems_set_particles(h, 2, xy.ctypes.data, R.ctypes.data, bad.ctypes.data) == -7
    # a (4*20+2)^2 block for the second particle is refused: no particles are set
    S = np.zeros(14 * 14 + 82 * 82, complex)
    off = np.array([0, 196, 196 + 82 * 82], dtype=np.int64)
    assert lib.ems_set_smatrices(h, S.ctypes.data, off.ctypes.data) == -5
    assert lib.ems_build(h, None) == -5
    # a valid call restores a usable state; a bad S call clears it again
    assert lib.ems_set_particles(h, 2, xy.ctypes.data, R.ctypes.data, p.ctypes.data) == 0
    S2 = np.zeros(2 * 14 * 14, complex)
    off2 = np.array([0, 196, 392], dtype=np.int64)
    assert lib.ems_set_smatrices(h, S2.ctypes.data, off2.ctypes.data) == 0
    off_bad = np.array([0, 196, 300], dtype=np.int64)
    assert lib.ems_set_smatrices(h, S2.ctypes.data, off_bad.ctypes.data) == -1
    assert lib.ems_build(h, None) == -5
    rneg = np.array([0.4, -0.4])
    assert lib.ems_set_particles(h, 2, xy.ctypes.data, rneg.ctypes.data, p.ctypes.data) == -1
    lib.ems_destroy(h)
