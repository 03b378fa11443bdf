"""GPU parity: the HIP operator (through the C ABI) against the CPU oracle.

Tolerances: FP64 apply <= 1e-11 relative L2, checked on y = x - S T x and on
the non-identity part z = S T x (the identity would hide errors in y), plus
the free and reflected parts separately; GMRES solution: backward residual
||b - A_oracle x_gpu|| / ||b|| <= 1e-9 under the oracle's operator.
"""
import math

import numpy as np
import pytest

import workloads as W
from tests.helpers import oracle_media, product_operator, rel, rows_of, to_gpu, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402
from oracle import graf, incident, operator, smatrix, sommerfeld  # noqa: E402

TOL_APPLY = 1e-11


def _parts(op, x):
    xg = to_gpu(x[None, :])
    out = {}
    for name, flags in (("free", E.EMS_PART_FREE), ("s_refl", E.EMS_PART_REFL | E.EMS_PART_S),
                        ("z", E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S),
                        ("y", E.EMS_APPLY_ALL)):
        out[name] = to_np(op.apply(xg, flags=flags))[0]
    torch.cuda.synchronize()
    return out


def _oracle_parts(w, m, S, x, targets=None, tol=1e-13):
    tf = graf.apply_free(w, m, x, targets=targets)
    sr = sommerfeld.apply_refl(w, m, x, targets=targets, S_blocks=S, tol=tol)
    z = operator.s_multiply(w, S, tf, targets=targets) + sr
    y = x - z
    if targets is not None:
        y = np.where(rows_of(w, targets), y, 0)
    return {"free": tf, "s_refl": sr, "z": z, "y": y}


def _compare(w, gpu, orc, targets=None, tol=TOL_APPLY):
    sel = rows_of(w, targets if targets is not None else range(w.n))
    errs = {k: rel(gpu[k][sel], orc[k][sel]) for k in orc}
    print("parity", w.name, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    return errs


def test_c0_apply_parity():
    """16 rigid circles, p = 10, omega = 4 (kp a = 1), direct Graf, graded real-axis rule."""
    w = W.c0_circles()
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    op = product_operator(w)
    info = op.build()
    print("c0 build", info, flush=True)
    x = W.random_coeffs(w.n_coeff, 1000)[0]
    _compare(w, _parts(op, x), _oracle_parts(w, m, S, x))


def test_c0_paper_contour_parity():
    """The paper's tanh contour (Section 5.1) with q = 1024 nodes meets the bound too."""
    w = W.c0_circles()
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    op = product_operator(w, sommerfeld=dict(kind=0, q=1024, delta=0.5))
    op.build()
    x = W.random_coeffs(w.n_coeff, 1001)[0]
    _compare(w, _parts(op, x), _oracle_parts(w, m, S, x))


def test_ragged_random_s_parity():
    """Ragged p, random S blocks given to both sides, traction-free + rigid mix,
    a cloud spanning several 256-lane tiles of nodes and a ragged last tile."""
    w = W.small_cloud(70, seed=12, p=6, omega=5.0, width=50.0, depth=(1.0, 9.0), ragged=True)
    m = oracle_media(w)
    S = W.random_smatrix_blocks(w.p, seed=99)
    op = product_operator(w, S_blocks=S)
    info = op.build()
    print("ragged build", info, flush=True)
    x = W.random_coeffs(w.n_coeff, 1002)[0]
    _compare(w, _parts(op, x), _oracle_parts(w, m, S, x))


def test_single_particle_and_p1():
    """N = 1: no free-space pair, only the self-reflection; p = 1 edge."""
    for p in (1, 4):
        w = W.small_cloud(1, seed=3, p=p, omega=4.0, width=4.0, depth=(1.0, 2.0))
        m = oracle_media(w)
        S = smatrix.workload_blocks(w, m)
        op = product_operator(w)
        op.build()
        x = W.random_coeffs(w.n_coeff, 7)[0]
        g = _parts(op, x)
        assert np.all(g["free"] == 0)
        o = _oracle_parts(w, m, S, x)
        for k in ("s_refl", "z", "y"):
            assert rel(g[k], o[k]) <= TOL_APPLY


def test_max_order_p16():
    """The largest truncation order the kernels compile for (p = 16: 33
    modes, three 16-mode matrix-core column tiles, 64-lane Graf rows),
    uniform and ragged, against the oracle."""
    for ragged in (False, True):
        w = W.small_cloud(8, seed=5, p=16, omega=4.0, width=14.0, depth=(1.0, 4.0), ragged=ragged)
        m = oracle_media(w)
        S = smatrix.workload_blocks(w, m)
        op = product_operator(w)
        op.build()
        x = W.random_coeffs(w.n_coeff, 11)[0]
        g = _parts(op, x)
        o = _oracle_parts(w, m, S, x)
        for k in ("free", "s_refl", "z", "y"):
            e = rel(g[k], o[k])
            print("p16", ragged, k, e, flush=True)
            assert e <= TOL_APPLY, (ragged, k, e)


def test_batched_rhs_matches_single():
    w = W.small_cloud(30, seed=4, p=5, omega=4.0, width=30.0, depth=(1.0, 6.0))
    op = product_operator(w)
    op.build()
    X = W.random_coeffs(w.n_coeff, 3, nrhs=5)
    Yb = to_np(op.apply(to_gpu(X)))
    for r in range(5):
        y1 = to_np(op.apply(to_gpu(X[r:r + 1])))[0]
        assert rel(Yb[r], y1) < 1e-14


def test_adjoint_dot_product():
    """<w, A v> = <A^H w, v> for the whole operator and for each part."""
    w = W.small_cloud(25, seed=8, p=5, omega=4.0, width=25.0, depth=(1.0, 6.0), ragged=True)
    S = W.random_smatrix_blocks(w.p, seed=5)
    op = product_operator(w, S_blocks=S)
    op.build()
    v = W.random_coeffs(w.n_coeff, 1)[0]
    u = W.random_coeffs(w.n_coeff, 2)[0]
    for flags in (E.EMS_APPLY_ALL, E.EMS_PART_FREE, E.EMS_PART_REFL,
                  E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S):
        Av = to_np(op.apply(to_gpu(v[None]), flags=flags))[0]
        Ahu = to_np(op.apply(to_gpu(u[None]), flags=flags, adjoint=True))[0]
        lhs = np.vdot(u, Av)
        rhs = np.vdot(Ahu, v)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(u) * np.linalg.norm(Av)), flags


def test_incident_rhs_parity():
    w = W.c0_circles()
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    op = product_operator(w)
    op.build()
    waves = [(0, math.radians(30.0)), (1, math.radians(-55.0)), (1, math.radians(20.0))]
    b = to_np(op.incident(waves))
    for r, (wv, ang) in enumerate(waves):
        assert rel(b[r], incident.rhs(w, m, S, wv, ang)) < 1e-12


def test_c0_gmres_solution_parity():
    """GMRES to 1e-10 on the GPU; backward residual under the oracle <= 1e-9."""
    w = W.c0_circles()
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    op = product_operator(w)
    op.build()
    wave, ang = w.incidence[0]
    b_orc = incident.rhs(w, m, S, wave, ang)
    bg = op.incident([(wave, ang)])
    x, info = op.solve(bg, tol=1e-10, restart=200, maxit=400)
    print("c0 solve", info, flush=True)
    assert info["converged"] == 1
    xg = to_np(x)[0]
    r = b_orc - operator.apply(w, m, S, xg, tol=1e-13)
    assert np.linalg.norm(r) / np.linalg.norm(b_orc) <= 1e-9


def test_geometry_and_argument_errors():
    w = W.small_cloud(3, seed=2, p=3)
    xy = w.xy.copy()
    xy[1] = xy[0] + np.array([0.1, 0.0])
    media = E.make_media(w.host, w.substrate, w.omega)
    op = E.Operator(xy, w.radius, w.p, media, bc=w.bc)
    with pytest.raises(E.EmsError) as ei:
        op.build()
    assert ei.value.code == -2
    xy = w.xy.copy()
    xy[0, 1] = -0.1
    op = E.Operator(xy, w.radius, w.p, media, bc=w.bc)
    with pytest.raises(E.EmsError) as ei:
        op.build()
    assert ei.value.code == -2


def test_scattered_field_parity():
    """Scattered displacement (direct outgoing fields + reflected Sommerfeld
    field) at receivers between the interface and the particles and among
    them, against the oracle."""
    from oracle import field
    w = W.small_cloud(12, seed=6, p=6, omega=4.0, width=14.0, depth=(1.0, 4.0))
    m = oracle_media(w)
    op = product_operator(w)
    op.build()
    g = W.random_coeffs(w.n_coeff, 77, nrhs=2)
    pts = np.stack([np.linspace(-2.0, 16.0, 23), np.full(23, -0.3)], 1)
    pts = np.concatenate([pts, np.array([[7.1, -6.5], [3.3, -5.9]])])
    far = np.min(np.hypot(pts[:, None, 0] - w.xy[None, :, 0], pts[:, None, 1] - w.xy[None, :, 1])
                 - w.radius[None, :], axis=1)
    pts = pts[far > 0.05]
    u = to_np(op.scattered_field(to_gpu(g), pts))
    for r in range(2):
        ref = field.scattered(w, m, g[r], pts, tol=1e-13)
        e = rel(u[r], ref)
        print("field rel err", e, flush=True)
        assert e <= 1e-11


def test_scattered_field_rejects_receiver_inside_disk():
    w = W.small_cloud(3, seed=6, p=3, omega=4.0, width=8.0, depth=(1.0, 4.0))
    op = product_operator(w)
    op.build()
    g = to_gpu(W.random_coeffs(w.n_coeff, 1))
    with pytest.raises(E.EmsError) as ei:
        op.scattered_field(g, w.xy[:1] + 0.01)
    assert ei.value.code == -2


@pytest.mark.parametrize("flags_name", ["fp64", "mixed"])
def test_batched_chunks_match_single(flags_name):
    """11 right-hand sides (chunks of 8 plus a ragged tail in the direct Graf,
    FMM and matrix-core kernels) against one-at-a-time applies, forward and
    adjoint; the FP32 form to its own rounding level."""
    w = W.small_cloud(40, seed=14, p=5, omega=4.0, width=40.0, depth=(1.0, 6.0), ragged=True)
    op = product_operator(w)
    op.build()
    flags = E.EMS_APPLY_ALL | (E.EMS_MIXED if flags_name == "mixed" else 0)
    tol = 1e-14 if flags_name == "fp64" else 1e-6
    X = W.random_coeffs(w.n_coeff, 8, nrhs=11)
    for adjoint in (False, True):
        Yb = to_np(op.apply(to_gpu(X), flags=flags, adjoint=adjoint))
        for r in (0, 7, 8, 10):
            y1 = to_np(op.apply(to_gpu(X[r:r + 1]), flags=flags, adjoint=adjoint))[0]
            assert rel(Yb[r], y1) < tol, (adjoint, r, rel(Yb[r], y1))


def test_autotune_keeps_results():
    w = W.small_cloud(30, seed=4, p=6, omega=4.0, width=30.0, depth=(1.0, 6.0))
    op = product_operator(w)
    op.build()
    X = to_gpu(W.random_coeffs(w.n_coeff, 3, nrhs=6))
    before = {m: to_np(op.apply(X, flags=E.EMS_APPLY_ALL | m)) for m in (0, E.EMS_MIXED)}
    for nr in (1, 6):
        choice = op.autotune(nr)
        print("autotune", nr, choice, flush=True)
        assert choice["aggregate_fp64"][0] > 0
    for m in (0, E.EMS_MIXED):
        after = to_np(op.apply(X, flags=E.EMS_APPLY_ALL | m))
        assert rel(after, before[m]) < (1e-14 if m == 0 else 1e-6)
