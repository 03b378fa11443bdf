"""GPU tests of the block GMRES solver (one Krylov space for a group of up to
64 right-hand sides, block Gram-Schmidt and Cholesky QR on the matrix cores).

Pins (the solution of A x = b is unique, so every column is checked against
the oracle's operator, not against another solver of the library):
* the 16-particle workload with 8 plane-wave right-hand sides, with and
  without the cluster preconditioner: every column meets the
  backward-residual bound ||b - A_oracle x|| / ||b|| <= 1e-9;
* short restarts (two block steps) with columns converging at different
  cycles: the converged columns leave the block and the rest still meet 1e-10;
* the adjoint block solve against the oracle's dense A^H (6 particles);
* 70 right-hand sides (two groups, 64 + 6) against the dense oracle matrix;
* a block of 1 right-hand side agrees with the lock-step solver to the
  solvers' own tolerance.
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import oracle_media, product_operator, to_gpu, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402
from oracle import incident, operator, smatrix  # noqa: E402


def waves8():
    return [(k % 2, a) for k, a in enumerate(np.radians([-60, -40, -20, -5, 5, 20, 40, 60]))]


@pytest.mark.parametrize("precond", [0, 1])
def test_block_gmres_c0_against_oracle(precond):
    w = W.c0_circles()
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    op = product_operator(w)
    if precond:
        op.set_precond(4 * 42)
    op.build()
    wv = waves8()
    b = op.incident(wv)
    x, info = op.solve(b, tol=1e-10, restart=0, maxit=300, precond=precond, block=True)
    print("block c0", precond, info, flush=True)
    assert info["converged"] == 1 and info["relres"] <= 1e-10
    hist = op.solve_history()
    assert len(hist) == info["iters"] and hist[-1] <= 1e-10 * 1.01
    X = to_np(x)
    for r, (wave, ang) in enumerate(wv):
        b_orc = incident.rhs(w, m, S, wave, ang)
        res = b_orc - operator.apply(w, m, S, X[r], tol=1e-13)
        assert np.linalg.norm(res) / np.linalg.norm(b_orc) <= 1e-9, r


def test_block_gmres_short_restarts_and_deflation():
    """Random right-hand sides of very different sizes; two block steps per
    cycle, so the solve runs through many restarts and columns leave the
    block as they converge (a sparse cloud: weak coupling keeps GMRES with
    such short cycles from stagnating)."""
    w = W.small_cloud(10, seed=51, p=4, omega=5.0, width=80.0, depth=(1.0, 6.0), ragged=True)
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    op = product_operator(w)
    op.build()
    B = W.random_coeffs(w.n_coeff, 52, nrhs=6)
    B *= np.array([1.0, 1e-3, 10.0, 1.0, 0.1, 1.0])[:, None]
    x, info = op.solve(to_gpu(B), tol=1e-10, restart=2, maxit=400, block=True)
    print("block restarts", info, flush=True)
    assert info["converged"] == 1
    X = to_np(x)
    for r in range(6):
        res = B[r] - operator.apply(w, m, S, X[r], tol=1e-13)
        assert np.linalg.norm(res) / np.linalg.norm(B[r]) <= 1e-9, r


def test_block_gmres_adjoint_against_dense_oracle():
    w = W.small_cloud(6, seed=46, p=3, omega=4.0, width=9.0, depth=(1.0, 4.0), ragged=True)
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    A = operator.dense_matrix(w, m, S, tol=1e-12)
    op = product_operator(w)
    op.set_precond(3 * 14)
    op.build()
    B = W.random_coeffs(w.n_coeff, 12, nrhs=3)
    lam, info = op.solve(to_gpu(B), tol=1e-12, restart=0, maxit=200, adjoint=True, precond=1,
                         block=True)
    assert info["converged"] == 1
    L = to_np(lam)
    for r in range(3):
        assert np.linalg.norm(B[r] - A.conj().T @ L[r]) / np.linalg.norm(B[r]) <= 1e-10


def test_block_gmres_two_groups():
    w = W.small_cloud(5, seed=53, p=3, omega=4.0, width=8.0, depth=(1.0, 4.0), ragged=True)
    m = oracle_media(w)
    S = smatrix.workload_blocks(w, m)
    A = operator.dense_matrix(w, m, S, tol=1e-12)
    op = product_operator(w)
    op.build()
    B = W.random_coeffs(w.n_coeff, 54, nrhs=70)
    x, info = op.solve(to_gpu(B), tol=1e-11, restart=0, maxit=200, block=True)
    assert info["converged"] == 1
    X = to_np(x)
    res = np.linalg.norm(B - X @ A.T, axis=1) / np.linalg.norm(B, axis=1)
    print("two groups", info, res.max(), flush=True)
    assert res.max() <= 1e-10


def test_block_of_one_matches_lockstep():
    w = W.small_cloud(12, seed=55, p=4, omega=4.0, width=15.0, depth=(1.0, 5.0))
    op = product_operator(w)
    op.build()
    b = to_gpu(W.random_coeffs(w.n_coeff, 56, nrhs=1))
    x1, i1 = op.solve(b, tol=1e-12, restart=0, maxit=300, block=True)
    x0, i0 = op.solve(b, tol=1e-12, restart=0, maxit=300)
    assert i1["converged"] == 1 and i0["converged"] == 1
    d = np.linalg.norm(to_np(x1) - to_np(x0)) / np.linalg.norm(to_np(x0))
    print("block of one vs lock-step", d, i1["iters"], i0["iters"], flush=True)
    assert d <= 1e-9


def test_block_gmres_argument_errors():
    w = W.small_cloud(4, seed=57, p=3, omega=4.0, width=6.0, depth=(1.0, 3.0))
    op = product_operator(w)
    op.build()
    b = to_gpu(W.random_coeffs(w.n_coeff, 58, nrhs=2))
    with pytest.raises(RuntimeError, match="FP64"):
        op.solve(b, tol=1e-8, maxit=10, precision=1, block=True)
