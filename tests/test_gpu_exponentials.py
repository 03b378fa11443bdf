"""GPU tests of the register form of the Sommerfeld exponentials.

With ``set_exponentials(False)`` (and for every form whose tables were not
built) the matrix-core aggregate and disaggregate form each exponential
E = exp(s_w(xi_j) y -+ i xi_j x) in registers instead of reading a table
(Sections 5.3 and 5.4).  Pins:

* against the oracle, FP64, <= 1e-11 relative L2 on each part of the
  operator: a ragged cloud with random S blocks spanning several node tiles,
  the largest order (p = 16, three 16-mode column tiles) uniform and ragged,
  and the paper's tanh contour (complex nodes, so every coefficient of the
  exponent is non-zero);
* <u, A v> = <A^H u, v> with the adjoint's register-formed factors;
* the mixed form within the mixed tolerance 3e-5 of FP64 (and not FP64 itself);
* the register form against the tables on a 2000-particle cloud: FP64 forward
  and adjoint within 1e-13 (the two differ only in the rounding of the
  exponent and of exp / sin / cos), the complex64 forms within 1e-6 of each
  other (each carries the complex64 rounding of E, 6e-8 relative per entry);
* a tile choice by the autotuner leaves the results unchanged.
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import oracle_media, product_operator, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402
from oracle import graf, operator, smatrix, sommerfeld  # noqa: E402

TOL_APPLY = 1e-11
TOL_MIXED = 3e-5
Z = E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S
PARTS = (("free", E.EMS_PART_FREE), ("s_refl", E.EMS_PART_REFL | E.EMS_PART_S), ("z", Z),
         ("y", E.EMS_APPLY_ALL))


def register_operator(w, **kw):
    op = product_operator(w, **kw)
    op.set_exponentials(False)
    info = op.build()
    assert info["somm_kept"] <= 1.0
    return op, info


def oracle_parts(w, m, S, x):
    tf = graf.apply_free(w, m, x)
    sr = sommerfeld.apply_refl(w, m, x, S_blocks=S, tol=1e-13)
    z = operator.s_multiply(w, S, tf) + sr
    return {"free": tf, "s_refl": sr, "z": z, "y": x - z}


def check_against_oracle(w, op, S, seed, label):
    m = oracle_media(w)
    x = W.random_coeffs(w.n_coeff, seed)[0]
    o = oracle_parts(w, m, S, x)
    for k, flags in PARTS:
        g = to_np(op.apply(to_gpu(x[None]), flags=flags))[0]
        e = rel(g, o[k])
        print(label, k, f"{e:.2e}", flush=True)
        assert e <= TOL_APPLY, (label, k, e)


def test_register_form_ragged_against_oracle():
    w = W.small_cloud(70, seed=12, p=6, omega=5.0, width=50.0, depth=(1.0, 9.0), ragged=True)
    S = W.random_smatrix_blocks(w.p, seed=99)
    op, info = register_operator(w, S_blocks=S)
    print("register build", info, flush=True)
    check_against_oracle(w, op, S, 1002, "ragged")


@pytest.mark.parametrize("ragged", [False, True])
def test_register_form_max_order(ragged):
    w = W.small_cloud(8, seed=5, p=16, omega=4.0, width=14.0, depth=(1.0, 4.0), ragged=ragged)
    S = smatrix.workload_blocks(w, oracle_media(w))
    op, _ = register_operator(w)
    check_against_oracle(w, op, S, 11, f"p16 ragged={ragged}")


def test_register_form_tanh_contour():
    w = W.c0_circles()
    S = smatrix.workload_blocks(w, oracle_media(w))
    op, _ = register_operator(w, sommerfeld=dict(kind=0, q=1024, delta=0.5))
    check_against_oracle(w, op, S, 1001, "tanh contour")


def test_register_form_adjoint_and_mixed():
    w = W.small_cloud(70, seed=12, p=6, omega=5.0, width=50.0, depth=(1.0, 9.0), ragged=True)
    op, info = register_operator(w, S_blocks=W.random_smatrix_blocks(w.p, seed=99))
    assert info["mixed_somm_fp64"] == 0
    v = W.random_coeffs(w.n_coeff, 1)[0]
    u = W.random_coeffs(w.n_coeff, 2)[0]
    for flags in (E.EMS_APPLY_ALL, E.EMS_PART_REFL):
        Av = to_np(op.apply(to_gpu(v[None]), flags=flags))[0]
        Ahu = to_np(op.apply(to_gpu(u[None]), flags=flags, adjoint=True))[0]
        lhs, rhs = np.vdot(u, Av), np.vdot(Ahu, v)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(u) * np.linalg.norm(Av))
    x = to_gpu(W.random_coeffs(w.n_coeff, 31, nrhs=2))
    for flags in (Z, E.EMS_PART_REFL):
        z64 = to_np(op.apply(x, flags=flags))
        z32 = to_np(op.apply(x, flags=flags | E.EMS_MIXED))
        e = rel(z32, z64)
        print("register mixed vs fp64", flags, e, flush=True)
        assert 1e-10 < e <= TOL_MIXED, (flags, e)


def test_register_form_matches_tables():
    w = W.c1_cloud()
    x = to_gpu(W.random_coeffs(w.n_coeff, 77, nrhs=1))
    out = {}
    for tab in (True, False):
        op = product_operator(w)
        op.set_exponentials(tab)
        op.build()
        out[tab] = {
            "fp64": to_np(op.apply(x, flags=E.EMS_PART_REFL)),
            "mixed": to_np(op.apply(x, flags=E.EMS_PART_REFL | E.EMS_MIXED)),
            "adj": to_np(op.apply(x, flags=E.EMS_PART_REFL, adjoint=True)),
        }
        del op
    for k, tol in (("fp64", 1e-13), ("adj", 1e-13), ("mixed", 1e-6)):
        e = rel(out[False][k], out[True][k])
        print("register vs tables", k, f"{e:.2e}", flush=True)
        assert e <= tol, (k, e)
    assert rel(out[False]["mixed"], out[False]["fp64"]) <= TOL_MIXED


def test_register_form_autotune_keeps_results():
    w = W.small_cloud(300, seed=21, p=8, omega=5.0, width=120.0, depth=(1.0, 12.0), ragged=True)
    op, _ = register_operator(w)
    x = to_gpu(W.random_coeffs(w.n_coeff, 5, nrhs=3))
    before = to_np(op.apply(x, flags=E.EMS_PART_REFL))
    tiles = op.autotune(3)
    print("register tiles", tiles, flush=True)
    after = to_np(op.apply(x, flags=E.EMS_PART_REFL))
    assert rel(after, before) <= 1e-14
