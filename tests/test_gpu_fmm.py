"""GPU parity of the free-space FMM (and of the full operator at full size).

* FMM free part against the oracle's dense Graf sum on a cloud deep enough
  for three tree levels (P2M, M2M, M2L on two levels, top-level M2L, L2L,
  L2P all exercised), with physical disk S and with random S.
* FMM against the direct GPU sum on the 2000-particle cloud.
* adjoint dot-product test with the FMM on.
* the 2000- and 20000-particle clouds at their benchmark settings against the
  oracle's sampled rows stored under tests/golden (written by
  tests/golden/make_goldens.py from the oracle only).
"""
import hashlib
import os

import numpy as np
import pytest

import workloads as W
from tests.helpers import oracle_media, product_operator, rel, rows_of, to_gpu, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402
from oracle import graf, operator, smatrix  # noqa: E402

HERE = os.path.dirname(__file__)
SF = E.EMS_PART_FREE | E.EMS_PART_S


def _deep_cloud():
    w = W.cloud(400, 120.0, (1.0, 15.0), seed=5, p=8, omega=8.0, name="deep400")
    return w


def test_fmm_free_part_vs_oracle_deep_tree():
    w = _deep_cloud()
    m = oracle_media(w)
    x = W.random_coeffs(w.n_coeff, 31)[0]
    tf = graf.apply_free(w, m, x)
    for S in (smatrix.workload_blocks(w, m), W.random_smatrix_blocks(w.p, seed=8)):
        op = product_operator(w, S_blocks=S)
        op.set_fmm(mode=2, leaf=6, top_boxes=4)
        info = op.build()
        print("deep fmm", info, flush=True)
        assert info["fmm_levels"] >= 3
        g = to_np(op.apply(to_gpu(x[None]), flags=SF))[0]
        ref = operator.s_multiply(w, S, tf)
        e = rel(g, ref)
        print("S T_free x rel err", e, flush=True)
        assert e <= 1e-11
        graw = to_np(op.apply(to_gpu(x[None]), flags=E.EMS_PART_FREE))[0]
        assert rel(graw, tf) <= 1e-11


def test_fmm_vs_direct_c1():
    w = W.c1_cloud()
    x = to_gpu(W.random_coeffs(w.n_coeff, 1003))
    op_f = product_operator(w)
    op_f.set_fmm(mode=2)
    info = op_f.build()
    print("c1 fmm", info, flush=True)
    op_d = product_operator(w)
    op_d.set_fmm(mode=1)
    op_d.build()
    for flags in (SF, E.EMS_APPLY_ALL):
        a = to_np(op_f.apply(x, flags=flags))
        b = to_np(op_d.apply(x, flags=flags))
        e = rel(a, b)
        print("fmm vs direct", flags, e, flush=True)
        assert e <= 1e-11


def test_fmm_adjoint_dot_product():
    w = _deep_cloud()
    S = W.random_smatrix_blocks(w.p, seed=9)
    op = product_operator(w, S_blocks=S)
    op.set_fmm(mode=2, leaf=6, top_boxes=4)
    op.build()
    v = W.random_coeffs(w.n_coeff, 1)[0]
    u = W.random_coeffs(w.n_coeff, 2)[0]
    for flags in (E.EMS_PART_FREE, E.EMS_APPLY_ALL):
        Av = to_np(op.apply(to_gpu(v[None]), flags=flags))[0]
        Ahu = to_np(op.apply(to_gpu(u[None]), flags=flags, adjoint=True))[0]
        lhs, rhs = np.vdot(u, Av), np.vdot(Ahu, v)
        assert abs(lhs - rhs) <= 1e-11 * np.linalg.norm(u) * np.linalg.norm(Av), (flags, lhs, rhs)


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_full_size_sampled_rows_vs_oracle(name):
    path = os.path.join(HERE, "golden", f"{name}_sampled.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_goldens.py)")
    g = np.load(path)
    w = W.c1_cloud() if name == "c1" else W.c2_cloud()
    x = W.random_coeffs(w.n_coeff, 1002)
    assert str(g["x_digest"]) == _digest(x[0]) and str(g["xy_digest"]) == _digest(w.xy)
    op = product_operator(w)
    info = op.build()
    print(name, info, flush=True)
    xg = to_gpu(x)
    rows = g["rows"]
    out = {}
    for key, flags in (("free", E.EMS_PART_FREE), ("s_refl", E.EMS_PART_REFL | E.EMS_PART_S),
                       ("z", E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S)):
        out[key] = to_np(op.apply(xg, flags=flags))[0][rows]
    errs = {k: rel(out[k], g[k]) for k in out}
    print(name, "sampled-row parity", {k: f"{v:.2e}" for k, v in errs.items()},
          "oracle refl err est", float(g["refl_err"]) / float(g["refl_scale"]), flush=True)
    for k, v in errs.items():
        assert v <= 1e-11, (k, v)


def test_fmm_batched_chunks_match_single():
    """The FMM task kernel with 8 right-hand sides per workgroup (and a tail)
    against single applies, forward and adjoint."""
    w = W.small_cloud(400, seed=17, p=4, omega=3.0, width=120.0, depth=(1.0, 30.0))
    op = product_operator(w)
    op.set_fmm(mode=2, leaf=6)
    op.build()
    X = W.random_coeffs(w.n_coeff, 21, nrhs=10)
    for adjoint in (False, True):
        Yb = to_np(op.apply(to_gpu(X), flags=E.EMS_PART_FREE, adjoint=adjoint))
        for r in (0, 9):
            y1 = to_np(op.apply(to_gpu(X[r:r + 1]), flags=E.EMS_PART_FREE, adjoint=adjoint))[0]
            assert rel(Yb[r], y1) < 1e-14, (adjoint, r)
