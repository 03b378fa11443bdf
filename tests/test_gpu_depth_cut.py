"""GPU tests of the depth truncation of the tabulated Sommerfeld contractions.

The truncated matrix-core aggregate and disaggregate (rows and columns of the
exponential tables in depth order, per-node particle prefixes, per-particle
node ranges) must agree with the same kernels over every (node, particle)
pair to 1e-13 relative: the pairs left out are bounded far below that (the
host-side pin of the rule).  Checked for the forward and the adjoint apply,
one and three right-hand sides (the batched tile shapes, a ragged last
batch), every tile candidate the autotuner picks, and the mixed form against
the untruncated FP64 apply at the mixed tolerance.
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import product_operator, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402

TOL = 1e-13
TOL_MIXED = 3e-5
Z = E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S


@pytest.fixture(scope="module")
def ops():
    w = W.c1_cloud()
    cut = product_operator(w)
    ic = cut.build()
    full = product_operator(w, sommerfeld={"depth_cut": -1.0})
    iff = full.build()
    print("kept", ic["somm_kept"], iff["somm_kept"], "q", ic["q"], flush=True)
    assert iff["somm_kept"] == 1.0 and ic["somm_kept"] < 0.9
    yield w, cut, full
    del cut, full
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nrhs", [1, 3])
def test_truncated_apply_matches_full(ops, nrhs):
    w, cut, full = ops
    x = to_gpu(W.random_coeffs(w.n_coeff, 40 + nrhs, nrhs=nrhs))
    for flags in (E.EMS_PART_REFL, Z):
        zc = to_np(cut.apply(x, flags=flags))
        zf = to_np(full.apply(x, flags=flags))
        e = rel(zc, zf)
        print("forward", nrhs, flags, e, flush=True)
        assert e <= TOL
        zm = to_np(cut.apply(x, flags=flags | E.EMS_MIXED))
        em = rel(zm, zf)
        print("mixed", nrhs, flags, em, flush=True)
        assert 1e-10 < em <= TOL_MIXED
        ac = to_np(cut.apply(x, flags=flags, adjoint=True))
        af = to_np(full.apply(x, flags=flags, adjoint=True))
        ea = rel(ac, af)
        print("adjoint", nrhs, flags, ea, flush=True)
        assert ea <= TOL


def test_truncated_apply_after_autotune(ops):
    w, cut, full = ops
    for nrhs in (1, 3):
        tiles = cut.autotune(nrhs=nrhs)
        print("tiles", nrhs, tiles, flush=True)
        x = to_gpu(W.random_coeffs(w.n_coeff, 50 + nrhs, nrhs=nrhs))
        e = rel(to_np(cut.apply(x, flags=E.EMS_PART_REFL)), to_np(full.apply(x, flags=E.EMS_PART_REFL)))
        print("after autotune", nrhs, e, flush=True)
        assert e <= TOL


def test_field_with_shallow_receivers(ops):
    """Receivers above the shallowest particle: the field and its adjoint use
    depth ranges formed for the receivers' depth and agree with the
    untruncated kernels (the misfit gradient shares the same ranges)."""
    w, cut, full = ops
    rng = np.random.default_rng(77)
    pts = np.stack([np.linspace(5.0, 195.0, 300), -rng.uniform(0.2, 0.6, 300)], axis=1)
    # keep receivers outside every enclosing disk
    d2 = ((pts[:, None, :] - w.xy[None, :, :]) ** 2).sum(-1)
    pts = pts[np.all(d2 > (1.01 * w.radius[None, :]) ** 2, axis=1)]
    assert len(pts) > 200 and (-pts[:, 1]).min() < (-w.xy[:, 1]).min()
    g = to_gpu(W.random_coeffs(w.n_coeff, 61, nrhs=2))
    uc = to_np(cut.scattered_field(g, pts))
    uf = to_np(full.scattered_field(g, pts))
    e = rel(uc, uf)
    print("field", e, flush=True)
    assert e <= TOL
    res = torch.from_numpy(rng.standard_normal((2, len(pts), 2)) + 1j * rng.standard_normal((2, len(pts), 2))).cuda()
    ac = to_np(cut.scattered_field_adjoint(res, pts))
    af = to_np(full.scattered_field_adjoint(res, pts))
    ea = rel(ac, af)
    print("field adjoint", ea, flush=True)
    assert ea <= TOL
    # deep receivers below the shallowest particle use the build's ranges
    deep = np.stack([np.linspace(5.0, 195.0, 50), np.full(50, -60.0)], axis=1)
    ed = rel(to_np(cut.scattered_field(g, deep)), to_np(full.scattered_field(g, deep)))
    print("deep field", ed, flush=True)
    assert ed <= TOL
