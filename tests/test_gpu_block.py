"""A block of 64 right-hand sides on a cloud shaped like the uneven-order
batch (orders p_i = ceil(ks a_i) + 8, 11 to 14 at omega = 8; 24 particles),
with the FMM forced on over several quadtree levels and the Sommerfeld tiles
tuned for 64 right-hand sides, against the oracle.

The oracle's z = S (T_free + T_refl) x of four of the 64 columns (0, 17, 38,
63: the first and last and two inside the right-hand-side chunks of the
kernels) is stored by tests/golden/make_goldens.py (block64).  Bounds: FP64
1e-11 relative L2 per column; mixed (FP32 contractions, FP32 near field and
FP32 matrix-core M2L where the symbols fit) 3e-5, the mixed-form tolerance;
the captured HIP graph of the block apply equals the eager apply bit for bit
on every replay.
"""
import hashlib
import os

import numpy as np
import pytest

import workloads as W
from tests.helpers import product_operator, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402
from tests.golden.make_goldens import BLOCK_COLS, block_cloud  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
Z = E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def test_block64_against_oracle():
    g = np.load(os.path.join(HERE, "golden", "block64_sampled.npz"))
    w = block_cloud()
    x = W.random_coeffs(w.n_coeff, 1003, nrhs=64)
    assert str(g["x_digest"]) == _digest(x) and str(g["xy_digest"]) == _digest(w.xy)
    assert list(g["cols"]) == BLOCK_COLS
    op = product_operator(w)
    op.set_fmm(mode=2, leaf=2, top_boxes=4)
    info = op.build()
    assert info["fmm_levels"] >= 2
    tiles = op.autotune(64)
    xg = to_gpu(x)
    z64 = to_np(op.apply(xg, flags=Z))
    z32 = to_np(op.apply(xg, flags=Z | E.EMS_MIXED))
    print("block64", info["fmm_levels"], tiles, flush=True)
    for i, c in enumerate(BLOCK_COLS):
        e64, e32 = rel(z64[c], g["z"][i]), rel(z32[c], g["z"][i])
        print("column", c, "fp64", e64, "mixed", e32, flush=True)
        assert e64 <= 1e-11 and e32 <= 3e-5
    # the captured graph of the block apply, replayed with eager work between
    y = torch.empty_like(xg)
    for _ in range(3):
        op.apply_graph(xg, y, flags=Z)
        torch.cuda.synchronize()
        assert np.array_equal(to_np(y), z64)
        op.apply(xg, flags=Z)
