"""Captured applies (HIP graphs): every replay equals the eager apply.

Replays are interleaved with eager work on other buffers and host
synchronisations; the input buffer is rewritten between replays (the graph
reads it at replay time); FP64 and mixed, forward and adjoint, direct and
FMM free part.  Same kernels in the same order: equality to rounding order
(<= 1e-15 relative, in practice bitwise).
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


@pytest.mark.parametrize("fmm", [False, True])
def test_graph_replays_match_eager(fmm):
    if fmm:
        w = W.small_cloud(300, seed=19, p=4, omega=3.0, width=100.0, depth=(1.0, 25.0))
    else:
        w = W.small_cloud(30, seed=11, p=5, omega=4.0, width=30.0, depth=(1.0, 6.0), ragged=True)
    op = product_operator(w)
    if fmm:
        op.set_fmm(mode=2, leaf=6)
    op.build()
    X1 = to_gpu(W.random_coeffs(w.n_coeff, 1, nrhs=3))
    X2 = to_gpu(W.random_coeffs(w.n_coeff, 2, nrhs=3))
    for flags in (E.EMS_APPLY_ALL, E.EMS_APPLY_ALL | E.EMS_MIXED):
        for adjoint in (False, True):
            ref1 = to_np(op.apply(X1, flags=flags, adjoint=adjoint))
            ref2 = to_np(op.apply(X2, flags=flags, adjoint=adjoint))
            x = X1.clone()
            y = torch.empty_like(x)
            z = torch.empty_like(x)
            op.apply_graph(x, y, flags=flags, adjoint=adjoint)      # eager + capture
            assert rel(to_np(y), ref1) <= 1e-15
            for rep in range(3):
                op.apply(X2, z, flags=flags, adjoint=adjoint)       # eager work between replays
                torch.cuda.synchronize()
                y.zero_()
                op.apply_graph(x, y, flags=flags, adjoint=adjoint)  # replay
                torch.cuda.synchronize()
                assert rel(to_np(y), ref1) <= 1e-15, (flags, adjoint, rep)
                assert rel(to_np(z), ref2) <= 1e-15
            x.copy_(X2)                                             # new input, same buffer
            op.apply_graph(x, y, flags=flags, adjoint=adjoint)
            torch.cuda.synchronize()
            assert rel(to_np(y), ref2) <= 1e-15
