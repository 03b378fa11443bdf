"""The allocation-free apply (ems_apply_noalloc, workspace in the library's
static device array) against ems_apply, through the C ABI.

Two calls in a row, the second with a smaller input (the 2000-particle cloud
with the FMM and three right-hand sides, then the 16-particle workload with
one): each must equal ems_apply on the same input to 1e-13 relative on the
non-identity part z = S T x (only the order of partial sums may differ: the
static array can force fewer split-K chunks), FP64 and mixed; ems_apply keeps
working after it, and a workspace beyond the array is refused.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from tests.helpers import product_operator, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2608_26875_amd as E  # noqa: E402

Z = E.EMS_PART_FREE | E.EMS_PART_REFL | E.EMS_PART_S


def _noalloc(op, x, flags):
    y = torch.empty_like(x)
    rc = E.lib().ems_apply_noalloc(op.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   int(x.shape[0]), int(flags), None)
    assert rc == 0, E.lib().ems_last_error(op.h)
    return y


def _check(op, w, nrhs, seed):
    x = to_gpu(W.random_coeffs(w.n_coeff, seed, nrhs=nrhs))
    for flags, tol in ((Z, 1e-13), (E.EMS_APPLY_ALL, 1e-13), (Z | E.EMS_MIXED, 1e-5)):
        y0 = to_np(op.apply(x, flags=flags))
        y1 = to_np(_noalloc(op, x, flags))
        torch.cuda.synchronize()
        e = rel(y1, y0)
        print(w.name, nrhs, flags, "noalloc vs apply", e, flush=True)
        assert np.all(np.isfinite(y1)) and e <= tol, (flags, e)
    return x


def test_noalloc_apply_matches_apply_two_calls():
    w1 = W.c1_cloud()
    op1 = product_operator(w1)
    assert op1.build()["fmm_levels"] > 0
    _check(op1, w1, 3, 51)
    w0 = W.c0_circles()
    op0 = product_operator(w0)
    op0.build()
    x0 = _check(op0, w0, 1, 52)
    # the handle's own workspace is untouched: ems_apply still agrees with a
    # fresh operator
    op2 = product_operator(w0)
    op2.build()
    assert rel(to_np(op0.apply(x0, flags=Z)), to_np(op2.apply(x0, flags=Z))) <= 1e-13


def test_noalloc_rejects_oversized_workspace():
    w1 = W.c1_cloud()
    op1 = product_operator(w1)
    op1.build()
    x = torch.zeros((200, w1.n_coeff), dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    rc = E.lib().ems_apply_noalloc(op1.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   200, E.EMS_APPLY_ALL, None)
    assert rc == -1  # EMS_ERR_ARG
    assert b"static scratch" in E.lib().ems_last_error(op1.h)
