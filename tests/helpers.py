"""Shared test helpers: build the HIP operator and the oracle for one workload."""
from __future__ import annotations

import numpy as np


def product_operator(w, S_blocks=None, sommerfeld=None):
    """Operator of the HIP library for a workload (closed-form disk S unless given)."""
    import paper_2608_26875_amd as E
    media = E.make_media(w.host, w.substrate, w.omega)
    op = E.Operator(w.xy, w.radius, w.p, media, S_blocks=S_blocks, bc=w.bc, sommerfeld=sommerfeld)
    return op


def oracle_media(w):
    from oracle import media
    return media.Media.from_workload(w)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_gpu(v):
    import torch
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.complex128)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()


def rows_of(w, targets):
    """Boolean mask of the coefficient rows of the given particles."""
    off = w.offsets()
    sel = np.zeros(int(off[-1]), bool)
    for i in targets:
        sel[off[i]: off[i + 1]] = True
    return sel
