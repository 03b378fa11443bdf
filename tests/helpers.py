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


def traction_fd(ufun, x, y, lam, mu, h=2e-5):
    """(u, t) at points (x, y): displacement ufun(X, Y) -> [n, 2] and the
    traction T_y u = (mu (d_y u1 + d_x u2), (lambda + 2 mu) d_y u2 + lambda d_x u1)
    from 4th-order central differences of it."""
    def d(dx, dy):
        c = np.array([1.0, -8.0, 8.0, -1.0]) / (12.0 * h)
        offs = (-2, -1, 1, 2)
        return sum(ci * ufun(x + o * dx * h, y + o * dy * h) for ci, o in zip(c, offs))
    u = ufun(x, y)
    ux, uy = d(1, 0), d(0, 1)
    t1 = mu * (uy[:, 0] + ux[:, 1])
    t2 = (lam + 2 * mu) * uy[:, 1] + lam * ux[:, 0]
    return u, np.stack([t1, t2], axis=1)


def at_interface(ufun, x, side, lam, mu):
    """(u, t) at y = 0 from one side (side = -1 host, +1 substrate): cubic
    extrapolation from four heights inside that layer."""
    ds = np.array([1.0, 2.0, 3.0, 4.0]) * 1e-4
    us, ts = [], []
    for dlt in ds:
        u, t = traction_fd(ufun, x, np.full_like(x, side * dlt), lam, mu)
        us.append(u)
        ts.append(t)
    wts = [np.prod([-dj / (di - dj) for dj in ds if dj != di]) for di in ds]
    return sum(wi * u for wi, u in zip(wts, us)), sum(wi * t for wi, t in zip(wts, ts))
