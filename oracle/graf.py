"""Dense free-space multiple-scattering translations (Section 4.2).

The incoming coefficients of particle m collect, from every other particle l,
T^{ml} applied to (alpha^l, beta^l), with T^{ml} = diag(A, B):
  A_ij = H_{i-j}(kp |x_l - x_m|) exp(-i (i - j)(theta_ml - pi)),
  B_ij = the same with ks,
i in Z_{p_m}, j in Z_{p_l}.  theta_ml is read as the polar angle of x_m - x_l
(source l to target m); the Graf-identity test pins this reading.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _translate_one(k: float, xm, xl, pm: int, pl: np.ndarray, coef: list) -> np.ndarray:
    """sum_l T^{ml}(k) c^l for one target m; sources share no particular p."""
    out = np.zeros(2 * pm + 1, dtype=complex)
    for pl_val in np.unique(pl):
        sel = np.nonzero(pl == pl_val)[0]
        if sel.size == 0:
            continue
        d = xm[None, :] - xl[sel]
        r = np.hypot(d[:, 0], d[:, 1])
        th = np.arctan2(d[:, 1], d[:, 0])
        nu = np.arange(-(pm + pl_val), pm + pl_val + 1)
        t = special.hankel1(nu[None, :], k * r[:, None]) * np.exp(
            -1j * nu[None, :] * (th[:, None] - np.pi))
        i = np.arange(-pm, pm + 1)
        j = np.arange(-pl_val, pl_val + 1)
        idx = (i[:, None] - j[None, :]) + (pm + pl_val)
        C = np.stack([coef[s] for s in sel])            # [L, 2 pl + 1]
        for c0 in range(0, sel.size, 512):
            T = t[c0:c0 + 512][:, idx]                     # [L, 2pm+1, 2pl+1]
            out += np.einsum("lij,lj->i", T, C[c0:c0 + 512])
    return out


def apply_free(w, media, x: np.ndarray, targets=None) -> np.ndarray:
    """T_free x for one coefficient vector (layout [alpha, beta] per particle).

    Returns the full-length vector; rows of particles not in ``targets`` are 0.
    """
    kp, ks = media.kp, media.ks
    off = w.offsets()
    p = w.p.astype(int)
    y = np.zeros_like(x, dtype=complex)
    n = w.n
    alpha = [x[off[l]: off[l] + 2 * p[l] + 1] for l in range(n)]
    beta = [x[off[l] + 2 * p[l] + 1: off[l + 1]] for l in range(n)]
    tg = range(n) if targets is None else targets
    for m in tg:
        src = np.array([l for l in range(n) if l != m], dtype=int)
        if src.size == 0:
            continue
        a = _translate_one(kp, w.xy[m], w.xy[src], int(p[m]), p[src], [alpha[l] for l in src])
        b = _translate_one(ks, w.xy[m], w.xy[src], int(p[m]), p[src], [beta[l] for l in src])
        y[off[m]: off[m] + 2 * p[m] + 1] = a
        y[off[m] + 2 * p[m] + 1: off[m + 1]] = b
    return y


def translation_block(k: float, xm, xl, pm: int, pl: int) -> np.ndarray:
    """One Graf block A (or B) as a dense (2pm+1) x (2pl+1) matrix."""
    d = np.asarray(xm, float) - np.asarray(xl, float)
    r = float(np.hypot(d[0], d[1]))
    th = float(np.arctan2(d[1], d[0]))
    i = np.arange(-pm, pm + 1)[:, None]
    j = np.arange(-pl, pl + 1)[None, :]
    return special.hankel1(i - j, k * r) * np.exp(-1j * (i - j) * (th - np.pi))
