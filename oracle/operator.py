"""The multiple-scattering operator of the Schur-complement system (Section 5.2).

Section 4.2 gives the S-preconditioned free-space system (identity on the
diagonal blocks, -S_m T^{ml} off it).  Section 5.2 eliminates the interface
densities (A is block diagonal, inverted directly) and leaves
[D - C A^{-1} B] gamma = rhs on the multipole unknowns only.  Applied to a
coefficient vector x:
    y_m = x_m - S_m ( (T_free x)_m + (T_refl x)_m ),
with T_free the dense Graf translations and T_refl the Sommerfeld reflected
part (every pair, self-pair included).  The adjoint is the conjugate
transpose.
"""
from __future__ import annotations

import numpy as np

from . import graf, sommerfeld


def s_multiply(w, S_blocks, v: np.ndarray, targets=None, adjoint: bool = False) -> np.ndarray:
    off = w.offsets()
    out = np.zeros_like(v)
    for i in (range(w.n) if targets is None else targets):
        S = S_blocks[i]
        out[off[i]: off[i + 1]] = (S.conj().T if adjoint else S) @ v[off[i]: off[i + 1]]
    return out


def apply(w, m, S_blocks, x: np.ndarray, targets=None, tol: float = 1e-13,
          parts: str = "y", return_parts: bool = False):
    """y = x - S (T_free + T_refl) x on the requested target rows.

    ``parts``: "y" full operator, "z" the non-identity part S (T_free + T_refl) x.
    With ``return_parts`` also returns T_free x and S T_refl x.
    """
    x = np.asarray(x, complex)
    tf = graf.apply_free(w, m, x, targets=targets)
    z_free = s_multiply(w, S_blocks, tf, targets=targets)
    z_refl = sommerfeld.apply_refl(w, m, x, targets=targets, S_blocks=S_blocks, tol=tol)
    z = z_free + z_refl
    if parts == "z":
        out = z
    else:
        out = -z
        sel = np.zeros(len(x), bool)
        off = w.offsets()
        for i in (range(w.n) if targets is None else targets):
            sel[off[i]: off[i + 1]] = True
        out[sel] += x[sel]
    if return_parts:
        return out, {"free": tf, "s_free": z_free, "s_refl": z_refl}
    return out


def dense_matrix(w, m, S_blocks, tol: float = 1e-13) -> np.ndarray:
    """Assemble the whole operator column by column (small problems only)."""
    n = int(w.offsets()[-1])
    A = np.zeros((n, n), dtype=complex)
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        A[:, j] = apply(w, m, S_blocks, e, tol=tol)
    return A
