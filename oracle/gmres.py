"""Textbook GMRES (Saad and Schultz 1986), the solver named in Sections 4.2 and 5.2.

x0 = 0; Arnoldi with classical Gram-Schmidt applied twice; Givens rotations
G = [[c, s], [-conj(s), conj(c)]] on the Hessenberg matrix; stop when the relative residual estimate
|g_{k+1}| / ||b|| <= tol.  No restart (the paper does not state one).
"""
from __future__ import annotations

import numpy as np


def gmres(apply, b: np.ndarray, tol: float = 1e-10, maxit: int = 500):
    """Returns (x, info) with info = {"iters", "relres", "history"}."""
    b = np.asarray(b, complex)
    n = b.size
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n, complex), {"iters": 0, "relres": 0.0, "history": [0.0]}
    V = np.zeros((maxit + 1, n), complex)
    H = np.zeros((maxit + 1, maxit), complex)
    cs = np.zeros(maxit, complex)
    sn = np.zeros(maxit, complex)
    g = np.zeros(maxit + 1, complex)
    g[0] = beta
    V[0] = b / beta
    hist = [1.0]
    k_done = 0
    for k in range(maxit):
        wv = apply(V[k])
        h = np.zeros(k + 2, complex)
        for _ in range(2):
            c = V[: k + 1].conj() @ wv
            wv = wv - V[: k + 1].T @ c
            h[: k + 1] += c
        h[k + 1] = np.linalg.norm(wv)
        if h[k + 1] != 0:
            V[k + 1] = wv / h[k + 1]
        for i in range(k):
            t = cs[i] * h[i] + sn[i] * h[i + 1]
            h[i + 1] = -np.conj(sn[i]) * h[i] + np.conj(cs[i]) * h[i + 1]
            h[i] = t
        den = np.hypot(abs(h[k]), abs(h[k + 1]))
        if den == 0:
            cs[k], sn[k] = 1.0, 0.0
        else:
            cs[k] = np.conj(h[k]) / den
            sn[k] = np.conj(h[k + 1]) / den
        h[k] = cs[k] * h[k] + sn[k] * h[k + 1]
        h[k + 1] = 0.0
        g[k + 1] = -np.conj(sn[k]) * g[k]
        g[k] = cs[k] * g[k]
        H[: k + 2, k] = h
        k_done = k + 1
        rel = abs(g[k + 1]) / beta
        hist.append(rel)
        if rel <= tol:
            break
    y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
    x = V[:k_done].T @ y
    return x, {"iters": k_done, "relres": hist[-1], "history": hist}
