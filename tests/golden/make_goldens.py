"""Write the oracle's sampled-row references for the full-size clouds.

Calls only the CPU oracle and the seeded input generators.  For each cloud it
stores, for a few target particles, the free part T_free x, the reflected part
S T_refl x and z = S (T_free + T_refl) x of the operator at the seeded random
vector x (seed 1002), plus a checksum of x and of the centres so a test can
tell that its inputs are the same.

    python tests/golden/make_goldens.py c1 c2 block64 grad9

block64: the full z rows of four columns of a 64-column block on a cloud
shaped like the uneven-order batch; grad9: the oracle's misfit gradient of a
nine-particle case (tests run it with the FMM forced on).
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import graf, media, smatrix, sommerfeld  # noqa: E402

TARGETS = {"c1": [0, 999, 1998], "c2": [0, 7777, 19999]}


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def make(name):
    w = W.c1_cloud() if name == "c1" else W.c2_cloud()
    m = media.Media.from_workload(w)
    tg = TARGETS[name]
    x = W.random_coeffs(w.n_coeff, 1002)[0]
    Sb = [None] * w.n
    for i in tg:
        Sb[i] = smatrix.disk(m, float(w.radius[i]), int(w.p[i]), int(w.bc[i]))
    t0 = time.time()
    tf = graf.apply_free(w, m, x, targets=tg)
    t1 = time.time()
    sr, info = sommerfeld.apply_refl(w, m, x, targets=tg, S_blocks=Sb, tol=1e-12, return_info=True)
    t2 = time.time()
    off = w.offsets()
    rows = np.concatenate([np.arange(off[i], off[i + 1]) for i in tg])
    sf = np.zeros_like(tf)
    for i in tg:
        sf[off[i]: off[i + 1]] = Sb[i] @ tf[off[i]: off[i + 1]]
    np.savez(os.path.join(HERE, f"{name}_sampled.npz"), targets=np.array(tg), rows=rows,
             free=tf[rows], s_free=sf[rows], s_refl=sr[rows], z=(sf + sr)[rows],
             x_digest=np.array(digest(x)), xy_digest=np.array(digest(w.xy)),
             refl_err=np.array(info["err"]), refl_scale=np.array(info["scale"]),
             refl_neval=np.array(info["neval"]), refl_seconds=np.array(t2 - t1))
    print(f"{name}: free {t1 - t0:.1f}s refl {t2 - t1:.1f}s {info}", flush=True)


def block_cloud():
    """A cloud shaped like the uneven-order batch (orders p_i = ceil(ks a_i) + 8
    at omega = 8, 11 to 14 here), small enough for the oracle: 24 particles."""
    return W.cloud(24, 30.0, (1.0, 6.0), seed=33, p=None, omega=8.0, name="block64")


BLOCK_COLS = [0, 17, 38, 63]


def make_block():
    """z = S (T_free + T_refl) x for sampled columns of a 64-column block x
    (seed 1003)."""
    from oracle import operator
    w = block_cloud()
    m = media.Media.from_workload(w)
    S = smatrix.workload_blocks(w, m)
    x = W.random_coeffs(w.n_coeff, 1003, nrhs=64)
    t0 = time.time()
    z = np.stack([operator.apply(w, m, S, x[c], tol=1e-13, parts="z") for c in BLOCK_COLS])
    np.savez(os.path.join(HERE, "block64_sampled.npz"), cols=np.array(BLOCK_COLS), z=z,
             x_digest=np.array(digest(x)), xy_digest=np.array(digest(w.xy)))
    print(f"block64: {time.time() - t0:.1f}s", flush=True)


def grad_case():
    """Nine particles in a row (ragged orders up to 4), two plane waves, seven
    receivers: small enough for the oracle's gradient, wide enough for a
    quadtree of several levels."""
    import math
    w = W.small_cloud(9, seed=61, p=4, omega=4.0, width=20.0, depth=(1.0, 3.0), ragged=True)
    pts = np.stack([np.linspace(-1.0, 21.0, 7), np.full(7, -0.4)], 1)
    waves = [(0, math.radians(25)), (1, math.radians(-40))]
    rng = np.random.default_rng(61)
    u_obs = (rng.normal(size=(2, 7, 2)) + 1j * rng.normal(size=(2, 7, 2))) * 0.1
    return w, pts, waves, u_obs


def make_grad():
    from oracle import gradient
    w, pts, waves, u_obs = grad_case()
    m = media.Media.from_workload(w)
    S = smatrix.workload_blocks(w, m)
    t0 = time.time()
    J, gxy, gl = gradient.gradient(w, m, S, waves, pts, u_obs)
    np.savez(os.path.join(HERE, "grad9_oracle.npz"), J=np.array(J), gxy=gxy, glame=np.array(gl),
             xy_digest=np.array(digest(w.xy)), u_digest=np.array(digest(u_obs)))
    print(f"grad9: {time.time() - t0:.1f}s J={J}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c1", "c2", "block64", "grad9"]:
        if nm == "block64":
            make_block()
        elif nm == "grad9":
            make_grad()
        else:
            make(nm)
