"""Write the oracle's sampled-row references for the full-size clouds.

Calls only the CPU oracle and the seeded input generators.  For each cloud it
stores, for a few target particles, the free part T_free x, the reflected part
S T_refl x and z = S (T_free + T_refl) x of the operator at the seeded random
vector x (seed 1002), plus a checksum of x and of the centres so a test can
tell that its inputs are the same.

    python tests/golden/make_goldens.py c1 c2
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


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c1", "c2"]:
        make(nm)
