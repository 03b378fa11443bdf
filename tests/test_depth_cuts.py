"""Host-side checks of the depth truncation of the tabulated Sommerfeld
contractions (no GPU).

Each real node of the Sommerfeld rule (Section 5.1) keeps a prefix of the
particles in depth order; each particle keeps a node range.  Pinned here
against quantities computed independently from the node table:

* the order is by increasing depth and the ranges are the hulls of the nodes
  whose prefix contains the particle;
* with the truncation off, or on the complex tanh contour, every pair is kept;
* every pair the rule drops is negligible against the largest node term of
  the shallowest pair, measured with the node's own factors: the quadrature
  weight, the 2x2 reflection R(xi) (host routine, itself pinned against the
  oracle), 1/s, the powers zeta^n of orders up to p on both ends and the
  depth decay exp(-Re s d) of both ends;
* the rule is active where the workload is deep (the kept fraction at the
  20000-particle cloud is well below one).
"""
import numpy as np
import pytest

import paper_2608_26875_amd as E
import workloads as W


def _cuts(w, **kw):
    md = E.make_media(w.host, w.substrate, w.omega)
    return md, E.sommerfeld_depth_cuts(md, w.xy, w.p, **kw)


def _branch(xi, k):
    """s = sqrt(xi^2 - k^2) with Re s >= 0 on the real axis (s = -i sqrt(k^2 -
    xi^2) inside the branch points; only |s| and Re s are used here)."""
    t = np.abs(xi)
    return np.where(t > k, np.sqrt(np.maximum(t * t - k * k, 0.0)) + 0j,
                    -1j * np.sqrt(np.maximum(k * k - t * t, 0.0)))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_order_and_ranges(name):
    w = getattr(W, f"{name}_cloud")()
    _, (perm, kcut, rng, kept) = _cuts(w)
    d = -w.xy[:, 1]
    n = len(d)
    assert sorted(perm.tolist()) == list(range(n))
    assert np.all(np.diff(d[perm]) >= 0)
    assert 0.0 < kept < 1.0
    for wv in range(2):
        kc = kcut[wv]
        assert kc.min() >= 0 and kc.max() <= n
        # first and last node keeping particle i, on a sample of 200 i
        for i in range(0, n, max(1, n // 200)):
            js = np.nonzero(kc > i)[0]
            lo, hi = rng[wv, i]
            if len(js):
                assert (lo, hi) == (js[0], js[-1] + 1), (wv, i)
            else:
                assert lo == hi == 0


def test_truncation_off_and_complex_nodes_keep_everything():
    w = W.c1_cloud()
    _, (perm, kcut, rng, kept) = _cuts(w, depth_cut=-1.0)
    assert kept == 1.0 and np.all(kcut == len(perm))
    # the tanh contour of Section 5.1 has complex nodes: no truncation
    w0 = W.c0_circles()
    _, (perm0, kcut0, _, kept0) = _cuts(w0, kind=0)
    assert kept0 == 1.0 and np.all(kcut0 == len(perm0))


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_dropped_pairs_negligible_with_node_factors(name):
    w = getattr(W, f"{name}_cloud")()
    md, (perm, kcut, rng, kept) = _cuts(w)
    nodes, _ = E.sommerfeld_nodes(md, w.xy, w.p)
    xi = nodes[:, 0]
    wt = np.abs(nodes[:, 2] + 1j * nodes[:, 3])
    assert np.all(nodes[:, 1] == 0.0)
    h = md.host
    kap = (w.omega * np.sqrt(h.rho / (h.lam + 2 * h.mu)), w.omega * np.sqrt(h.rho / h.mu))
    p = int(w.p.max())
    d = np.sort(-w.xy[:, 1])
    dmin = d[0]
    s = [_branch(xi, k) for k in kap]
    zeta = [np.abs((xi - s[i]) / kap[i]) for i in range(2)]
    vmax = [np.maximum(z, 1.0 / z) ** p for z in zeta]           # max_n |zeta^n|
    Rmax = np.array([np.abs(E.reflection(md, complex(x))).max() for x in xi])
    mid = wt * Rmax / (np.pi * np.minimum(np.abs(s[0]), np.abs(s[1])))
    with np.errstate(divide="ignore"):
        lmid = np.log(mid)                                       # -inf at zero weights
    # log of one end's factor for wave v at depth dd
    end = lambda v, dd: -s[v].real * dd + np.log(vmax[v])
    other = np.maximum(end(0, dmin), end(1, dmin))
    logP = max(np.max(end(v, dmin) + lmid + other) for v in range(2))
    worst = -np.inf
    for v in range(2):
        kc = kcut[v]
        drop = kc < len(d)
        dd = d[np.minimum(kc, len(d) - 1)]                       # shallowest dropped
        val = end(v, dd) + lmid + other
        if drop.any():
            worst = max(worst, float(np.max(val[drop])))
    print(name, "kept", kept, "worst dropped / peak = exp", worst - logP)
    assert worst - logP < np.log(1e-20)
    if name == "c2":
        assert kept < 0.5
