"""Pins of the oracle's substructure linker (Sec. 2.2, Eq. linkingcriteria):
brute force over all pairs with an independent formulation (norms, speed
ratio, opening angle by arccos) on a random set kept away from every
threshold, and hand cases at the thresholds.
"""
import math

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

GB = 21


def mk(ref, q, v):
    return ref.Particles(q.astype(np.uint32), v.astype(np.float32), None, 1.0, 1.0, GB)


def test_fof_sub_brute_force(ref):
    rng = np.random.default_rng(17)
    n = 700
    q = rng.uniform(0.46, 0.54, (3, n))
    q = np.floor(q * 2 ** GB).astype(np.int64)
    # three streams with scattered directions and speeds around a local mean
    base = np.array([[150.0, 0, 0], [0, 120.0, 40.0], [-90.0, 60.0, 0]])
    which = rng.integers(0, 3, n)
    v = (base[which] + rng.normal(0, 35.0, (n, 3))).T
    vbar = rng.normal(0, 5.0, (3, n))
    L = rng.normal(3.0, 1.0, n).astype(np.float32)
    host_of = np.where(rng.random(n) < 0.1, -1, rng.integers(0, 2, n)).astype(np.int32)
    ellx_s, Vr, th = 0.012, 2.0, math.pi / 10
    P = mk(ref, q, v)
    got = ref.fof_sub(P, host_of, 2, vbar, ellx_s, L, 2.5, Vr, theta_op=th)
    # independent brute force
    v32 = v.astype(np.float32).astype(np.float64)
    u = v32 - vbar.astype(np.float32).astype(np.float64)
    s = np.linalg.norm(u, axis=0)
    d = (q[:, :, None] - q[:, None, :])
    size = 1 << GB
    d = (d + size // 2) % size - size // 2
    d2 = (d * d).sum(0)
    ell2 = (ellx_s * 2 ** GB) ** 2
    cosang = np.clip((u.T @ u) / np.outer(s, s), -1, 1)
    ang = np.arccos(cosang)
    ratio = np.maximum.outer(s, s) / np.minimum.outer(s, s)
    part = (host_of >= 0) & (L >= np.float32(2.5))
    both = part[:, None] & part[None, :] & (host_of[:, None] == host_of[None, :])
    near = both & (d2 < ell2)
    # nothing within round-off of a threshold among the candidate pairs
    assert np.abs(d2[both] - ell2).min() > 1
    assert np.abs(ratio[near] - Vr).min() > 1e-9
    assert np.abs(ang[near] - th).min() > 1e-9
    adj = near & (ratio <= Vr) & (ang <= th)
    np.fill_diagonal(adj, False)
    assert adj.sum() > 100  # links exist, and so do near pairs rejected by velocity
    assert (near & ~adj).sum() > adj.sum() // 4
    ncomp, comp = connected_components(sp.csr_matrix(adj), directed=False)
    mins = np.full(ncomp, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    exp = np.where(part, mins[comp], -1).astype(np.int32)
    np.testing.assert_array_equal(got, exp)


def test_fof_sub_threshold_cases(ref):
    c = 1 << 20
    q = np.array([[c, c + 100, c + 200, c + 300, c + 400, c + 500, c + 600, (1 << GB) - 50, 30],
                  [c] * 7 + [c, c], [c] * 7 + [c, c]], np.int64)
    v = np.array([[100.0, 200.0, 200.0001, 0.0, -100.0, 100.0, 100.0, 100.0, 150.0],
                  [0.0] * 9, [0.0] * 9])
    vbar = np.zeros((3, 9))
    L = np.full(9, 3.0, np.float32)
    host = np.zeros(9, np.int32)
    host[6] = 1
    P = mk(ref, q, v)
    ellx_s = 150 / 2 ** GB  # 150 grid units: neighbours 100 apart are near
    lab = ref.fof_sub(P, host, 2, vbar, ellx_s, L, 2.5, 2.0)
    # 0-1: speeds 100 and 200, ratio exactly 2: linked; 1-2: ratio ~1: linked,
    # so 0, 1, 2 join; 3 has zero speed; 4 runs against 3 and 5; 5-6 differ in host
    assert list(lab[:7]) == [0, 0, 0, 3, 4, 5, 6]
    # 7 and 8 straddle the periodic edge (80 units apart) with equal directions
    assert lab[7] == lab[8] == 7
    # a speed ratio just above 2 breaks the link
    v2 = v.copy()
    v2[0, 1] = 200.0001
    lab2 = ref.fof_sub(mk(ref, q, v2), host, 2, vbar, ellx_s, L, 2.5, 2.0)
    assert lab2[0] == 0 and lab2[1] == 1 and lab2[2] == 1
    # below the L threshold: not a participant
    L2 = L.copy()
    L2[1] = 2.4999
    lab3 = ref.fof_sub(P, host, 2, vbar, ellx_s, L2, 2.5, 2.0)
    assert lab3[1] == -1 and lab3[0] == 0 and lab3[2] == 2
    # the opening angle: 17 degrees links, 19 does not (against 18)
    for deg, linked in ((17.0, True), (19.0, False)):
        a = math.radians(deg)
        qq = np.array([[c, c + 100], [c, c], [c, c]], np.int64)
        vv = np.array([[100.0, 100.0 * math.cos(a)], [0.0, 100.0 * math.sin(a)], [0.0, 0.0]])
        ll = ref.fof_sub(mk(ref, qq, vv), np.zeros(2, np.int32), 1, np.zeros((3, 2)), ellx_s,
                         np.full(2, 3.0, np.float32), 2.5, 2.0)
        assert (ll[1] == 0) == linked


def relaxed_adjacency(q, v, vbar, host, L, Lth, ell, Vr, theta):
    """All-pairs relaxed links by numpy (norms, speed ratio, arccos angle)."""
    n = q.shape[1]
    size = 1 << GB
    d = (q[:, :, None] - q[:, None, :] + size // 2) % size - size // 2
    d2 = (d * d).sum(0)
    u = v.astype(np.float32).astype(np.float64) - vbar.astype(np.float32).astype(np.float64)
    s = np.linalg.norm(u, axis=0)
    with np.errstate(divide="ignore", invalid="ignore"):
        cosang = np.clip((u.T @ u) / np.outer(s, s), -1, 1)
        ratio = np.maximum.outer(s, s) / np.minimum.outer(s, s)
    part = (host >= 0) & (L >= np.float32(Lth))
    adj = (part[:, None] & part[None, :] & (host[:, None] == host[None, :]) & (d2 < (ell * 2 ** GB) ** 2)
           & (np.outer(s, s) > 0) & (ratio <= Vr) & (np.arccos(cosang) <= theta))
    np.fill_diagonal(adj, False)
    return adj, d2, ratio, np.arccos(cosang)


def grow_brute(adj, label1, n_min, f_merge):
    n = len(label1)
    sizes = np.bincount(label1[label1 >= 0], minlength=n)
    tag = np.where((label1 >= 0) & (sizes[np.maximum(label1, 0)] >= n_min), label1, -1)
    rounds = 0
    while True:
        new = tag.copy()
        for u in np.nonzero(tag < 0)[0]:
            t = tag[adj[u]]
            t = t[t >= 0]
            if len(t):
                new[u] = t.min()
        if (new == tag).all():
            break
        tag, rounds = new, rounds + 1
    ii, jj = np.nonzero(np.triu(adj, 1))
    a, b = tag[ii], tag[jj]
    keep = (a >= 0) & (b >= 0) & (a != b)
    pairs = {}
    for x, y in zip(np.minimum(a[keep], b[keep]), np.maximum(a[keep], b[keep])):
        pairs[(x, y)] = pairs.get((x, y), 0) + 1
    parent = {}

    def find(x):
        while parent.get(x, x) != x:
            x = parent[x]
        return x
    for (x, y), c in pairs.items():
        if c > f_merge * sizes[x] or c > f_merge * sizes[y]:
            rx, ry = find(x), find(y)
            if rx != ry:
                parent[max(rx, ry)] = min(rx, ry)
    root = np.array([find(t) if t >= 0 else -1 for t in tag])
    out = np.full(n, -1, np.int64)
    for r in np.unique(root[root >= 0]):
        m = root == r
        out[m] = np.nonzero(m)[0].min()
    return out, rounds, pairs


def test_sub_grow_brute_force(ref):
    rng = np.random.default_rng(29)
    n = 600
    # a few compact clumps with coherent velocities inside a sparser cloud
    # three pairs of clumps: the two clumps of a pair move alike and sit
    # close enough for relaxed links between their outskirts
    c3 = rng.uniform(0.45, 0.55, (3, 3))
    centres = np.concatenate([c3, c3 + [0.011, 0.0, 0.0]])
    which = rng.integers(0, 6, n)
    x = centres[which] + rng.normal(0, 0.003, (n, 3))
    q = np.floor(x.T * 2 ** GB).astype(np.int64)
    vdir = np.tile(rng.normal(0, 1, (3, 3)), (2, 1))
    v = (vdir[which] * 100 + rng.normal(0, 15, (n, 3))).T
    vbar = np.zeros((3, n))
    L = rng.normal(3.0, 0.8, n).astype(np.float32)
    host = np.where(rng.random(n) < 0.05, -1, 0).astype(np.int32)
    P = mk(ref, q, v)
    ellxs, th, Vr = 0.003, math.pi / 10, 2.0
    lab1 = ref.fof_sub(P, host, 1, vbar, ellxs, L, 2.5, Vr, theta_op=th)
    assert (np.unique(lab1[lab1 >= 0], return_counts=True)[1] >= 20).sum() >= 3
    ngroups = {}
    for f_merge in (0.0, 0.25, 100.0):
        got, nr = ref.sub_grow(P, host, 1, vbar, L, lab1, ellxs, 2.5, gamma_L=1.2, gamma_x=2.0, Vr=Vr, gamma_V=1.0,
                               theta_op=th, gamma_theta=1.3, f_merge=f_merge, n_min=20)
        adj, d2, ratio, ang = relaxed_adjacency(q, v, vbar, host, L, 2.5 / 1.2, 2 * ellxs, Vr, 1.3 * th)
        exp, rounds, pairs = grow_brute(adj, lab1, 20, f_merge)
        np.testing.assert_array_equal(got, exp)
        assert nr == rounds and rounds >= 1
        ngroups[f_merge] = len(np.unique(got[got >= 0]))
    # groups touch through relaxed links; a large f_merge keeps them apart
    assert len(pairs) >= 1 and ngroups[100.0] > ngroups[0.25]


def test_sub_grow_chain_and_join(ref):
    c = 1 << 20
    # group A: 20 members 10 units apart; a chain of 5 particles 60 units
    # apart running on from it; group B: 20 members further on
    xa = c + 10 * np.arange(20)
    xchain = xa[-1] + 60 * np.arange(1, 6)
    xb = xchain[-1] + 60 + 10 * np.arange(20)
    xs = np.r_[xa, xchain, xb]
    n = len(xs)
    q = np.stack([xs, np.full(n, c), np.full(n, c)]).astype(np.int64)
    v = np.stack([np.full(n, 100.0), np.zeros(n), np.zeros(n)])
    vbar = np.zeros((3, n))
    L = np.full(n, 3.0, np.float32)
    host = np.zeros(n, np.int32)
    P = mk(ref, q, v)
    ell = 40 / 2 ** GB  # first stage: 40 units; relaxed (x2): 80 units
    lab1 = ref.fof_sub(P, host, 1, vbar, ell, L, 2.5, 2.0)
    assert lab1[0] == 0 and lab1[44] == 25 and len(set(lab1[20:25])) == 5
    # growth: the chain joins A from one end and B from the other; the link
    # between the chain's two halves then connects the groups by one link,
    # below 0.25 x 20: they stay apart
    got, nr = ref.sub_grow(P, host, 1, vbar, L, lab1, ell, 2.5, f_merge=0.25)
    assert nr == 3
    assert (got[:23] == 0).all() and (got[23:] == 23).all()
    # with f_merge = 0 a single link joins them
    got0, _ = ref.sub_grow(P, host, 1, vbar, L, lab1, ell, 2.5, f_merge=0.0)
    assert (got0 == 0).all()
