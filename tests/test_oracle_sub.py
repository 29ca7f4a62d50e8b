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
