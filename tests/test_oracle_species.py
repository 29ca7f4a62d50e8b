"""Pins of the oracle's two-species steps (DM+Baryons mode): 3D FOF in which
baryons never link to each other (Sec. 2.1), and the assignment of baryons
to the substructure of the nearest dark-matter member in phase space
(Sec. 2.4, Eq. baryondist) -- brute force with scipy and numpy, and hand
cases.
"""
import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

GB = 21


def mk(ref, q, v=None, mass=None):
    n = q.shape[1]
    if v is None:
        v = np.zeros((3, n), np.float32)
    return ref.Particles(q.astype(np.uint32), v.astype(np.float32), mass, 1.0, 1.0, GB)


def d2_all(q):
    size = 1 << GB
    qi = q.astype(np.int64)
    d = (qi[:, :, None] - qi[:, None, :] + size // 2) % size - size // 2
    return (d * d).sum(0)


def test_fof3d_dm_brute_force(ref):
    rng = np.random.default_rng(41)
    n = 1500
    q = np.floor(rng.uniform(0.4, 0.6, (3, n)) * 2 ** GB).astype(np.int64)
    q[:, :40] = (q[:, :40] + [[0], [0], [1 << 20]]) % (1 << GB)  # some across the periodic edge
    isb = (rng.random(n) < 0.35).astype(np.uint8)
    ellx = 0.012
    lab = ref.fof3d_dm(mk(ref, q), ellx, isb)
    d2 = d2_all(q)
    ell2 = (ellx * 2 ** GB) ** 2
    assert np.abs(d2 - ell2).min() > 1
    adj = (d2 < ell2) & ~((isb[:, None] == 1) & (isb[None, :] == 1))
    np.fill_diagonal(adj, False)
    ncomp, comp = connected_components(sp.csr_matrix(adj), directed=False)
    mins = np.full(ncomp, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    np.testing.assert_array_equal(lab, mins[comp])
    # baryon pairs within ellx that only each other would join stay apart
    bb = (d2 < ell2) & (isb[:, None] == 1) & (isb[None, :] == 1)
    np.fill_diagonal(bb, False)
    assert bb.any()


def test_fof3d_dm_cases(ref):
    c = 1 << 20
    # 0-1 baryons 10 apart, nothing else near: two singletons.  Chains of dark
    # matter 2-3 and 5-6, 50 units apart, with baryon 4 between them within
    # 40 of both: the baryon joins them (dark matter links to it).
    xs = np.array([c, c + 10, c + 1000, c + 1030, c + 1065, c + 1100, c + 1130])
    q = np.stack([xs, np.full(7, c), np.full(7, c)]).astype(np.int64)
    isb = np.array([1, 1, 0, 0, 1, 0, 0], np.uint8)
    lab = ref.fof3d_dm(mk(ref, q), 40 / 2 ** GB, isb)
    assert list(lab) == [0, 1, 2, 2, 2, 2, 2]
    # with no baryons it is the plain 3D FOF
    rng = np.random.default_rng(3)
    q2 = np.floor(rng.uniform(0.45, 0.55, (3, 800)) * 2 ** GB).astype(np.int64)
    P2 = mk(ref, q2)
    np.testing.assert_array_equal(ref.fof3d_dm(P2, 0.01, np.zeros(800, np.uint8)), ref.fof3d(P2, 0.01))


def test_assign_baryons_brute_force(ref):
    rng = np.random.default_rng(43)
    n = 1200
    q = np.floor(rng.uniform(0.45, 0.55, (3, n)) * 2 ** GB).astype(np.int64)
    v = rng.normal(0, 100, (3, n)).astype(np.float32)
    isb = (rng.random(n) < 0.3).astype(np.uint8)
    sub = np.where(rng.random(n) < 0.5, rng.integers(0, 5, n) * 7, -1).astype(np.int32)
    perm = rng.permutation(n)
    h0, h1 = np.sort(perm[:500]), np.sort(perm[500:1100])
    off = np.array([0, 500, 1100], np.int32)
    mem = np.concatenate([h0, h1]).astype(np.int32)
    ellx, sv = 0.01, 120.0
    out = ref.assign_baryons(mk(ref, q, v), off, mem, isb, sub, ellx, sv)
    d2 = d2_all(q)
    vv = v.astype(np.float64)
    dv2 = ((vv[:, :, None] - vv[:, None, :]) ** 2).sum(0)
    D2 = d2 / (ellx * 2 ** GB) ** 2 + dv2 / sv ** 2
    for hm in (h0, h1):
        dm = hm[isb[hm] == 0]
        for i in hm:
            if not isb[i]:
                assert out[i] == sub[i]
                continue
            j = dm[np.lexsort((dm, D2[i, dm]))[0]]
            assert out[i] == sub[j]
    rest = np.setdiff1d(np.arange(n), mem)
    assert (out[rest] == -7).all()


def test_assign_baryons_cases(ref):
    c = 1 << 20
    # baryon 0 at the phase-space point of dark-matter 2; baryon 1 exactly
    # between dark matter 3 and 4 (equal D2): the smaller index wins
    xs = np.array([c, c + 500, c, c + 400, c + 600])
    q = np.stack([xs, np.full(5, c), np.full(5, c)]).astype(np.int64)
    v = np.stack([np.array([50.0, 0.0, 50.0, 0.0, 0.0]), np.zeros(5), np.zeros(5)]).astype(np.float32)
    isb = np.array([1, 1, 0, 0, 0], np.uint8)
    sub = np.array([-1, -1, 11, 22, 33], np.int32)
    out = ref.assign_baryons(mk(ref, q, v), np.array([0, 5], np.int32), np.arange(5, dtype=np.int32), isb, sub,
                             0.001, 100.0)
    assert list(out) == [11, 22, 11, 22, 33]
    # a host of baryons only: no dark matter to take a label from
    out2 = ref.assign_baryons(mk(ref, q, v), np.array([0, 2], np.int32), np.arange(2, dtype=np.int32), isb, sub,
                              0.001, 100.0)
    assert list(out2[:2]) == [-1, -1]
