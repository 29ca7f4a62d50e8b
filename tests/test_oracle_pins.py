"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute force
on tiny inputs, closed forms, library routines (scipy), limits and invariants.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components
from scipy.stats import multivariate_normal

from paper_1902_01010_amd import synth

GB = 21


def particles(ref, q, v=None, mass=None, mass_value=1.0, box=1.0, gb=GB):
    return ref.Particles(q, v, mass, mass_value, box, gb)


def minimage(d, gb=GB):
    size = 1 << gb
    return ((d + size // 2) % size) - size // 2


def brute_labels(adj):
    n = adj.shape[0]
    ncomp, comp = connected_components(sp.csr_matrix(adj), directed=False)
    mins = np.full(ncomp, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].astype(np.int32)


def pair_d2(q, gb=GB):
    qi = q.astype(np.int64)
    d = minimage(qi[:, :, None] - qi[:, None, :], gb)
    return (d * d).sum(0)


# --------------------------------------------------------------------------- quantise
def test_quantize_closed_form(ref):
    box = 1.0
    k = np.array([0, 1, 12345, (1 << GB) - 1], np.int64)
    x = (k / float(1 << GB) * box).astype(np.float32)  # exact grid points
    X = np.stack([x, x, x])
    q = ref.quantize(X, box, GB)
    assert (q[0] == k).all()
    # the box edge and negative coordinates wrap periodically
    q2 = ref.quantize(np.array([[1.0, -0.25], [0.5, 0.0], [0.75, 0.999999]], np.float32), 1.0, GB)
    assert q2[0, 0] == 0 and q2[0, 1] == 3 << (GB - 2)
    assert q2[1, 0] == 1 << (GB - 1)
    assert (q2 < (1 << GB)).all()


def test_quantize_random_invariant(ref):
    rng = np.random.default_rng(0)
    box = 100.0
    x = (rng.random((3, 5000)) * box).astype(np.float32)
    q = ref.quantize(x, box, GB)
    lo = q.astype(np.float64) * box / (1 << GB)
    hi = (q.astype(np.float64) + 1) * box / (1 << GB)
    xd = x.astype(np.float64)
    assert ((lo <= xd) & (xd < hi)).all()


# --------------------------------------------------------------------------- 3D FOF
@pytest.mark.parametrize("seed,n,ell", [(1, 300, 0.08), (2, 1500, 0.03), (3, 2000, 0.05)])
def test_fof3d_brute_force(ref, seed, n, ell):
    rng = np.random.default_rng(seed)
    # clumpy points so that components of many sizes appear, some across the box edge
    centres = rng.random((3, 12))
    x = centres[:, rng.integers(0, 12, n)] + rng.normal(0, 0.04, (3, n))
    x = np.mod(x, 1.0).astype(np.float32)
    q = ref.quantize(x, 1.0, GB)
    P = particles(ref, q)
    lab = ref.fof3d(P, ell)
    ell2 = (ell * (1 << GB)) ** 2
    adj = pair_d2(q) < ell2
    np.fill_diagonal(adj, False)
    assert (lab == brute_labels(adj)).all()


def test_fof3d_lattice_strict(ref):
    # a cubic lattice with spacing s: linking length just above s joins all,
    # exactly s joins nothing (strict inequality of the link predicate)
    s = 1 << 12
    g = np.arange(8) * s + 1000
    qx, qy, qz = np.meshgrid(g, g, g, indexing="ij")
    q = np.stack([qx.ravel(), qy.ravel(), qz.ravel()]).astype(np.uint32)
    P = particles(ref, q)
    unit = 1.0 / (1 << GB)
    assert (ref.fof3d(P, (s + 0.5) * unit) == 0).all()
    assert (ref.fof3d(P, s * unit) == np.arange(q.shape[1])).all()


def test_fof3d_periodic_pair(ref):
    size = 1 << GB
    q = np.array([[5, size - 5, 1000], [7, 7, 7], [9, 9, 9]], np.uint32)
    P = particles(ref, q)
    lab = ref.fof3d(P, 11.0 / size)
    assert list(lab) == [0, 0, 2]


def test_fof3d_rejects_half_box(ref):
    q = np.zeros((3, 4), np.uint32)
    with pytest.raises(RuntimeError):
        ref.fof3d(particles(ref, q), 0.5)


# --------------------------------------------------------------------------- groups
def test_groups_order_and_members(ref):
    rng = np.random.default_rng(5)
    lab = rng.integers(0, 40, 3000)
    # relabel to min index of each class
    mins = np.full(40, 10 ** 9)
    np.minimum.at(mins, lab, np.arange(3000))
    lab = mins[lab].astype(np.int32)
    lab[rng.random(3000) < 0.05] = -1
    ng, gof, off, mem = ref.groups(lab, 60)
    uniq, cnt = np.unique(lab[lab >= 0], return_counts=True)
    keep = cnt >= 60
    first = np.array([np.nonzero(lab == u)[0][0] for u in uniq])
    exp = sorted(zip(-cnt[keep], first[keep], uniq[keep]))
    assert ng == len(exp)
    for g, (negc, first_member, root) in enumerate(exp):
        m = mem[off[g]:off[g + 1]]
        assert len(m) == -negc and m[0] == first_member
        assert (np.diff(m) > 0).all() and (lab[m] == root).all()
        assert (gof[m] == g).all()
    assert (gof >= 0).sum() == off[-1]


# --------------------------------------------------------------------------- cells
def test_entropy_closed_forms(ref):
    assert ref.entropy(np.ones(16)) == pytest.approx(1.0, abs=1e-15)
    assert ref.entropy(np.r_[5.0, np.zeros(15)]) == 0.0
    h = np.r_[1.0, 1.0, np.zeros(14)]
    assert ref.entropy(h) == pytest.approx(math.log(2) / math.log(16), rel=1e-15)


def _host_workload(seed, n):
    w = synth.isolated_halo(seed=seed, n_host=n, n_sub=2, sub_range=(n // 10, n // 5))
    return w


def _make_P(ref, w):
    q = ref.quantize(w.x, w.box, w.grid_bits)
    return particles(ref, q, w.v, w.mass, w.mass_value, w.box, w.grid_bits)


@pytest.mark.parametrize("seed,n", [(11, 3000), (12, 12000)])
def test_cells_structure_and_moments(ref, seed, n):
    w = _host_workload(seed, n)
    P = _make_P(ref, w)
    mem = np.arange(P.n, dtype=np.int32)
    off = np.array([0, P.n], np.int32)
    out = ref.cell_moments(P, off, mem)
    cells = out["cells"]
    NH = P.n
    ncell = min(max(math.ceil(0.01 * NH), 100), NH // 8)
    sizes = cells[:, 1]
    assert sizes.sum() == NH
    assert (sizes <= ncell).all() and (sizes >= (ncell + 1) // 2).all()
    # leaves tile the root box: volumes add up and integer boxes are disjoint
    lo, hi = cells[:, 15:18], cells[:, 18:21]
    vol = np.prod(hi - lo + 1, axis=1)
    unit = w.box / (1 << GB)
    u = np.empty((3, NH))
    for d in range(3):
        ref0 = P.q[d, 0].astype(np.int64)
        u[d] = ref0 + minimage(P.q[d].astype(np.int64) - ref0)
    root = np.prod(u.max(1) - u.min(1) + 1)
    assert vol.sum() == pytest.approx(root, rel=1e-12)
    # moments (Eqs. meanpos, meanvel, meandispvel) against numpy per cell
    cof = out["cell_of"]
    for c in range(0, len(cells), max(1, len(cells) // 25)):
        idx = np.nonzero(cof == c)[0]
        assert len(idx) == sizes[c]
        m = np.ones(len(idx))
        xb = np.average(u[:, idx] * unit, axis=1, weights=m)
        vb = np.average(w.v[:, idx].astype(np.float64), axis=1, weights=m)
        cov = np.cov(w.v[:, idx].astype(np.float64), aweights=m, bias=True)
        np.testing.assert_allclose(cells[c, 3:6], xb, rtol=1e-12)
        np.testing.assert_allclose(cells[c, 6:9], vb, rtol=1e-10, atol=1e-9)
        got = cells[c, 9:15]
        expv = [cov[0, 0], cov[1, 1], cov[2, 2], cov[0, 1], cov[0, 2], cov[1, 2]]
        np.testing.assert_allclose(got, expv, rtol=1e-9, atol=1e-6)
        assert cells[c, 2] == pytest.approx(len(idx) * w.mass_value)
    # face neighbours touch the face they were probed from
    for c in range(len(cells)):
        for f in range(6):
            nb = int(cells[c, 21 + f])
            if nb < 0:
                continue
            d = f // 2
            if f % 2 == 0:
                assert cells[nb, 18 + d] == cells[c, 15 + d] - 1
            else:
                assert cells[nb, 15 + d] == cells[c, 18 + d] + 1
            assert nb != c
    # interpolated tensors are convex combinations: inside the cell-value hull, SPD
    vbar, sig = out["vbar"], out["sigma"]
    for k in range(0, NH, 97):
        c = cof[k]
        nbrs = [c] + [int(x) for x in cells[c, 21:27] if x >= 0]
        vals = cells[nbrs, 6:9]
        assert (vbar[:, k] >= vals.min(0) - 1e-3).all() and (vbar[:, k] <= vals.max(0) + 1e-3).all()
        S = np.array([[sig[0, k], sig[3, k], sig[4, k]], [sig[3, k], sig[1, k], sig[5, k]],
                      [sig[4, k], sig[5, k], sig[2, k]]], np.float64)
        assert np.linalg.eigvalsh(S).min() > 0
        assert out["rho_cell"][k] == pytest.approx(cells[c, 2] / cells[c, 27], rel=1e-6)


def test_cells_idw_weights_favour_nearest(ref):
    # Eq. cellinterp weights are inverse distances: a particle next to its own
    # cell's centre of mass takes nearly that cell's value.
    w = _host_workload(13, 6000)
    P = _make_P(ref, w)
    off = np.array([0, P.n], np.int32)
    out = ref.cell_moments(P, off, np.arange(P.n, dtype=np.int32))
    cells = out["cells"]
    unit = w.box / (1 << GB)
    u = np.empty((3, P.n))
    for d in range(3):
        r0 = P.q[d, 0].astype(np.int64)
        u[d] = (r0 + minimage(P.q[d].astype(np.int64) - r0)) * unit
    best = None
    for k in range(P.n):
        c = out["cell_of"][k]
        dist = np.linalg.norm(u[:, k] - cells[c, 3:6])
        others = [int(x) for x in cells[c, 21:27] if x >= 0]
        far = min(np.linalg.norm(u[:, k] - cells[o, 3:6]) for o in others) if others else np.inf
        ratio = dist / far
        if best is None or ratio < best[0]:
            best = (ratio, k, c, others)
    ratio, k, c, others = best
    assert ratio < 0.05
    # own weight >= (1/0.05) / (1/0.05 + 6): at most 23% of the way to the others
    own = cells[c, 6:9]
    spread = max(np.abs(cells[o, 6:9] - own).max() for o in others)
    assert np.abs(out["vbar"][:, k] - own).max() < 0.25 * spread


@pytest.mark.parametrize("rule,expect_y", [(0, True), (1, False)])
def test_cells_split_rule_picks_structured_dimension(ref, rule, expect_y):
    # two clumps separated along y, uniform along x and z: the mass histogram
    # of y has the lowest entropy, so the minimum-entropy rule splits y first
    rng = np.random.default_rng(3)
    n = 4000
    x = np.empty((3, n))
    x[0] = 0.3 + 0.4 * rng.random(n)
    x[2] = 0.3 + 0.4 * rng.random(n)
    x[1] = np.where(rng.random(n) < 0.5, 0.35, 0.65) + rng.normal(0, 0.01, n)
    q = ref.quantize(x.astype(np.float32), 1.0, GB)
    v = rng.normal(0, 10, (3, n)).astype(np.float32)
    P = particles(ref, q, v)
    out = ref.cell_moments(P, np.array([0, n], np.int32), np.arange(n, dtype=np.int32),
                           split_rule=rule)
    cells = out["cells"]
    lo, hi = cells[:, 15:18], cells[:, 18:21]
    # is there a y plane that no cell straddles, at the median of y?
    ys = np.sort(np.r_[lo[:, 1], hi[:, 1] + 1])
    def separates(d):
        for t in np.unique(np.r_[lo[:, d], hi[:, d] + 1]):
            if t <= lo[:, d].min() or t > hi[:, d].max():
                continue
            if ((hi[:, d] < t) | (lo[:, d] >= t)).all():
                return True
        return False
    del ys
    assert separates(1) == expect_y


# --------------------------------------------------------------------------- R
def _knn_case(rng, nh, ext=0.01):
    x = 0.5 + (rng.random((3, nh)) - 0.5) * ext
    v = rng.normal(0, 100, (3, nh)).astype(np.float32)
    return x.astype(np.float32), v


def test_knn_sets_brute_force(ref):
    rng = np.random.default_rng(21)
    n1, n2 = 120, 300
    x1, v1 = _knn_case(rng, n1)
    x2, v2 = _knn_case(rng, n2)
    x = np.concatenate([x1, x2], 1)
    v = np.concatenate([v1, v2], 1)
    # coincident points create exact distance ties broken by index
    x[:, 5] = x[:, 9]
    perm = rng.permutation(n1 + n2)
    x, v = x[:, perm], v[:, perm]
    hostid = np.r_[np.zeros(n1, int), np.ones(n2, int)][perm]
    q = ref.quantize(x, 1.0, GB)
    P = particles(ref, q, v)
    mem = np.r_[np.nonzero(hostid == 0)[0], np.nonzero(hostid == 1)[0]].astype(np.int32)
    off = np.array([0, n1, n1 + n2], np.int32)
    vbar = np.zeros((3, P.n), np.float32)
    sig = np.zeros((6, P.n), np.float32)
    sig[:3] = 100.0 ** 2
    n_se, n_v = 16, 5
    out = ref.local_vdensity(P, off, mem, vbar, sig, n_se, n_v, want_sets=True)
    D2 = pair_d2(q)
    vd = v.astype(np.float64)
    for row, k in enumerate(mem):
        same = np.nonzero(hostid == hostid[k])[0]
        order = np.lexsort((same, D2[k, same]))
        S = same[order[:n_se]]
        assert (out["nbr_s"][row] == S).all()
        dv2 = ((vd[:, S] - vd[:, [k]]) ** 2).sum(0)
        Vs = S[np.lexsort((S, dv2))[:n_v]]
        assert (out["nbr_v"][row] == Vs).all()
        assert Vs[0] == k  # self is always its own nearest velocity neighbour


def test_fbg_matches_scipy(ref):
    rng = np.random.default_rng(22)
    nh = 200
    x, v = _knn_case(rng, nh)
    q = ref.quantize(x, 1.0, GB)
    P = particles(ref, q, v)
    vbar = rng.normal(0, 30, (3, nh)).astype(np.float32)
    A = rng.normal(0, 60, (nh, 3, 3))
    Sm = A @ A.transpose(0, 2, 1) + np.eye(3) * 100.0
    sig = np.stack([Sm[:, 0, 0], Sm[:, 1, 1], Sm[:, 2, 2], Sm[:, 0, 1], Sm[:, 0, 2], Sm[:, 1, 2]])
    sig = sig.astype(np.float32)
    out = ref.local_vdensity(P, np.array([0, nh], np.int32), np.arange(nh, dtype=np.int32),
                             vbar, sig, 32, 8)
    for k in range(nh):
        S = np.array([[sig[0, k], sig[3, k], sig[4, k]], [sig[3, k], sig[1, k], sig[5, k]],
                      [sig[4, k], sig[5, k], sig[2, k]]], np.float64)
        e = multivariate_normal.logpdf(v[:, k].astype(np.float64), mean=vbar[:, k].astype(np.float64), cov=S)
        assert out["lnfbg"][k] == pytest.approx(e, rel=1e-10, abs=1e-10)
    np.testing.assert_allclose(out["R"], (out["lnfl"] - out["lnfbg"]).astype(np.float32), rtol=1e-6)


def test_fl_closed_form(ref):
    # four host members; velocities 0, 1, 2, 3 km/s along x.  For particle 0
    # with N_se = 4 and N_v = 3: V = {0, 1, 2}, h = 2, and the Epanechnikov
    # estimate is m (15/8pi) [1 + (1 - 1/4) + 0] / (h^3 * 4m).
    q = np.array([[100, 110, 120, 130], [100] * 4, [100] * 4], np.uint32)
    v = np.array([[0.0, 1.0, 2.0, 3.0], [0] * 4, [0] * 4], np.float32)
    P = particles(ref, q, v, mass_value=2.5)
    vbar = np.zeros((3, 4), np.float32)
    sig = np.zeros((6, 4), np.float32)
    sig[:3] = 1.0
    out = ref.local_vdensity(P, np.array([0, 4], np.int32), np.arange(4, dtype=np.int32),
                             vbar, sig, 4, 3, subset=np.array([0], np.int32))
    expect = (15.0 / (8 * math.pi)) * 1.75 / (8.0 * 4.0)
    assert out["lnfl"][0] == pytest.approx(math.log(expect), rel=1e-13)
    # identical velocities give an infinite density: R = +inf
    v2 = np.zeros((3, 4), np.float32)
    P2 = particles(ref, q, v2)
    out2 = ref.local_vdensity(P2, np.array([0, 4], np.int32), np.arange(4, dtype=np.int32),
                              vbar, sig, 4, 3)
    assert np.isposinf(out2["R"]).all()


def _mc_R(rng, n_samples, n_se, n_v, sigma):
    """Independent Monte Carlo of the ratio for iid Gaussian velocities with the
    true background: density estimate from the N_v nearest of N_se draws."""
    vs = rng.normal(0, sigma, (n_samples, n_se, 3))
    dv2 = ((vs - vs[:, :1, :]) ** 2).sum(-1)
    dv2.sort(axis=1)
    V = dv2[:, :n_v]
    h2 = V[:, -1]
    kern = (15 / (8 * np.pi)) * (1 - V / h2[:, None])
    f_l = kern.sum(1) / (h2 ** 1.5 * n_se)
    lnfbg = -0.5 * (vs[:, 0] ** 2).sum(1) / sigma ** 2 - 1.5 * np.log(2 * np.pi * sigma ** 2)
    return np.log(f_l) - lnfbg


def test_maxwellian_R_statistics(ref):
    # A smooth Maxwellian background has no velocity substructure: the ratio
    # sits near zero, with few particles above the outlier threshold 2.
    w = synth.maxwellian_host(seed=7, n=12000, sigma=150.0)
    P = _make_P(ref, w)
    off = np.array([0, P.n], np.int32)
    mem = np.arange(P.n, dtype=np.int32)
    cm = ref.cell_moments(P, off, mem)
    out = ref.local_vdensity(P, off, mem, cm["vbar"], cm["sigma"], 32, 8)
    R = out["R"]
    assert np.isfinite(R).all()
    mc = _mc_R(np.random.default_rng(1), 40000, 32, 8, 150.0)
    assert 0.0 < R.mean() < 0.6
    assert abs(R.mean() - mc.mean()) < 0.1
    assert abs(np.median(R) - np.median(mc)) < 0.1
    frac = (R >= 2).mean()
    assert 0.002 < frac < 0.05
    assert abs(frac - (mc >= 2).mean()) < 0.015


def test_planted_subhalo_outliers(ref):
    # physics sanity: cold planted subhalos are far more often outliers than the host
    w = synth.isolated_halo(seed=4, n_host=20000, n_sub=3, sub_range=(800, 1500))
    P = _make_P(ref, w)
    off = np.array([0, P.n], np.int32)
    mem = np.arange(P.n, dtype=np.int32)
    cm = ref.cell_moments(P, off, mem)
    R = ref.local_vdensity(P, off, mem, cm["vbar"], cm["sigma"], 32, 8)["R"]
    vd = np.abs(w.v.astype(np.float64))
    # subhalo particles are the cold ones: dispersion 10-30 km/s around a bulk;
    # identify them through the generator order-independent flag below
    n_sub = sum(s["n"] for s in w.meta["subhalos"])
    assert n_sub > 0 and vd.shape[1] == P.n
    frac_all = (R >= 2).mean()
    assert frac_all > 0.03  # ~n_sub / N of the particles are substructure


# --------------------------------------------------------------------------- 6D FOF
def test_host_ellv_matches_numpy(ref):
    rng = np.random.default_rng(31)
    n = 500
    x = (0.5 + rng.random((3, n)) * 0.01).astype(np.float32)
    v = rng.normal(0, [[50], [80], [120]], (3, n)).astype(np.float32)
    m = rng.uniform(0.5, 2.0, n).astype(np.float32)
    q = ref.quantize(x, 1.0, GB)
    P = particles(ref, q, v, mass=m)
    mem = np.arange(n, dtype=np.int32)
    out = ref.host_ellv(P, np.array([0, 200, n], np.int32), mem, 1.25)
    for h, (a, b) in enumerate([(0, 200), (200, n)]):
        cov = np.cov(v[:, a:b].astype(np.float64), aweights=m[a:b].astype(np.float64), bias=True)
        assert out[h] == pytest.approx(1.25 * np.linalg.det(cov) ** (1 / 6), rel=1e-10)


def test_fof6d_brute_force(ref):
    rng = np.random.default_rng(41)
    n = 1200
    x = (0.5 + rng.normal(0, 0.01, (3, n))).astype(np.float32)
    v = np.where(rng.random(n) < 0.5, 0.0, 300.0)[None, :] + rng.normal(0, 40, (3, n))
    v = v.astype(np.float32)
    q = ref.quantize(x, 1.0, GB)
    P = particles(ref, q, v)
    host_of = np.where(rng.random(n) < 0.8, 0, 1).astype(np.int32)
    host_of[rng.random(n) < 0.1] = -1
    R = rng.normal(1.5, 1.0, n).astype(np.float32)
    ellv = np.array([60.0, 90.0])
    ellxs = 0.004
    lab = ref.fof6d(P, host_of, ellv, ellxs, R, 2.0)
    part = (host_of >= 0) & (R >= 2.0)
    ell2 = (ellxs * (1 << GB)) ** 2
    D2 = pair_d2(q).astype(np.float64)
    vd = v.astype(np.float64)
    dv2 = ((vd[:, :, None] - vd[:, None, :]) ** 2).sum(0)
    ev = ellv[np.maximum(host_of, 0)]
    adj = (D2 / ell2 + dv2 / (ev[:, None] ** 2) < 1.0) & part[:, None] & part[None, :]
    adj &= host_of[:, None] == host_of[None, :]
    np.fill_diagonal(adj, False)
    exp = brute_labels(adj)
    exp[~part] = -1
    assert (lab == exp).all()


@pytest.mark.parametrize("dv,split", [(50.0, False), (100.0, True), (150.0, True)])
def test_fof6d_cold_clumps_split_at_ellv(ref, dv, split):
    # two cold clumps at one place, bulk velocities dv apart: they link iff dv < ellv
    rng = np.random.default_rng(42)
    n = 60
    x = (0.5 + rng.normal(0, 1e-4, (3, n))).astype(np.float32)
    v = np.zeros((3, n), np.float32)
    v[0, n // 2:] = dv
    q = ref.quantize(x, 1.0, GB)
    P = particles(ref, q, v)
    lab = ref.fof6d(P, np.zeros(n, np.int32), np.array([100.0]), 0.01, None)
    assert (len(np.unique(lab)) == 2) == split


# --------------------------------------------------------------------------- unbinding
G = synth.G_GRAV


def test_unbind_two_body_closed_form(ref):
    # two equal masses at separation r, moving apart at relative speed u in
    # their centre-of-mass frame: phi = -G m / sqrt(r^2 + eps^2) for both, and
    # with T = m u^2 / 8, W = m phi the pair is bound iff u^2 < -8 phi / beta_E.
    box = 1.0
    unit = box / (1 << GB)
    q = np.array([[1000, 1000 + 4096], [50, 50], [70, 70]], np.uint32)
    r = 4096 * unit
    m, eps = 1e10, 0.001
    phi_exact = -G * m / math.sqrt(r * r + eps * eps)
    u_crit = math.sqrt(-8 * phi_exact / 0.95)
    for u, bound in [(0.99 * u_crit, 1), (1.01 * u_crit, 0)]:
        v = np.array([[u / 2, -u / 2], [0, 0], [0, 0]], np.float32)
        P = particles(ref, q, v, mass_value=m, box=box)
        out = ref.unbind(P, np.array([0, 2]), np.array([0, 1]), G, eps, n_min=2, n_ref_min=1,
                         frame_type=0)
        assert out["phi"][0] == pytest.approx(phi_exact, rel=1e-14)
        assert out["phi"][1] == pytest.approx(phi_exact, rel=1e-14)
        assert out["bound"].tolist() == [bound, bound]


def test_unbind_plummer_potential(ref):
    a = 0.01
    w = synth.plummer_sphere(seed=8, n=6000, a=a, sigma=1.0, m=1e10)
    P = _make_P(ref, w)
    out = ref.unbind(P, np.array([0, P.n]), np.arange(P.n), G, eps=1e-5, n_min=20)
    M = P.n * w.mass_value / 0.999
    xd = w.x.astype(np.float64) - 0.5
    r = np.linalg.norm(xd, axis=0)
    inner = r < 3 * a
    expect = -G * M / np.sqrt(r ** 2 + a ** 2)
    rel = np.abs(out["phi"][inner] / expect[inner] - 1)
    assert np.median(rel) < 0.02
    assert out["bound"].all()  # nearly cold sphere: everything bound
    assert out["iters"][0] == 1


def test_unbind_removes_contaminants(ref):
    w = synth.unbind_groups(seed=3, n_groups=6, n_max=3000)
    P = _make_P(ref, w)
    off, mem = w.groups
    out = ref.unbind(P, off, mem, w.params["G"], w.params["eps"])
    con = w.meta["is_contaminant"]
    assert (out["bound"][con] == 0).all()
    assert out["bound"][~con].mean() > 0.5
    assert (out["iters"] >= 2).all()


def test_unbind_dissolves_hot_group(ref):
    rng = np.random.default_rng(9)
    n = 50
    x = (0.5 + rng.normal(0, 0.001, (3, n))).astype(np.float32)
    v = rng.normal(0, 5000.0, (3, n)).astype(np.float32)
    P = particles(ref, ref.quantize(x, 1.0, GB), v, mass_value=1e6)
    out = ref.unbind(P, np.array([0, n]), np.arange(n), G, 1e-4)
    assert out["bound"].sum() == 0 and out["iters"][0] == 1


def test_unbind_not_converged_status(ref):
    w = synth.unbind_groups(seed=3, n_groups=2, n_max=500)
    P = _make_P(ref, w)
    with pytest.raises(RuntimeError, match="converge"):
        ref.unbind(P, w.groups[0], w.groups[1], w.params["G"], w.params["eps"], max_iter=1)
