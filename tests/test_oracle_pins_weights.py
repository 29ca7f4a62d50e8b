"""Pins of the oracle's weights: the inverse-distance weights of Eq. cellinterp,
the mass weighting of Eqs. meanpos-meandispvel and of the entropy histogram
(Sec. 2.2), and the velocity frame of the unbinding (the footnote to Eq.
binding: the frame of the members around the potential minimum).

Each case is built so that its answer follows from the construction by hand
(exact fractions, or decisions with wide margins), and so that the plausible
mistakes -- 1/r^2 or unnormalised weights, count instead of mass weights,
the centre-of-mass frame, a wrong size of the frame set -- give a different
answer.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_1902_01010_amd import synth

GB = 21
G = synth.G_GRAV


# --------------------------------------------------------------------------- Eq. cellinterp
# Sixteen particles on a line along x (y and z shared), four cells of four.
# Only x varies, so every split is along x at the median; the cells are the
# four runs below and each cell's face neighbours are the cells beside it
# along x (probes in y and z leave the degenerate root box).
X0 = 1000
XS = [0, 10, 20, 30,          # cell 0
      100, 110, 120, 130,     # cell 1 (first member three times as heavy)
      200, 215, 215, 230,     # cell 2 (two members exactly at its centre of mass)
      300, 310, 320, 330]     # cell 3
MS = [1, 1, 1, 1, 3, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1]
VX_CELL = [0, 60, 120, 0]          # every member of cell c moves at VX_CELL[c] along x
SY_CELL = [10, 20, 30, 40]         # vy = +-s_c around a zero mass-weighted mean


def _line_case(ref):
    n = len(XS)
    q = np.empty((3, n), np.uint32)
    q[0] = [X0 + x for x in XS]
    q[1] = 5000
    q[2] = 7000
    v = np.zeros((3, n), np.float32)
    for k in range(n):
        c = k // 4
        v[0, k] = VX_CELL[c]
    # vy: mass-weighted mean zero, dispersion s_c^2 in every cell
    signs = [1, -1, 1, -1]
    for c in range(4):
        for j in range(4):
            k = 4 * c + j
            v[1, k] = SY_CELL[c] * (signs[j] if c != 1 else (1 if j == 0 else -1))
    mass = np.array(MS, np.float32)
    P = ref.Particles(q, v, mass, 1.0, 1.0, GB)
    out = ref.cell_moments(P, np.array([0, n], np.int32), np.arange(n, dtype=np.int32),
                           f_cell=0.25, ncell_floor=1, ncell_div=4)
    return out


def _com(c):
    mem = range(4 * c, 4 * c + 4)
    return Fr(sum(MS[k] * XS[k] for k in mem), sum(MS[k] for k in mem))


def test_cellinterp_hand_case_inverse_distance(ref):
    out = _line_case(ref)
    cells = out["cells"]
    unit = 1.0 / (1 << GB)
    assert cells.shape[0] == 4
    assert out["cell_of"].tolist() == [k // 4 for k in range(16)]
    # Eq. meanpos with the heavy member: cell 1's centre is 110, not 115
    assert _com(1) == 110 and _com(2) == 215
    for c in range(4):
        assert cells[c, 3] == pytest.approx((X0 + float(_com(c))) * unit, rel=1e-14)
        assert cells[c, 6] == VX_CELL[c]
        assert cells[c, 10] == pytest.approx(SY_CELL[c] ** 2, rel=1e-12)  # Sigma_yy
    # neighbours along x only
    nbr = cells[:, 21:27].astype(int)
    assert nbr[:, 0].tolist() == [-1, 0, 1, 2] and nbr[:, 1].tolist() == [1, 2, 3, -1]
    assert (nbr[:, 2:] == -1).all()

    def idw(k, power):
        c = k // 4
        cs = [c] + [d for d in (c - 1, c + 1) if 0 <= d < 4]
        w = [1 / abs(Fr(XS[k]) - _com(d)) ** power for d in cs]
        vx = sum(wi * VX_CELL[d] for wi, d in zip(w, cs)) / sum(w)
        syy = sum(wi * SY_CELL[d] ** 2 for wi, d in zip(w, cs)) / sum(w)
        return float(vx), float(syy)

    vbar, sig = out["vbar"], out["sigma"]
    at_com = [k for k in range(16) if XS[k] == _com(k // 4)]
    assert at_com == [5, 9, 10]
    for k in range(16):
        if k in at_com:
            continue
        vx, syy = idw(k, 1)
        assert vbar[0, k] == pytest.approx(vx, rel=2e-7, abs=1e-5), k
        assert sig[1, k] == pytest.approx(syy, rel=2e-7), k
    # particle 6 (x = 120) by hand: d = 10, 105, 95 to cells 1, 0, 2
    hand = (Fr(60, 10) + Fr(0, 105) + Fr(120, 95)) / (Fr(1, 10) + Fr(1, 105) + Fr(1, 95))
    assert vbar[0, 6] == pytest.approx(float(hand), rel=2e-7)
    # the same case under 1/r^2 or without normalisation is far off
    assert abs(idw(6, 2)[0] - float(hand)) > 0.3
    assert abs(float(Fr(60, 10) + Fr(120, 95)) - float(hand)) > 50
    # members exactly at their cell's centre of mass take the cell's values
    for k in at_com:
        c = k // 4
        assert vbar[0, k] == VX_CELL[c] and sig[1, k] == pytest.approx(SY_CELL[c] ** 2, rel=1e-7)
    # leaf density: mass over the leaf region (y, z one grid unit wide)
    widths = [100, 100, 100, 31]
    for c in range(4):
        m = sum(MS[4 * c:4 * c + 4])
        assert cells[c, 27] == pytest.approx(widths[c] * unit ** 3, rel=1e-12)
        assert out["rho_cell"][4 * c] == pytest.approx(m / (widths[c] * unit ** 3), rel=1e-6)


# --------------------------------------------------------------------------- mass weights
def _minimage(d):
    size = 1 << GB
    return ((d + size // 2) % size) - size // 2


@pytest.mark.parametrize("seed,n", [(31, 4000), (32, 12000)])
def test_cell_moments_mass_weighted(ref, seed, n):
    """Eqs. meanpos, meanvel, meandispvel with unequal masses against
    numpy.average and numpy.cov(aweights, bias=True) per cell."""
    w = synth.isolated_halo(seed=seed, n_host=n, n_sub=2, sub_range=(n // 10, n // 5))
    q = ref.quantize(w.x, w.box, w.grid_bits)
    rng = np.random.default_rng(seed)
    m = (rng.uniform(0.5, 1.5, q.shape[1]) * 1e8).astype(np.float32)
    P = ref.Particles(q, w.v, m, 0.0, w.box, w.grid_bits)
    N = P.n
    out = ref.cell_moments(P, np.array([0, N], np.int32), np.arange(N, dtype=np.int32))
    cells, cof = out["cells"], out["cell_of"]
    unit = w.box / (1 << GB)
    u = np.empty((3, N))
    for d in range(3):
        r0 = q[d, 0].astype(np.int64)
        u[d] = (r0 + _minimage(q[d].astype(np.int64) - r0)) * unit
    mm = m.astype(np.float64)
    for c in range(len(cells)):
        idx = np.nonzero(cof == c)[0]
        wt = mm[idx]
        xb = np.average(u[:, idx], axis=1, weights=wt)
        vb = np.average(w.v[:, idx].astype(np.float64), axis=1, weights=wt)
        cov = np.cov(w.v[:, idx].astype(np.float64), aweights=wt, bias=True)
        assert cells[c, 2] == pytest.approx(wt.sum(), rel=1e-12)
        np.testing.assert_allclose(cells[c, 3:6], xb, rtol=1e-12)
        np.testing.assert_allclose(cells[c, 6:9], vb, rtol=1e-10, atol=1e-9)
        expv = [cov[0, 0], cov[1, 1], cov[2, 2], cov[0, 1], cov[0, 2], cov[1, 2]]
        np.testing.assert_allclose(cells[c, 9:15], expv, rtol=1e-9, atol=1e-6)
        # the count-weighted mean is measurably different: the pin can tell
        if c == 0:
            assert np.abs(np.mean(w.v[:, idx].astype(np.float64), axis=1) - vb).max() > 1e-3
        k = idx[0]
        assert out["rho_cell"][k] == pytest.approx(wt.sum() / cells[c, 27], rel=1e-6)


def _entropy_np(h):
    p = h[h > 0] / h.sum()
    return float(-(p * np.log(p)).sum() / math.log(len(h)))


def test_entropy_split_weights_by_mass(ref):
    """The entropy of the split choice is that of the MASS histogram.  Light
    particles (3000 of mass 1) sit in two clumps along x; heavy ones (1000 of
    mass 100) in a thin sheet along y.  By count x is the most structured
    dimension, by mass y; the minimum-entropy rule must split y."""
    rng = np.random.default_rng(5)
    nA, nB = 3000, 1000
    xa = np.stack([np.where(rng.random(nA) < 0.5, 0.35, 0.65) + rng.normal(0, 0.003, nA),
                   0.3 + 0.4 * rng.random(nA), 0.3 + 0.4 * rng.random(nA)])
    xb = np.stack([0.3 + 0.4 * rng.random(nB), 0.5 + rng.normal(0, 0.003, nB), 0.3 + 0.4 * rng.random(nB)])
    x = np.concatenate([xa, xb], 1)
    m = np.r_[np.ones(nA), np.full(nB, 100.0)].astype(np.float32)
    perm = rng.permutation(nA + nB)
    x, m = np.ascontiguousarray(x[:, perm]), m[perm]
    q = ref.quantize(x.astype(np.float32), 1.0, GB)
    v = rng.normal(0, 10, (3, nA + nB)).astype(np.float32)
    # the construction discriminates: count histograms favour x, mass ones y
    qi = q.astype(np.int64)
    S_count, S_mass = [], []
    for d in range(3):
        lo, hi = qi[d].min(), qi[d].max()
        b = ((qi[d] - lo) * 16) // (hi - lo + 1)
        S_count.append(_entropy_np(np.bincount(b, minlength=16).astype(float)))
        S_mass.append(_entropy_np(np.bincount(b, weights=m.astype(float), minlength=16)))
    assert int(np.argmin(S_count)) == 0 and int(np.argmin(S_mass)) == 1
    # one split only: N_cell = N / 2
    N = nA + nB
    for mass, split_dim in [(m, 1), (None, 0)]:
        P = ref.Particles(q, v, mass, 1.0, 1.0, GB)
        out = ref.cell_moments(P, np.array([0, N], np.int32), np.arange(N, dtype=np.int32),
                               f_cell=0.5, ncell_floor=1, ncell_div=2)
        cells = out["cells"]
        assert cells.shape[0] == 2
        lo, hi = cells[:, 15:18], cells[:, 18:21]
        differs = [d for d in range(3) if lo[0, d] != lo[1, d] or hi[0, d] != hi[1, d]]
        assert differs == [split_dim]


# --------------------------------------------------------------------------- velocity frame
def _sphere_dirs(k, upper=False):
    """k unit vectors spread on the sphere (or its upper half), golden spiral."""
    i = np.arange(k) + 0.5
    z = 1 - i / k if upper else 1 - 2 * i / k
    r = np.sqrt(1 - z * z)
    ph = math.pi * (1 + 5 ** 0.5) * i
    return np.stack([r * np.cos(ph), r * np.sin(ph), z])


def _frame_case(n_core, n_ring, a_units, extra_at, vel_core, u, w_extra, R=0.05):
    """A compact core (particle 0 at its centre, the others at radii
    a (1 + 0.03 k)), one extra particle at extra_at * a below it, and a ring
    of n_ring particles on the upper hemisphere of radius R; 1-unit box,
    2^21 grid.  vel_core(rank) is the x velocity of the core member of that
    distance rank from particle 0; the ring moves at u along x, the extra
    particle at w_extra."""
    c0 = np.array([1 << 20] * 3, np.int64)
    dc = _sphere_dirs(n_core - 1)
    rad = a_units * (1 + 0.03 * np.arange(1, n_core))
    core = c0[:, None] + np.rint(dc * rad).astype(np.int64)
    extra = c0 + np.array([0, 0, -extra_at * a_units])
    ring = c0[:, None] + np.rint(_sphere_dirs(n_ring, upper=True) * R * (1 << GB)).astype(np.int64)
    q = np.concatenate([c0[:, None], core, extra[:, None], ring], 1)
    n = q.shape[1]
    d2 = ((q - c0[:, None]) ** 2).sum(0)
    order = np.lexsort((np.arange(n), d2))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    # the core members are the n_core nearest to particle 0, the extra next
    assert (np.sort(order[:n_core]) == np.arange(n_core)).all() and order[n_core] == n_core
    v = np.zeros((3, n), np.float32)
    for k in range(n_core):
        v[0, k] = vel_core(rank[k])
    v[0, n_core] = w_extra
    v[0, n_core + 1:] = u
    return q.astype(np.uint32), v


def _phi_bounds(q, m, eps, idx, partners):
    """Bounds of |phi_i| for i in idx from distances alone (no potential sum):
    each partner j contributes G m / sqrt(d_ij^2 + eps^2), so with the
    nearest and farthest partner of i, G m k / sqrt(d_max^2 + eps^2) <=
    |phi_i| restricted to k partners, and |phi_i| over all partners <=
    G m (n-1) / sqrt(d_min^2 + eps^2).  Returns (lower over the partners,
    upper over all)."""
    x = q.astype(np.float64) / (1 << GB)
    n = q.shape[1]
    lo, hi = np.inf, 0.0
    for i in idx:
        d = np.sqrt(((x - x[:, i:i + 1]) ** 2).sum(0))
        dp = d[[j for j in partners if j != i]]
        lo = min(lo, G * m * len(dp) / math.sqrt(dp.max() ** 2 + eps ** 2))
        hi = max(hi, G * m * (n - 1) / math.sqrt(np.delete(d, i).min() ** 2 + eps ** 2))
    return lo, hi


def _argmin_phi_brute(q, idx):
    x = q[:, idx].astype(np.float64) / (1 << GB)
    d = np.sqrt(((x[:, :, None] - x[:, None, :]) ** 2).sum(0))
    np.fill_diagonal(d, np.inf)
    return int(idx[int(np.argmax((1 / d).sum(1)))])


def test_unbind_frame_type1_vs_centre_of_mass(ref):
    """41 members: a core of 10 at rest, one extra particle just outside it
    moving at 11 u, 30 ring particles moving at u.  The frame of the 10
    members nearest the potential minimum is at rest, so the ring (|v| = u,
    above its escape threshold) and the extra leave; the core stays.  The
    centre-of-mass frame moves at u: the ring is at rest there and stays
    (then the frame of core + ring moves at 0.75 u and the ring is still
    bound).  A frame set of 11, or one without the minimum itself, moves at
    about u and would keep the ring."""
    m, eps, beta = 1e10, 1e-7, 0.95
    n_core, n_ring, a = 10, 30, 1000
    q, _ = _frame_case(n_core, n_ring, a, 3, lambda r: 0.0, 0.0, 0.0)
    n = q.shape[1]
    core, extra, ring = np.arange(n_core), [n_core], np.arange(n_core + 1, n)
    every = np.arange(n)
    ring_lo, ring_hi = _phi_bounds(q, m, eps, ring, every)
    core_lo, _ = _phi_bounds(q, m, eps, core, core)
    _, extra_hi = _phi_bounds(q, m, eps, extra, every)
    u = math.sqrt(2 * 1.5 * ring_hi / beta)        # beta u^2 / 2 = 1.5 max |phi_ring|
    # margins of the construction (distance bounds only)
    assert beta * 0.5 * (0.25 * u) ** 2 < 0.5 * ring_lo          # ring bound at 0.25 u
    assert beta * 0.5 * (0.75 * u) ** 2 < 0.5 * core_lo          # core bound at 0.75 u
    assert beta * 0.5 * (10 * u) ** 2 > 2 * extra_hi             # extra unbound at >= 10 u
    assert _argmin_phi_brute(q, every) == 0 and _argmin_phi_brute(q, core) == 0
    q, v = _frame_case(n_core, n_ring, a, 3, lambda r: 0.0, u, 11 * u)
    P = ref.Particles(q, v, None, m, 1.0, GB)
    off, mem = np.array([0, n]), np.arange(n)
    f1 = ref.unbind(P, off, mem, G, eps, n_min=5, frame_type=1)
    assert f1["bound"].tolist() == [1] * n_core + [0] * (1 + n_ring)
    assert f1["iters"][0] == 2
    f0 = ref.unbind(P, off, mem, G, eps, n_min=5, frame_type=0)
    assert f0["bound"].tolist() == [1] * n_core + [0] + [1] * n_ring


def test_unbind_frame_set_is_ten_percent(ref):
    """145 members: n_ref = max(10, ceil(14.5)) = 15.  The 10 members nearest
    the minimum move at +u, the next 5 at -2u (mean of the 15: zero), the
    16th nearest (extra) at 16u, and 129 ring particles at u.  Only the
    frame of exactly 15 is at rest, where the ring leaves; frames of 10 or
    16 members (or 15 without the minimum) move at u and would keep it.
    Once the ring is gone, the 15 core members (n_ref = 10: a frame at u)
    stay bound at relative speeds up to 3u."""
    m, eps, beta = 1e10, 1e-7, 0.95
    n_core, n_ring, a = 15, 129, 30
    q, _ = _frame_case(n_core, n_ring, a, 6, lambda r: 0.0, 0.0, 0.0)
    n = q.shape[1]
    assert n == 145 and max(10, math.ceil(0.1 * n)) == 15
    core, extra, ring = np.arange(n_core), [n_core], np.arange(n_core + 1, n)
    every = np.arange(n)
    _, ring_hi = _phi_bounds(q, m, eps, ring, every)
    core_lo, _ = _phi_bounds(q, m, eps, core, core)
    _, extra_hi = _phi_bounds(q, m, eps, extra, every)
    u = math.sqrt(2 * 1.2 * ring_hi / beta)
    assert beta * 0.5 * (3 * u) ** 2 < 0.5 * core_lo
    assert beta * 0.5 * (15 * u) ** 2 > 1.5 * extra_hi
    assert _argmin_phi_brute(q, every) == 0 and _argmin_phi_brute(q, core) == 0
    q, v = _frame_case(n_core, n_ring, a, 6, lambda r: u if r < 10 else -2 * u, u, 16 * u)
    P = ref.Particles(q, v, None, m, 1.0, GB)
    f1 = ref.unbind(P, np.array([0, n]), np.arange(n), G, eps, n_min=5, frame_type=1)
    assert f1["bound"].tolist() == [1] * n_core + [0] * (1 + n_ring)
    assert f1["iters"][0] == 2
