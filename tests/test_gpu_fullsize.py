"""Parity at the benchmark's full size: the 256^3 box (16,777,216 particles,
100 Mpc/h) through the GPU pipeline in the configuration bench.py times
(same knobs), checked where the oracle can follow it exactly:

* every FOF label is canonical (label[i] <= i, label[label[i]] = label[i])
  and the group table is consistent;
* for 20,000 random particles, every particle within ellx (exact integer
  distance, found with scipy's periodic KD-tree) carries the same label;
* for groups sampled over the size range, the component grown from the
  group's smallest member through all links (the plain definition) is
  exactly the GPU group;
* on hosts among those (all members known from that growth), the oracle's
  cells, R, 6D FOF and unbinding match the GPU's full-box outputs, with the
  tolerances of the small parity tests.

Host-level steps are independent between hosts, so a host's oracle result
is its result in the full box.
"""
import os

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree

from paper_1902_01010_amd import pipeline, synth

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def note(msg):
    # shown with the report of a failing test
    print(f"[fullsize] {msg}", flush=True)


@pytest.fixture(scope="module")
def full(ref):
    from paper_1902_01010_amd import vr
    w = synth.cosmo_box(seed=2, n_side=256)
    note(f"generated {w.n} particles")
    prm = pipeline.Params.from_workload(w)
    ctx = vr.Context(0)
    tune = os.path.join(ROOT, "paper_1902_01010_amd", "data", "autotune_gfx950.json")
    if os.path.exists(tune):
        ctx.autotune(tune)
    x, v, m = pipeline.device_inputs(w)
    out, _ = pipeline.run(ctx, x, v, m, w.mass_value, w.box, w.grid_bits, prm)
    torch.cuda.synchronize()
    got = dict(q=out["q"].cpu().numpy(), label=out["label"].cpu().numpy(), offsets=out["offsets"].cpu().numpy(),
               members=out["members"].cpu().numpy(), n_hosts=out["n_hosts"], R=out["R"].cpu().numpy(),
               vbar=out["cells"]["vbar"].cpu().numpy(), sigma=out["cells"]["sigma"].cpu().numpy(),
               rho=out["cells"]["rho_cell"].cpu().numpy(), label6=out["label6"].cpu().numpy(),
               bound=out["unbind"]["bound"].cpu().numpy())
    note("GPU pipeline done")
    q = ref.quantize(w.x, w.box, w.grid_bits)
    assert (q == got["q"]).all()
    Pr = ref.Particles(q, w.v, w.mass, w.mass_value, w.box, w.grid_bits)
    ell2 = (prm.ellx * 2.0 ** w.grid_bits / w.box) ** 2
    tree = cKDTree(q.T.astype(np.float64), boxsize=float(2 ** w.grid_bits), leafsize=32, balanced_tree=False,
                   compact_nodes=False)
    note("oracle side ready")
    return dict(w=w, prm=prm, got=got, Pr=Pr, q=q.astype(np.int64), ell2=ell2, tree=tree)


def links(F, idx):
    """(i, j) pairs with j linked to i by Eq. fof3d, for the particles idx:
    flat arrays, candidates from the KD-tree, decided on the exact integer
    squared distance."""
    q, ell2, gb = F["q"], F["ell2"], F["w"].grid_bits
    idx = np.asarray(idx, np.int64)
    cand = F["tree"].query_ball_point(q[:, idx].T.astype(np.float64), r=np.sqrt(ell2) * (1 + 1e-9))
    cnt = np.fromiter((len(c) for c in cand), np.int64, len(cand))
    ii = np.repeat(idx, cnt)
    jj = np.concatenate([np.asarray(c, np.int64) for c in cand]) if len(cand) else np.zeros(0, np.int64)
    size, half = 1 << gb, 1 << (gb - 1)
    d = (q[:, jj] - q[:, ii] + half) % size - half
    keep = (d * d).sum(0).astype(np.float64) < ell2
    return ii[keep], jj[keep]


def component(F, seed):
    """The FOF component of `seed`, grown link by link."""
    seen = np.zeros(F["q"].shape[1], bool)
    seen[seed] = True
    front = np.array([seed], np.int64)
    while len(front):
        _, jj = links(F, front)
        jj = np.unique(jj)
        front = jj[~seen[jj]]
        seen[front] = True
    return np.nonzero(seen)[0]


def test_fullsize_labels_and_groups_consistent(full):
    g = full["got"]
    lab = g["label"]
    n = lab.shape[0]
    assert (lab <= np.arange(n)).all()
    assert (lab[lab] == lab).all()
    off, mem = g["offsets"], g["members"]
    sizes = np.diff(off)
    assert (sizes >= 20).all() and (np.diff(sizes) <= 0).all()
    for gi in np.random.default_rng(0).choice(len(sizes), 200, replace=False):
        mm = mem[off[gi]:off[gi + 1]]
        assert (np.diff(mm) > 0).all() and (lab[mm] == mm[0]).all()
    # every particle of a group of >= 20 is listed once
    counts = np.bincount(lab, minlength=n)
    assert int(counts[counts >= 20].sum()) == int(off[-1])


def test_fullsize_sampled_links(full):
    lab = full["got"]["label"]
    idx = np.random.default_rng(1).choice(lab.shape[0], 20000, replace=False)
    ii, jj = links(full, idx)
    assert (lab[ii] == lab[jj]).all()
    assert len(ii) > 20000  # self links plus real ones
    note(f"{len(ii)} sampled links agree")


@pytest.fixture(scope="module")
def hosts(full):
    """Groups across the size range, each regrown from its smallest member."""
    g = full["got"]
    off, mem = g["offsets"], g["members"]
    sizes = np.diff(off)
    picks = []
    for target in (20, 60, 300, 1500, 8000, 40000):
        picks.append(int(np.argmin(np.abs(sizes - target))))
    out = {}
    for gi in picks:
        comp = component(full, mem[off[gi]])
        out[gi] = comp
    note(f"regrew {len(out)} groups of sizes {[len(c) for c in out.values()]}")
    return out


def test_fullsize_sampled_components(full, hosts):
    g = full["got"]
    off, mem = g["offsets"], g["members"]
    for gi, comp in hosts.items():
        np.testing.assert_array_equal(comp, mem[off[gi]:off[gi + 1]])


def test_fullsize_sampled_hosts_cells_and_R(full, hosts, ref):
    g, Pr, prm = full["got"], full["Pr"], full["prm"]
    rng = np.random.default_rng(2)
    checked = 0
    for gi, comp in hosts.items():
        if len(comp) < prm.host_min:
            continue
        hoff = np.array([0, len(comp)], np.int32)
        hmem = comp.astype(np.int32)
        cm = ref.cell_moments(Pr, hoff, hmem)
        for k, mine in (("vbar", "vbar"), ("sigma", "sigma"), ("rho_cell", "rho")):
            e = cm[k][..., comp]
            gv = g[mine][..., comp]
            np.testing.assert_allclose(gv, e, rtol=2e-6, atol=1e-6 * np.abs(e).max())
        sub = np.sort(rng.choice(comp, min(150, len(comp)), replace=False)).astype(np.int32)
        R = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v, subset=sub)["R"]
        e, gr = R[sub].astype(np.float64), g["R"][sub].astype(np.float64)
        fin = np.isfinite(e)
        assert (np.isnan(gr) == np.isnan(e)).all()
        err = np.abs(gr[fin] - e[fin]) / np.maximum(1.0, np.abs(e[fin]))
        assert err.max() <= 1e-4, err.max()
        checked += 1
        note(f"host of {len(comp)}: cells and R agree")
    assert checked >= 3


def test_fullsize_sampled_6d_and_unbinding(full, hosts, ref):
    g, Pr, prm, w = full["got"], full["Pr"], full["prm"], full["w"]
    checked = 0
    for gi, comp in hosts.items():
        if not (prm.host_min <= len(comp) <= 10000):
            continue
        hoff = np.array([0, len(comp)], np.int32)
        hmem = comp.astype(np.int32)
        cm = ref.cell_moments(Pr, hoff, hmem)
        R = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v)["R"]
        e = R[comp].astype(np.float64)
        if np.any(np.abs(e - prm.R_threshold) <= 2e-4):
            continue  # a member at the threshold: its class is not fixed by the tolerance
        ellv = ref.host_ellv(Pr, hoff, hmem, prm.alpha_v)
        host_of = np.full(Pr.n, -1, np.int32)
        host_of[comp] = 0
        lab6 = ref.fof6d(Pr, host_of, ellv, prm.alpha_xs * prm.ellx, R, prm.R_threshold)
        np.testing.assert_array_equal(g["label6"][comp], lab6[comp])
        ng, _, off6, mem6 = ref.groups(lab6, prm.n_min)
        if ng:
            ub = ref.unbind(Pr, off6, mem6, prm.G, prm.eps, beta_E=prm.beta_E, n_min=prm.n_min)
            clean = ub["min_margin"] > 1e-5
            for k in np.nonzero(clean)[0]:
                mm = mem6[off6[k]:off6[k + 1]]
                assert (g["bound"][mm] == ub["bound"][mm]).all()
        checked += 1
        note(f"host of {len(comp)}: 6D groups and unbinding agree ({ng} candidates)")
    assert checked >= 1


def regional_component(full, ref, centre_q, half):
    """The oracle's 3D FOF component of the particle nearest centre_q (grid
    units), linked among the particles of the cube of half-side `half`
    around it.  Returned (global indices, ascending) only when every member
    keeps more than ellx from the cube's faces: then no particle outside the
    cube links to it and it is the component in the whole box; else None."""
    w, q = full["w"], full["q"]
    size, hb = 1 << w.grid_bits, 1 << (w.grid_bits - 1)
    off = (q - centre_q[:, None] + hb) % size - hb
    sel = np.nonzero((np.abs(off) < half).all(0))[0]
    offs = off[:, sel]
    Ps = ref.Particles(q[:, sel].astype(np.uint32), w.v[:, sel], None, w.mass_value, w.box, w.grid_bits)
    lab = ref.fof3d(Ps, full["prm"].ellx)
    seed = int(np.argmin((offs * offs).sum(0)))
    loc = np.nonzero(lab == lab[seed])[0]
    if np.abs(offs[:, loc]).max() >= half - np.sqrt(full["ell2"]) - 1:
        return None
    return np.sort(sel[loc])


@pytest.fixture(scope="module")
def big_hosts(full, ref):
    """The components around the three largest planted halos and around the
    planted halo closest to 6e4 particles, each found by the oracle's FOF in
    a cube that the component provably does not leave."""
    w = full["w"]
    H = w.meta["halos"]
    scale = (1 << w.grid_bits) / w.box
    order = np.argsort(-H["size"], kind="stable")
    mid = int(np.argmin(np.abs(H["size"] - 60000)))
    out = []
    for h in list(order[:3]) + [mid]:
        c = np.floor(H["centre"][:, h] * scale).astype(np.int64) % (1 << w.grid_bits)
        half = int(1.5 * H["r200"][h] * scale)
        comp = None
        for _ in range(4):
            comp = regional_component(full, ref, c, half)
            if comp is not None:
                break
            half *= 2
        assert comp is not None, f"component of planted halo {h} not enclosed"
        out.append(comp)
    note(f"regional components of sizes {[len(c) for c in out]}")
    return out


@pytest.mark.timeout(1200)
def test_fullsize_largest_hosts(full, big_hosts, ref):
    """The largest hosts of the box (about 1e6 members: the deepest KD levels
    and the biggest neighbour trees) and one of 5e4-1e5 members: the oracle
    finds each component itself; the GPU group is exactly it; the oracle's
    cells (all members) and R (150 sampled members) match the GPU's
    full-box outputs; on the mid-size host also the 6D groups and the
    unbinding of every candidate decided outside the tolerance band."""
    g, Pr, prm = full["got"], full["Pr"], full["prm"]
    lab = g["label"]
    rng = np.random.default_rng(3)
    for i, comp in enumerate(big_hosts):
        gpu = np.nonzero(lab == lab[comp[0]])[0]
        np.testing.assert_array_equal(gpu, comp)
        assert len(comp) >= prm.host_min
        hoff = np.array([0, len(comp)], np.int32)
        hmem = comp.astype(np.int32)
        cm = ref.cell_moments(Pr, hoff, hmem)
        for k, mine in (("vbar", "vbar"), ("sigma", "sigma"), ("rho_cell", "rho")):
            e = cm[k][..., comp]
            gv = g[mine][..., comp]
            np.testing.assert_allclose(gv, e, rtol=2e-6, atol=1e-6 * np.abs(e).max())
        sub = np.sort(rng.choice(comp, 150, replace=False)).astype(np.int32)
        R = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v, subset=sub)["R"]
        e, gr = R[sub].astype(np.float64), g["R"][sub].astype(np.float64)
        fin = np.isfinite(e)
        assert (np.isnan(gr) == np.isnan(e)).all()
        err = np.abs(gr[fin] - e[fin]) / np.maximum(1.0, np.abs(e[fin]))
        assert err.max() <= 1e-4, err.max()
        note(f"host of {len(comp)}: group, cells and sampled R agree")
    comp = big_hosts[-1]
    assert len(comp) >= 50000
    hoff = np.array([0, len(comp)], np.int32)
    hmem = comp.astype(np.int32)
    cm = ref.cell_moments(Pr, hoff, hmem)
    R = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v)["R"]
    e, gr = R[comp].astype(np.float64), g["R"][comp].astype(np.float64)
    fin = np.isfinite(e)
    err = np.abs(gr[fin] - e[fin]) / np.maximum(1.0, np.abs(e[fin]))
    assert err.max() <= 1e-4, err.max()
    # the outlier classes must agree; inside the tolerance band a different
    # class is allowed, but then the 6D groups are not comparable
    near = np.abs(e - prm.R_threshold) <= 2e-4
    differ = (gr >= prm.R_threshold) != (e >= prm.R_threshold)
    assert not (differ & ~near).any()
    if differ.any():
        pytest.skip(f"{int(differ.sum())} member(s) classed differently inside the tolerance band")
    ellv = ref.host_ellv(Pr, hoff, hmem, prm.alpha_v)
    host_of = np.full(Pr.n, -1, np.int32)
    host_of[comp] = 0
    lab6 = ref.fof6d(Pr, host_of, ellv, prm.alpha_xs * prm.ellx, R, prm.R_threshold)
    np.testing.assert_array_equal(g["label6"][comp], lab6[comp])
    ng, _, off6, mem6 = ref.groups(lab6, prm.n_min)
    assert ng >= 1
    ub = ref.unbind(Pr, off6, mem6, prm.G, prm.eps, beta_E=prm.beta_E, n_min=prm.n_min)
    clean = ub["min_margin"] > 1e-5
    for k in np.nonzero(clean)[0]:
        mm = mem6[off6[k]:off6[k + 1]]
        assert (g["bound"][mm] == ub["bound"][mm]).all()
    note(f"host of {len(comp)}: {ng} 6D candidates, {int(clean.sum())} unbound-checked")
