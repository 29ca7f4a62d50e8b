"""GPU parity of the cells, R, 6D FOF and unbinding entry points against the
CPU oracle, on the same seeded inputs.

Tolerances: integer results (cell partitions, neighbour-derived labels,
bound flags) are bit-exact; FP64 reductions agree to round-off (rtol 1e-10);
R agrees to 1e-4 max(1, |R|) (the outlier classification is compared outside
that band); potentials agree to 1e-5 relative.
"""
import dataclasses

import numpy as np
import pytest
import torch

from paper_1902_01010_amd import synth
from tests.gpu_common import both, dev_tensor, gpu_particles

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vr():
    from paper_1902_01010_amd import vr as _vr
    return _vr


@pytest.fixture(scope="module")
def ctx(vr):
    return vr.Context(0)


def hosts_of(ref, Pr, w, host_min=256):
    lab = ref.fof3d(Pr, w.params["ellx"])
    ng, gof, off, mem = ref.groups(lab, 20)
    sizes = np.diff(off)
    nh = int((sizes >= host_min).sum())
    hoff = off[:nh + 1].copy()
    hmem = mem[:hoff[-1]].copy()
    host_of = np.where((gof >= 0) & (gof < nh), gof, -1).astype(np.int32)
    return hoff, hmem, host_of


CASES = {
    "halo12k": lambda: synth.isolated_halo(seed=21, n_host=12000, n_sub=3, sub_range=(400, 1500)),
    "box48": lambda: synth.cosmo_box(seed=22, n_side=48),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, ctx, vr, ref):
    w = CASES[request.param]()
    P, Pr = both(ctx, vr, ref, w)
    hoff, hmem, host_of = hosts_of(ref, Pr, w)
    assert len(hoff) > 1
    return dict(w=w, P=P, Pr=Pr, hoff=hoff, hmem=hmem, host_of=host_of)


def test_cell_moments_parity(ctx, ref, case):
    P, Pr, hoff, hmem = case["P"], case["Pr"], case["hoff"], case["hmem"]
    exp = ref.cell_moments(Pr, hoff, hmem)
    got = ctx.cell_moments(P, dev_tensor(hoff), dev_tensor(hmem))
    assert got["n_cells"] == exp["cells"].shape[0]
    gc = got["cells"].cpu().numpy()
    ec = exp["cells"]
    ints = [0, 1] + list(range(15, 27))
    assert (gc[:, ints] == ec[:, ints]).all()
    np.testing.assert_allclose(gc[:, [2, 27]], ec[:, [2, 27]], rtol=1e-12)
    np.testing.assert_allclose(gc[:, 3:6], ec[:, 3:6], rtol=1e-12)
    np.testing.assert_allclose(gc[:, 6:15], ec[:, 6:15], rtol=1e-9, atol=1e-9 * np.abs(ec[:, 6:15]).max())
    assert (got["cell_of"].cpu().numpy() == exp["cell_of"]).all()
    for k in ("vbar", "sigma", "rho_cell"):
        g = got[k].cpu().numpy()
        e = exp[k]
        fin = np.isfinite(e)
        assert (np.isfinite(g) == fin).all()
        np.testing.assert_allclose(g[fin], e[fin], rtol=2e-6, atol=1e-6 * np.abs(e[fin]).max())


def test_cells_and_R_with_coincident_members(ctx, vr, ref):
    """Hosts holding groups of exactly coincident members, larger than a
    cell: KD nodes that cannot be split stay leaves (fewer nodes than the
    member counts alone would give), and the neighbour sets meet exact
    distance ties, broken by particle index."""
    rng = np.random.default_rng(17)
    c = 1 << 20
    parts, host = [], []
    for h, (groups, spread) in enumerate([((150, 150, 150), 450), ((200, 200), 300)]):
        base = np.array([c + 400000 * h, c, c])[:, None]
        for g in groups:
            parts.append(np.repeat(base + rng.integers(-3000, 3000, (3, 1)), g, axis=1))
            host += [h] * g
        parts.append(base + rng.normal(0, 3000, (3, spread)).astype(np.int64))
        host += [h] * spread
    q = np.concatenate(parts, 1).astype(np.uint32)
    host = np.array(host)
    n = q.shape[1]
    perm = rng.permutation(n)
    q, host = np.ascontiguousarray(q[:, perm]), host[perm]
    v = rng.normal(0, 100, (3, n)).astype(np.float32)
    Pr = ref.Particles(q, v, None, 1.0, 1.0, 21)
    P = vr.Particles(dev_tensor(q), dev_tensor(v), None, 1.0, 1.0, 21)
    hmem = np.concatenate([np.nonzero(host == 0)[0], np.nonzero(host == 1)[0]]).astype(np.int32)
    hoff = np.array([0, (host == 0).sum(), n], np.int32)
    exp = ref.cell_moments(Pr, hoff, hmem)
    got = ctx.cell_moments(P, dev_tensor(hoff), dev_tensor(hmem))
    assert got["n_cells"] == exp["cells"].shape[0]
    assert (got["cell_of"].cpu().numpy() == exp["cell_of"]).all()
    for k in ("vbar", "sigma"):
        g, e = got[k].cpu().numpy(), exp[k]
        fin = np.isfinite(e)
        assert (np.isfinite(g) == fin).all()
        np.testing.assert_allclose(g[fin], e[fin], rtol=2e-6, atol=1e-6 * np.abs(e[fin]).max())
    for n_se, n_v in [(32, 8), (48, 16), (100, 20)]:
        e = ref.local_vdensity(Pr, hoff, hmem, exp["vbar"], exp["sigma"], n_se, n_v)["R"]
        g = ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(hmem), dev_tensor(exp["vbar"]),
                               dev_tensor(exp["sigma"]), n_se, n_v).cpu().numpy()
        _R_close(g, e)


@pytest.mark.parametrize("ncell_floor", [100, 24])
def test_cells_and_R_with_unequal_masses(ctx, vr, ref, case, ncell_floor):
    """Per-particle masses (0.5-1.5 m_p): the mass-weighted entropy histograms
    (with small cells, the deep KD levels put many nodes in one histogram
    chunk), the mass-weighted moments, and the kNN's per-member mass records
    (f_l of the ratio) against the oracle."""
    w = case["w"]
    rng = np.random.default_rng(101)
    m = (rng.uniform(0.5, 1.5, w.n) * w.mass_value).astype(np.float32)
    q_dev = case["P"].q
    P = vr.Particles(q_dev, dev_tensor(w.v), dev_tensor(m), 0.0, w.box, w.grid_bits)
    Pr = ref.Particles(case["Pr"].q, w.v, m, 0.0, w.box, w.grid_bits)
    hoff, hmem = case["hoff"], case["hmem"]
    kw = dict(ncell_floor=ncell_floor)
    exp = ref.cell_moments(Pr, hoff, hmem, **kw)
    got = ctx.cell_moments(P, dev_tensor(hoff), dev_tensor(hmem), **kw)
    assert got["n_cells"] == exp["cells"].shape[0]
    gc, ec = got["cells"].cpu().numpy(), exp["cells"]
    ints = [0, 1] + list(range(15, 27))
    assert (gc[:, ints] == ec[:, ints]).all()
    np.testing.assert_allclose(gc[:, [2, 27]], ec[:, [2, 27]], rtol=1e-12)
    np.testing.assert_allclose(gc[:, 3:6], ec[:, 3:6], rtol=1e-12)
    np.testing.assert_allclose(gc[:, 6:15], ec[:, 6:15], rtol=1e-9, atol=1e-9 * np.abs(ec[:, 6:15]).max())
    assert (got["cell_of"].cpu().numpy() == exp["cell_of"]).all()
    for k in ("vbar", "sigma", "rho_cell"):
        g, e = got[k].cpu().numpy(), exp[k]
        fin = np.isfinite(e)
        assert (np.isfinite(g) == fin).all()
        np.testing.assert_allclose(g[fin], e[fin], rtol=2e-6, atol=1e-6 * np.abs(e[fin]).max())
    # masses change the partition itself (entropy of the mass histogram)
    if ncell_floor == 24:
        plain = ref.cell_moments(case["Pr"], hoff, hmem, **kw)
        assert (plain["cell_of"] != exp["cell_of"]).any()
    e = ref.local_vdensity(Pr, hoff, hmem, exp["vbar"], exp["sigma"], 32, 8)["R"]
    g = ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(hmem), dev_tensor(exp["vbar"]),
                           dev_tensor(exp["sigma"]), 32, 8).cpu().numpy()
    _R_close(g, e)


def test_host_ellv_parity(ctx, ref, case):
    P, Pr, hoff, hmem = case["P"], case["Pr"], case["hoff"], case["hmem"]
    exp = ref.host_ellv(Pr, hoff, hmem, 1.25)
    got = ctx.host_ellv(P, dev_tensor(hoff), dev_tensor(hmem), 1.25).cpu().numpy()
    np.testing.assert_allclose(got, exp, rtol=1e-12)


def test_host_reads_beyond_the_staging_buffer(ctx, vr, ref):
    """20,000 hosts: the host offsets (80 KB) and the hosts' velocity
    linking lengths (160 KB) are read back through the context's pinned
    staging buffer, which grows past its initial 64 KB, while the chunk
    tables of host_ellv go up through the pinned upload buffer.  host_ellv,
    fof6d, host_ellv again: the second call reuses the upload buffer after
    the staging buffer grew, and both calls match the oracle."""
    w = synth.unbind_groups(seed=11, sizes=[20] * 20_000)
    off, mem = w.groups
    assert len(off) - 1 > 16_384
    P, Pr = both(ctx, vr, ref, w)
    host_of = np.full(w.n, -1, np.int32)
    for g in range(len(off) - 1):
        host_of[mem[off[g]:off[g + 1]]] = g
    exp = ref.host_ellv(Pr, off, mem, 1.25)
    off_d, mem_d = dev_tensor(off), dev_tensor(mem)
    e1 = ctx.host_ellv(P, off_d, mem_d, 1.25)
    lab = ctx.fof6d(P, dev_tensor(host_of), e1, 0.01 * w.box)
    e2 = ctx.host_ellv(P, off_d, mem_d, 1.25)
    lab2 = ctx.fof6d(P, dev_tensor(host_of), e2, 0.01 * w.box)
    np.testing.assert_allclose(e1.cpu().numpy(), exp, rtol=1e-12)
    assert (e2.cpu().numpy() == e1.cpu().numpy()).all()
    assert (lab2.cpu().numpy() == lab.cpu().numpy()).all()


def _R_close(g, e):
    fin = np.isfinite(e)
    assert (np.isnan(g) == np.isnan(e)).all()
    assert (np.isposinf(g) == np.isposinf(e)).all()
    err = np.abs(g[fin] - e[fin]) / np.maximum(1.0, np.abs(e[fin]))
    assert err.max() <= 1e-4, err.max()
    # classification at the threshold, outside the tolerance band
    band = np.abs(e - 2.0) <= 2e-4
    cls_g = g >= 2.0
    cls_e = e >= 2.0
    assert (cls_g[~band] == cls_e[~band]).all()


def test_local_vdensity_parity_same_inputs(ctx, ref, case):
    P, Pr, hoff, hmem = case["P"], case["Pr"], case["hoff"], case["hmem"]
    cm = ref.cell_moments(Pr, hoff, hmem)
    exp = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], 32, 8)["R"]
    got = ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(hmem), dev_tensor(cm["vbar"]),
                             dev_tensor(cm["sigma"]), 32, 8).cpu().numpy()
    _R_close(got, exp)


@pytest.mark.parametrize("n_se,n_v", [(256, 32), (100, 20), (64, 64)])
def test_local_vdensity_large_neighbour_sets(ctx, ref, case, n_se, n_v):
    # up to the paper's own defaults, 256 spatial and 32 velocity neighbours
    P, Pr, hoff, hmem = case["P"], case["Pr"], case["hoff"], case["hmem"]
    cm = ref.cell_moments(Pr, hoff, hmem)
    exp = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], n_se, n_v)["R"]
    got = ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(hmem), dev_tensor(cm["vbar"]),
                             dev_tensor(cm["sigma"]), n_se, n_v).cpu().numpy()
    _R_close(got, exp)


def test_local_vdensity_rejects_sizes(ctx, vr, case):
    P, hoff, hmem, w = case["P"], case["hoff"], case["hmem"], case["w"]
    z = torch.zeros(3 * P.n, dtype=torch.float32, device="cuda")
    for n_se, n_v in [(257, 8), (128, 33), (8, 9), (8, 1)]:
        with pytest.raises(vr.VrError):
            ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(hmem), z, torch.zeros(6 * P.n, device="cuda"), n_se,
                               n_v)


def test_local_vdensity_rejects_bad_members(ctx, vr, case):
    # a particle listed twice, or an index outside [0, n), is an error raised
    # before any kernel reads through the member list; R stays untouched
    P, hoff, hmem = case["P"], case["hoff"], case["hmem"]
    z = torch.zeros(3 * P.n, dtype=torch.float32, device="cuda")
    s = torch.ones(6 * P.n, dtype=torch.float32, device="cuda")
    m = np.asarray(hmem).copy()
    for bad in (np.r_[m[:1], m[:-1]], np.r_[m[:-1], P.n], np.r_[-1, m[1:]]):
        R = torch.full((P.n,), 7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(vr.VrError, match="twice or outside"):
            ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(bad.astype(np.int32)), z, s, 8, 4, R=R)
        assert bool((R == 7.0).all())


def test_local_vdensity_end_to_end(ctx, ref, case):
    P, Pr, hoff, hmem = case["P"], case["Pr"], case["hoff"], case["hmem"]
    cm = ref.cell_moments(Pr, hoff, hmem)
    exp = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], 32, 8)["R"]
    dh, dm = dev_tensor(hoff), dev_tensor(hmem)
    gm = ctx.cell_moments(P, dh, dm, want_table=False)
    got = ctx.local_vdensity(P, dh, dm, gm["vbar"], gm["sigma"], 32, 8).cpu().numpy()
    _R_close(got, exp)


def test_local_vdensity_subset_and_other_sizes(ctx, ref, case):
    P, Pr, hoff, hmem = case["P"], case["Pr"], case["hoff"], case["hmem"]
    cm = ref.cell_moments(Pr, hoff, hmem)
    rng = np.random.default_rng(3)
    sub = np.sort(rng.choice(hmem, size=min(500, len(hmem)), replace=False)).astype(np.int32)
    rng.shuffle(sub)
    for n_se, n_v in [(32, 8), (16, 4), (48, 16), (20, 5), (33, 7), (63, 9), (9, 2)]:
        exp = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], n_se, n_v, subset=sub)["R"]
        got = ctx.local_vdensity(P, dev_tensor(hoff), dev_tensor(hmem), dev_tensor(cm["vbar"]),
                                 dev_tensor(cm["sigma"]), n_se, n_v, subset=dev_tensor(sub)).cpu().numpy()
        _R_close(got, exp)
        untouched = np.ones(P.n, bool)
        untouched[sub] = False
        assert np.isnan(got[untouched]).all()


def test_fof6d_parity(ctx, ref, case):
    P, Pr, hoff, hmem, host_of = case["P"], case["Pr"], case["hoff"], case["hmem"], case["host_of"]
    w = case["w"]
    cm = ref.cell_moments(Pr, hoff, hmem)
    R = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], 32, 8)["R"]
    ellv = ref.host_ellv(Pr, hoff, hmem, 1.25)
    ellxs = 0.5 * w.params["ellx"]
    for RR in (R, None):
        exp = ref.fof6d(Pr, host_of, ellv, ellxs, RR, 2.0)
        got = ctx.fof6d(P, dev_tensor(host_of), dev_tensor(ellv), ellxs,
                        None if RR is None else dev_tensor(RR), 2.0).cpu().numpy()
        assert (got == exp).all()


def _unbind_case(seed, n_groups, n_max, masses=False):
    w = synth.unbind_groups(seed=seed, n_groups=n_groups, n_max=n_max)
    if masses:
        rng = np.random.default_rng(seed)
        w.mass = rng.uniform(0.5, 1.5, w.n).astype(np.float32) * np.float32(w.mass_value)
    return w


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("seed,ng,nmax,masses,frame", [(3, 40, 4000, False, 1), (4, 25, 3000, True, 1),
                                                        (5, 25, 3000, False, 0)])
def test_unbind_parity(ctx, vr, ref, seed, ng, nmax, masses, frame, persistent):
    w = _unbind_case(seed, ng, nmax, masses)
    P, Pr = both(ctx, vr, ref, w)
    off, mem = w.groups
    G, eps = w.params["G"], w.params["eps"]
    exp = ref.unbind(Pr, off, mem, G, eps, frame_type=frame)
    got = ctx.unbind(P, dev_tensor(off), dev_tensor(mem), G, eps, frame_type=frame, persistent=persistent)
    _check_unbind(w, exp, got)


def _check_unbind(w, exp, got):
    off, mem = w.groups
    gb, gphi, git = (got[k].cpu().numpy() for k in ("bound", "phi", "iters"))
    clean = exp["min_margin"] > 1e-5
    assert clean.mean() > 0.8
    for g in np.nonzero(clean)[0]:
        m = mem[off[g]:off[g + 1]]
        assert (gb[m] == exp["bound"][m]).all(), g
        assert git[g] == exp["iters"][g], g
        e = exp["phi"][m]
        fin = np.isfinite(e)
        assert (np.isfinite(gphi[m]) == fin).all()
        np.testing.assert_allclose(gphi[m][fin], e[fin], rtol=1e-5)
    con = w.meta["is_contaminant"]
    assert (gb[con] == 0).all()


@pytest.mark.parametrize("persistent", [0, 1])
def test_unbind_not_converged(ctx, vr, ref, persistent):
    w = _unbind_case(3, 3, 800)
    P, _ = both(ctx, vr, ref, w)
    off, mem = w.groups
    with pytest.raises(vr.VrError) as e:
        ctx.unbind(P, dev_tensor(off), dev_tensor(mem), w.params["G"], w.params["eps"], max_iter=1,
                   persistent=persistent)
    assert e.value.code == vr.VR_ERR_NOT_CONVERGED


@pytest.mark.parametrize("order", ["largest_first", "largest_last"])
def test_unbind_wide_groups_in_either_order(ctx, vr, ref, order):
    """Groups of 4096 or more members take 1024-thread group passes while they
    lead the table (the pipeline's size order); after a smaller group they
    take the 256-thread passes.  Both orders match the oracle group by group."""
    w = synth.unbind_groups(seed=8, sizes=[3600, 40, 4000, 300, 25, 120, 3500, 60])
    off, mem = w.groups
    sizes = np.diff(off)
    assert (sizes >= 4096).sum() >= 2
    idx = np.argsort(-sizes, kind="stable")
    if order == "largest_last":
        idx = idx[::-1]
    parts = [mem[off[g]:off[g + 1]] for g in idx]
    off2 = np.concatenate([[0], np.cumsum([len(q) for q in parts])]).astype(off.dtype)
    mem2 = np.concatenate(parts).astype(mem.dtype)
    w2 = dataclasses.replace(w, groups=(off2, mem2))
    P, Pr = both(ctx, vr, ref, w2)
    G, eps = w.params["G"], w.params["eps"]
    exp = ref.unbind(Pr, off2, mem2, G, eps)
    got = ctx.unbind(P, dev_tensor(off2), dev_tensor(mem2), G, eps, persistent=1)
    _check_unbind(w2, exp, got)


@pytest.mark.parametrize("wide", [256, 1 << 30])
def test_unbind_size_class_knob(ctx, vr, ref, wide):
    """The size-class knob moves the cut between the 1024- and 256-thread
    group passes (256: every leading group of >= 256 members is wide; 2^30:
    none is); the bound sets match the oracle either way, and values outside
    the knob's range are refused."""
    w = synth.unbind_groups(seed=8, sizes=[3600, 4000, 3500, 300, 120, 60, 40, 25])
    off, mem = w.groups
    P, Pr = both(ctx, vr, ref, w)
    G, eps = w.params["G"], w.params["eps"]
    exp = ref.unbind(Pr, off, mem, G, eps)
    saved = ctx.get_tune("unbind_wide")
    try:
        ctx.tune("unbind_wide", wide)
        assert ctx.get_tune("unbind_wide") == wide
        got = ctx.unbind(P, dev_tensor(off), dev_tensor(mem), G, eps, persistent=1)
    finally:
        ctx.tune("unbind_wide", saved)
    _check_unbind(w, exp, got)
    for bad in (255, (1 << 30) + 1):
        with pytest.raises(vr.VrError) as e:
            ctx.tune("unbind_wide", bad)
        assert e.value.code == vr.VR_ERR_INVALID_ARG
    assert ctx.get_tune("unbind_wide") == saved


def test_unbind_persistent_launch_shapes_and_graph_reuse(ctx, vr, ref):
    """The persistent path with work items split into several j-ranges,
    small tiles and few workgroups per CU, called twice in a row with the
    same arguments (cached graph replayed) and then on a smaller group set
    (graph captured again); every call matches the oracle."""
    w = _unbind_case(6, 30, 5000)
    P, Pr = both(ctx, vr, ref, w)
    off, mem = w.groups
    G, eps = w.params["G"], w.params["eps"]
    exp = ref.unbind(Pr, off, mem, G, eps)
    saved = {k: ctx.get_tune(k) for k in ("unbind_jchunk", "unbind_bpc")}
    try:
        ctx.tune("unbind_jchunk", 256)
        ctx.tune("unbind_bpc", 1)
        offd, memd = dev_tensor(off), dev_tensor(mem)
        for _ in range(2):
            _check_unbind(w, exp, ctx.unbind(P, offd, memd, G, eps, tile=64))
        ng2 = 7
        off2, mem2 = off[:ng2 + 1].copy(), mem[:off[ng2]].copy()
        exp2 = ref.unbind(Pr, off2, mem2, G, eps)
        got2 = ctx.unbind(P, dev_tensor(off2), dev_tensor(mem2), G, eps, tile=64)
        w2 = dataclasses.replace(w, groups=(off2, mem2), meta=dict(w.meta, is_contaminant=np.zeros(w.n, bool)))
        _check_unbind(w2, exp2, got2)
        assert (got2["bound"].cpu().numpy()[mem[off[ng2]:]] == 0).all()
    finally:
        for k, v in saved.items():
            ctx.tune(k, v)


def test_unbind_persistent_matches_host_planned(ctx, vr, ref):
    """Both schedules run the same passes: identical bound flags and pass
    counts; potentials equal to the FP32 tile error (the persistent schedule
    subtracts the removed members' terms where the host-planned one
    recomputes the sums)."""
    w = _unbind_case(7, 60, 3000)
    P, _ = both(ctx, vr, ref, w)
    off, mem = w.groups
    G, eps = w.params["G"], w.params["eps"]
    a = ctx.unbind(P, dev_tensor(off), dev_tensor(mem), G, eps, persistent=0)
    b = ctx.unbind(P, dev_tensor(off), dev_tensor(mem), G, eps, persistent=1)
    assert torch.equal(a["bound"], b["bound"])
    assert torch.equal(a["iters"], b["iters"])
    pa, pb = a["phi"].cpu().numpy(), b["phi"].cpu().numpy()
    assert (np.isfinite(pa) == np.isfinite(pb)).all()
    f = np.isfinite(pa)
    np.testing.assert_allclose(pb[f], pa[f], rtol=2e-6)


@pytest.mark.parametrize("name", list(CASES))
def test_field_halos_6d_pipeline_parity(ctx, vr, ref, name):
    """Field halos by adaptive 6D FOF (each 3D group re-linked with its own
    alpha_v sigma_v and the full ellx), then the substructure search on
    them: labels and group tables bit-exact, R within its tolerance."""
    from oracle import pipeline as opipe
    from paper_1902_01010_amd import pipeline
    w = CASES[name]()
    prm = dataclasses.replace(pipeline.Params.from_workload(w), field_6d=True)
    exp = opipe.run(w, prm)
    x, v, m = pipeline.device_inputs(w)
    got, _ = pipeline.run(ctx, x, v, m, w.mass_value, w.box, w.grid_bits, prm)
    assert (got["label3d"].cpu().numpy() == exp["label3d"]).all()
    assert (got["label"].cpu().numpy() == exp["label"]).all()
    assert got["n_groups"] == exp["n_groups"]
    ng = exp["n_groups"]
    np.testing.assert_array_equal(got["offsets"].cpu().numpy()[:ng + 1], exp["offsets"][:ng + 1])
    np.testing.assert_array_equal(got["members"].cpu().numpy()[:exp["offsets"][ng]], exp["members"][:exp["offsets"][ng]])
    # 6D only splits 3D groups: never more particles grouped, and every 6D
    # group lies inside one 3D group
    _, c3 = np.unique(exp["label3d"], return_counts=True)
    assert exp["offsets"][ng] <= c3[c3 >= 20].sum()
    lab3 = exp["label3d"]
    for g in range(ng):
        mm = exp["members"][exp["offsets"][g]:exp["offsets"][g + 1]]
        assert (lab3[mm] == lab3[mm[0]]).all()
    if exp["n_hosts"]:
        _R_close(got["R"].cpu().numpy(), exp["R"])


@pytest.mark.parametrize("seed", [21, 22])
def test_fof6d_dense_cells_bit_exact(ctx, vr, ref, seed):
    """Cells holding hundreds of participants: their tiles run first, many
    tiles of one cell merge the same core, and the candidate mask leaves
    out pairs already joined.  One clump is a single velocity population;
    the other holds two populations 10 units apart in velocity (ellv 2),
    which must stay two groups; sparse participants and non-participants
    around them.  Bit-exact against the oracle, with and without R."""
    rng = np.random.default_rng(seed)
    size = 1 << 21
    n_c = 4000
    ca = rng.normal(0.0, 600.0, (3, n_c)) + size * 0.3
    cb = rng.normal(0.0, 600.0, (3, n_c)) + size * 0.6
    sp = rng.uniform(0.25 * size, 0.65 * size, (3, 3000))
    q = np.mod(np.rint(np.concatenate([ca, cb, sp], axis=1)), size).astype(np.uint32)
    n = q.shape[1]
    v = rng.normal(0.0, 1.0, (3, n))
    v[0, n_c:n_c + n_c // 2] += 5.0
    v[0, n_c + n_c // 2:2 * n_c] -= 5.0
    v = v.astype(np.float32)
    host_of = np.zeros(n, np.int32)
    host_of[2 * n_c + 2000:] = -1  # some sparse particles outside every host
    Pd = vr.Particles(dev_tensor(q.view(np.int32)), dev_tensor(v), None, 1.0, 1.0, 21)
    Pr = ref.Particles(q, v, None, 1.0, 1.0, 21)
    ellv = np.array([2.0])
    ellxs = 500.0 / size
    R = rng.uniform(0.0, 4.0, n).astype(np.float32)
    for RR in (None, R):
        exp = ref.fof6d(Pr, host_of, ellv, ellxs, RR, 2.0)
        got = ctx.fof6d(Pd, dev_tensor(host_of), dev_tensor(ellv), ellxs, None if RR is None else dev_tensor(RR),
                        2.0).cpu().numpy()
        assert (got == exp).all()
        if RR is None:
            # every hosted particle takes part: clump a, and clump b's two
            # velocity populations
            ids, cnt = np.unique(exp[exp >= 0], return_counts=True)
            assert (cnt > 1000).sum() >= 3


def test_new_snapshot_drops_kept_sorts(vr):
    """Two builds over the same content share one set of sorted lists; after
    vr_new_snapshot the next build sorts again (counted in radix passes)."""
    c = vr.Context(0)
    w = synth.isolated_halo(seed=5, n_host=5000, n_sub=1, sub_range=(400, 500))
    P = gpu_particles(vr, c.quantize(dev_tensor(w.x), w.box, w.grid_bits), w)
    dh = dev_tensor(np.array([0, w.n], np.int32))
    dm = dev_tensor(np.arange(w.n, dtype=np.int32))

    def passes(fn):
        c.set_timing(True)
        fn()
        c.sync()
        n = c.kernel_time("radix_scatter")[0]
        c.set_timing(False)
        return n

    first = passes(lambda: c.cell_moments(P, dh, dm))
    again = passes(lambda: c.cell_moments(P, dh, dm))
    c.new_snapshot()
    fresh = passes(lambda: c.cell_moments(P, dh, dm))
    assert first > 0 and fresh == first
    assert again < first


def test_presort_reuse_follows_content(ctx, vr, ref):
    """The context reuses the sorted member lists of its last KD build only
    for the same content: R over the same tensors after their coordinates
    changed in place still matches the oracle on the changed inputs, and so
    does R after one member was swapped for another particle (same count,
    other content)."""
    w = synth.isolated_halo(seed=7, n_host=6000, n_sub=2, sub_range=(400, 800))
    P, Pr = both(ctx, vr, ref, w)
    lab = ref.fof3d(Pr, w.params["ellx"])
    _, _, off, mem = ref.groups(lab, 20)
    hoff, hmem = off[:2].copy(), mem[:off[1]].copy()
    dh, dm = dev_tensor(hoff), dev_tensor(hmem)
    for step in range(3):
        gm = ctx.cell_moments(P, dh, dm)
        got = ctx.local_vdensity(P, dh, dm, gm["vbar"], gm["sigma"], 32, 8).cpu().numpy()
        cm = ref.cell_moments(Pr, hoff, hmem)
        exp = ref.local_vdensity(Pr, hoff, hmem, cm["vbar"], cm["sigma"], 32, 8)["R"]
        _R_close(got, exp)
        if step == 0:
            # move some members by a few grid units, in place
            q = Pr.q.copy()
            idx = hmem[::7]
            q[0, idx] = (q[0, idx] + 3) % (1 << w.grid_bits)
            Pr = ref.Particles(q, w.v, w.mass, w.mass_value, w.box, w.grid_bits)
            P.q.copy_(dev_tensor(q.view(np.int32)))
        elif step == 1:
            # as many members, one of them another particle
            outside = np.setdiff1d(np.arange(P.n, dtype=np.int32), hmem)
            hmem = hmem.copy()
            hmem[len(hmem) // 2] = outside[len(outside) // 2]
            hmem.sort()
            dm.copy_(dev_tensor(hmem))
