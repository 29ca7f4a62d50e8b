"""The hot path end to end through the CPU oracle (test infrastructure):
same chain of steps as the GPU pipeline, every step an oracle call."""
from __future__ import annotations

import numpy as np

import oracle as ref


def run(w, prm, timings=None, is_baryon=None):
    import time

    def tick(name, t0):
        if timings is not None:
            timings[name] = time.perf_counter() - t0
        return time.perf_counter()

    t = time.perf_counter()
    q = ref.quantize(w.x, w.box, w.grid_bits)
    P = ref.Particles(q, w.v, w.mass, w.mass_value, w.box, w.grid_bits)
    t = tick("quantize", t)
    label = ref.fof3d(P, prm.ellx) if is_baryon is None else ref.fof3d_dm(P, prm.ellx, is_baryon)
    t = tick("fof3d", t)
    ng, group_of, off, mem = ref.groups(label, prm.n_min)
    label3d = label
    if getattr(prm, "field_6d", False) and ng > 0:
        # field halos (Sec. 2.1, Eq. fof6d): each 3D group re-linked in 6D
        # with ell_v = alpha_v sigma_v of that group and the full ellx
        ellv3 = ref.host_ellv(P, off, mem, prm.alpha_v)
        label = ref.fof6d(P, group_of, ellv3, prm.ellx, None)
        t = tick("field6d", t)
        ng, group_of, off, mem = ref.groups(label, prm.n_min)
    sizes = np.diff(off)
    nh = int((sizes >= prm.host_min).sum())
    hoff, hmem = off[:nh + 1], mem[:off[nh]]
    t = tick("groups", t)
    out = dict(q=q, label=label, label3d=label3d, n_groups=ng, group_of=group_of, offsets=off, members=mem,
               n_hosts=nh)
    if nh == 0:
        return out
    species = None
    if is_baryon is not None:
        # the substructure search runs on the hosts' dark matter
        species = (hoff, hmem, is_baryon)
        keep = is_baryon[hmem] == 0
        hmem = hmem[keep]
        hoff = np.r_[0, np.cumsum(np.add.reduceat(keep, hoff[:-1]))].astype(np.int32)
    res = search(P, group_of, nh, hoff, hmem, prm, tick, species)
    out.update(res)
    # the activity chart of the substructure search (Sec. 2.2): substructures
    # with enough bound members are searched again as hosts, level by level
    out["levels"] = []
    for _lev in range(2, getattr(prm, "levels", 1) + 1):
        if res["unbind"] is None:
            break
        lb = np.where(res["unbind"]["bound"] > 0, res["label6"], -1).astype(np.int32)
        nh2, g2, off2, mem2 = ref.groups(lb, prm.host_min)
        if nh2 == 0:
            break
        res = search(P, g2, nh2, off2, mem2, prm, None, None)
        res.update(n_hosts=nh2, host_group_of=g2, host_members=mem2, host_offsets=off2)
        out["levels"].append(res)
    return out


def search(P, group_of, nh, hoff, hmem, prm, tick=None, species=None):
    """One level of the substructure search (Sec. 2.2) over the hosts
    [0, nh) of group_of, members hoff/hmem: background by cells, R, the
    outliers linked, candidates unbound; species = (host offsets and members
    over both species, is_baryon) adds the baryon assignment (Sec. 2.4)."""
    import time
    if tick is None:
        def tick(name, t0):
            return time.perf_counter()
    t = time.perf_counter()
    cm = ref.cell_moments(P, hoff, hmem)
    t = tick("cells", t)
    R = ref.local_vdensity(P, hoff, hmem, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v)["R"]
    t = tick("R", t)
    ellv = ref.host_ellv(P, hoff, hmem, prm.alpha_v)
    ell = None
    if getattr(prm, "use_ell", False):
        # L = (R - Rbar) / sigma_R from each host's skew-Gaussian fit (Eqs.
        # skewgaus, ell); outliers are L >= ell_th
        ell = ref.ell_fit(R, hoff, hmem)["ell"]
        t = tick("ell", t)
        if getattr(prm, "linker", "6d") == "paper":
            # the paper's linker over L >= ell_th (Eq. linkingcriteria)
            host_of = np.where((group_of >= 0) & (group_of < nh), group_of, -1).astype(np.int32)
            label6 = ref.fof_sub(P, host_of, nh, cm["vbar"], prm.alpha_xs * prm.ellx, ell, prm.ell_th, prm.Vr,
                                 theta_op=prm.theta_op)
            if getattr(prm, "sub_grow", False):
                # the relaxed second stage: growth and joins
                label6, _ = ref.sub_grow(P, host_of, nh, cm["vbar"], ell, label6, prm.alpha_xs * prm.ellx,
                                         prm.ell_th, prm.gamma_L, prm.gamma_x, prm.Vr, prm.gamma_Vr, prm.theta_op,
                                         prm.gamma_theta, prm.f_merge, prm.n_min)
        else:
            label6 = ref.fof6d(P, group_of, ellv, prm.alpha_xs * prm.ellx, ell, prm.ell_th)
        t = tick("fof6d", t)
        nc, sub_of, sub_off, sub_mem = ref.groups(label6, prm.n_min)
        # significance cleaning of the candidates (Eq. ellsig)
        label6, _ = ref.ell_clean(ell, sub_off, sub_mem, label6, prm.ell_th, prm.beta_ell, prm.n_min)
        t = tick("clean", t)
    else:
        label6 = ref.fof6d(P, group_of, ellv, prm.alpha_xs * prm.ellx, R, prm.R_threshold)
        t = tick("fof6d", t)
    if species is not None:
        hoff_all, hmem_all, is_baryon = species
        # baryons take the candidate of the nearest dark matter in phase space
        lab = np.asarray(label6)
        cnt = np.bincount(lab[lab >= 0], minlength=P.n)
        sub = np.where((lab >= 0) & (cnt[np.maximum(lab, 0)] >= prm.n_min), lab, -1).astype(np.int32)
        w_dm = np.diff(hoff).astype(np.float64)
        sv = prm.baryon_sigma_v if prm.baryon_sigma_v > 0 else float(np.sum(w_dm * ellv) / np.sum(w_dm)) / prm.alpha_v
        lab_all = ref.assign_baryons(P, hoff_all, hmem_all, is_baryon, sub, prm.ellx, sv,
                                     out_init=np.full(P.n, -1, np.int32))
        # canonical labels: the smallest member of each candidate
        low = np.full(P.n, P.n, np.int64)
        ok = lab_all >= 0
        np.minimum.at(low, lab_all[ok], np.nonzero(ok)[0])
        label6 = np.where(ok, low[np.maximum(lab_all, 0)], -1).astype(np.int32)
        t = tick("baryons", t)
    nc, sub_of, sub_off, sub_mem = ref.groups(label6, prm.n_min)
    t = tick("subgroups", t)
    ub = ref.unbind(P, sub_off, sub_mem, prm.G, prm.eps, beta_E=prm.beta_E, n_min=prm.n_min) if nc else None
    tick("unbind", t)
    return dict(cells=cm, R=R, ell=ell, ellv=ellv, label6=label6, n_candidates=nc, sub_offsets=sub_off,
                sub_members=sub_mem, unbind=ub)
