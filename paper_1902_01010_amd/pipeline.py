"""The hot path end to end on the GPU: quantise -> 3D FOF -> groups -> KD
cells and moments -> R -> host velocity linking lengths -> 6D FOF over the
outliers -> candidate groups -> unbinding.  Every step is a libvr call;
this module only chains them and selects the searched hosts.

With a trained surrogate model, R comes from the learned path instead:
features -> network -> band selection -> exact R for the band only.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import vr as _vr

KERNELS = ("radix_scatter", "fof_link3d", "kd_level", "knn", "fof_link6d", "unbind_potential", "unbind_group",
           "unbind_persistent", "rs_features", "mlp_forward", "ell_fit", "ell_clean",
           "fof_link_sub", "sub_grow", "fof_attach", "assign_baryons")


@dataclasses.dataclass
class Params:
    ellx: float
    n_se: int = 32
    n_v: int = 8
    R_threshold: float = 2.0
    alpha_v: float = 1.25
    alpha_xs: float = 0.5
    eps: float = 0.0
    G: float = 4.30091e-9
    beta_E: float = 0.95
    n_min: int = 20
    host_min: int = 256
    field_6d: bool = False   # field halos by adaptive 6D FOF inside each 3D group (Sec. 2.1, Eq. fof6d)
    # outliers by the normalised ratio L >= ell_th (Sec. 2.2, Eq. ell) instead
    # of R >= R_threshold, and significance cleaning of the 6D groups with
    # beta_L (Eq. ellsig)
    use_ell: bool = False
    ell_th: float = 2.5
    beta_ell: float = 1.0
    # "6d": Eq. fof6d over the outliers; "paper": the paper's substructure
    # linker (Sec. 2.2, Eq. linkingcriteria; needs use_ell): speed ratio Vr
    # and opening angle theta_op about the local mean velocity
    linker: str = "6d"
    Vr: float = 2.0
    theta_op: float = math.pi / 10
    # the paper's second, relaxed stage (Sec. 2.2): candidates grow through
    # links with L >= ell_th / gamma_L, linking length gamma_x alpha_xs ellx,
    # speed ratio gamma_Vr Vr, angle gamma_theta theta_op; groups join when
    # their relaxed links exceed f_merge of either's first-stage size
    sub_grow: bool = True
    gamma_L: float = 1.0
    gamma_x: float = 2.0
    gamma_Vr: float = 1.0
    gamma_theta: float = 1.0
    f_merge: float = 0.25
    # two species (DM+Baryons mode, Sec. 2.1 and 2.4): baryons never start
    # 3D links, the substructure search runs on the dark matter, and baryons
    # join the substructure of the nearest dark matter in phase space with
    # this sigma_v (0: the hosts' sigma_v weighted by their dark matter)
    baryon_sigma_v: float = 0.0
    # levels of the substructure search: the bound substructures of level l
    # with >= host_min members are searched in turn as hosts of level l+1
    # (Sec. 2.2, activity chart of the substructure search); one process
    # per level, the parameters the same at every level
    levels: int = 1

    @classmethod
    def from_workload(cls, w):
        keys = {f.name for f in dataclasses.fields(cls)}
        return cls(**{k: v for k, v in w.params.items() if k in keys})


def device_inputs(w, device="cuda"):
    x = torch.from_numpy(np.ascontiguousarray(w.x)).to(device)
    v = torch.from_numpy(np.ascontiguousarray(w.v)).to(device)
    m = None if w.mass is None else torch.from_numpy(np.ascontiguousarray(w.mass)).to(device)
    return x, v, m


def surrogate_R(ctx, P, host_offsets, members, cm, prm: Params, model):
    """R of every host member by the learned path: the network's prediction,
    replaced by the exact R inside the band |Rhat - R_threshold| < margin."""
    feat = ctx.rs_features(P, host_offsets, members, cm["vbar"], cm["sigma"], cm["rho_cell"], prm.n_se,
                           model.cell_bits, model.shift, model.scale)
    m = feat.shape[0]
    rhat = ctx.mlp_forward(model.weights, feat)
    R = torch.full((P.n,), float("nan"), device=P.device)
    band = ctx.rs_select(members[:m], rhat, R, prm.R_threshold, model.margin)
    if band.shape[0] > 0:
        ctx.local_vdensity(P, host_offsets, members, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v, subset=band, R=R)
    return R, dict(rhat=rhat, n_band=int(band.shape[0]), n_rows=m)


def run(ctx: _vr.Context, x, v, mass, mass_value, box, grid_bits, prm: Params, stage_events=False, model=None,
        until=None, is_baryon=None):
    """One pass of the hot path over device-resident inputs (R from the
    learned path when a surrogate model is given; until="R" stops after R;
    is_baryon, a uint8 device flag per particle, selects the two-species
    mode).  Returns the outputs (device tensors) and counts."""
    if prm.levels > 1 and is_baryon is not None:
        raise ValueError("levels > 1 runs on one species only")
    ev = []

    def mark(name):
        if stage_events:
            e = torch.cuda.Event(enable_timing=True)
            e.record()
            ev.append((name, e))

    ctx.new_snapshot()
    mark("start")
    q = ctx.quantize(x, box, grid_bits)
    P = _vr.Particles(q, v, mass, mass_value, box, grid_bits)
    mark("quantize")
    label = ctx.fof3d(P, prm.ellx) if is_baryon is None else ctx.fof3d_dm(P, prm.ellx, is_baryon)
    mark("fof3d")
    ng, group_of, offsets, members = ctx.groups(label, prm.n_min)
    label3d = label
    if prm.field_6d and ng > 0:
        # every 3D group is re-linked in 6D with its own velocity scale
        # alpha_v sigma_v,k and the full ellx; the 6D groups are the halos
        ellv3 = ctx.host_ellv(P, offsets[:ng + 1], members, prm.alpha_v)
        label = ctx.fof6d(P, group_of, ellv3, prm.ellx, None)
        mark("field6d")
        ng, group_of, offsets, members = ctx.groups(label, prm.n_min)
    sizes = np.diff(offsets.cpu().numpy())
    n_hosts = int((sizes >= prm.host_min).sum())
    host_offsets = offsets[:n_hosts + 1]
    mark("groups")
    out = dict(q=q, label=label, label3d=label3d, n_groups=ng, group_of=group_of, offsets=offsets, members=members,
               n_hosts=n_hosts, n_searched=int(sizes[:n_hosts].sum()))
    if n_hosts == 0:
        out["R"] = torch.full((P.n,), float("nan"), device=x.device)
        return out, ev
    species = None
    if is_baryon is not None:
        # the substructure search runs on the hosts' dark matter
        species = (offsets[:n_hosts + 1], members, is_baryon)
        host_offsets, members = ctx.select_members(P.n, host_offsets, members[:int(sizes[:n_hosts].sum())], is_baryon)
        out.update(host_offsets_all=offsets[:n_hosts + 1], search_members=members,
                   n_searched=int(host_offsets[-1].item()))
    lev1 = _search(ctx, P, group_of, n_hosts, host_offsets, members, prm, mark, "", model, until, species)
    out.update(lev1)
    if until == "R":
        return out, ev
    out["levels"] = []
    res = lev1
    for lev in range(2, prm.levels + 1):
        if res["unbind"] is None:
            break
        # hosts of the next level: the bound members of this level's
        # substructures, where >= host_min of them remain
        lb = torch.where(res["unbind"]["bound"] > 0, res["label6"], torch.full_like(res["label6"], -1))
        nh, g_of, h_off, h_mem = ctx.groups(lb, prm.host_min)
        mark(f"L{lev}:groups")
        if nh == 0:
            break
        res = _search(ctx, P, g_of, nh, h_off, h_mem, prm, mark, f"L{lev}:")
        res.update(n_hosts=nh, host_group_of=g_of, host_members=h_mem)
        out["levels"].append(res)
    return out, ev


def _search(ctx, P, group_of, n_hosts, host_offsets, members, prm: Params, mark, tag, model=None, until=None,
            species=None):
    """One level of the substructure search over the hosts [0, n_hosts) of
    group_of (members in host_offsets/members): the background by cells,
    R (or the learned path), the outliers linked into candidates, and the
    candidates unbound.  species = (host offsets over both species, their
    members, is_baryon) adds the baryon assignment before unbinding."""
    out = {}
    # nothing downstream reads a member's cell index
    cm = ctx.cell_moments(P, host_offsets, members, want_table=False, want_cell_of=False)
    mark(tag + "cells")
    if model is None:
        R = ctx.local_vdensity(P, host_offsets, members, cm["vbar"], cm["sigma"], prm.n_se, prm.n_v)
    else:
        R, out["surrogate"] = surrogate_R(ctx, P, host_offsets, members, cm, prm, model)
    mark(tag + "R")
    out.update(cells=cm, R=R, host_offsets=host_offsets)
    if until == "R":
        return out
    ellv = ctx.host_ellv(P, host_offsets, members, prm.alpha_v)
    if prm.use_ell:
        # L from each host's skew-Gaussian fit of R; 6D groups over L >= ell_th,
        # cleaned by their mean L
        ef = ctx.ell_fit(R, host_offsets, members)
        out.update(ell=ef["ell"], ell_fit=ef["fit"], ell_status=ef["status"], ell_merge=ef["merge"])
        mark(tag + "ell")
        if prm.linker == "paper":
            label6 = ctx.fof_sub(P, group_of, n_hosts, cm["vbar"], prm.alpha_xs * prm.ellx, ef["ell"], prm.ell_th,
                                 prm.Vr, prm.theta_op)
            if prm.sub_grow:
                label6, out["grow_rounds"] = ctx.sub_grow(
                    P, group_of, n_hosts, cm["vbar"], ef["ell"], label6, prm.alpha_xs * prm.ellx, prm.ell_th,
                    prm.gamma_L, prm.gamma_x, prm.Vr, prm.gamma_Vr, prm.theta_op, prm.gamma_theta, prm.f_merge,
                    prm.n_min)
        else:
            label6 = ctx.fof6d(P, group_of, ellv, prm.alpha_xs * prm.ellx, ef["ell"], prm.ell_th)
        mark(tag + "fof6d")
        nc, sub_of, sub_off, sub_mem = ctx.groups(label6, prm.n_min)
        if nc > 0:
            ctx.ell_clean(ef["ell"], sub_off, sub_mem, label6, prm.ell_th, prm.beta_ell, prm.n_min)
        mark(tag + "clean")
    else:
        label6 = ctx.fof6d(P, group_of, ellv, prm.alpha_xs * prm.ellx, R, prm.R_threshold)
        mark(tag + "fof6d")
    if species is not None:
        host_offsets_all, all_members, is_baryon = species
        # baryons join the candidate of the nearest dark matter in phase space
        sub = ctx.relabel_min(label6, prm.n_min)
        # sigma_v <= 0: the library takes the typical sigma_v of a searched
        # particle's host, the mean over hosts of (det Sigma_H)^(1/6) weighted
        # by their dark matter
        lab_all, sv = ctx.assign_baryons(P, host_offsets_all, all_members, is_baryon, sub, prm.ellx,
                                         prm.baryon_sigma_v, ellv_host=ellv, alpha_v=prm.alpha_v)
        label6 = ctx.relabel_min(lab_all, 1)
        out.update(baryon_sigma_v=sv, label6_dm=sub)
        mark(tag + "baryons")
    nc, sub_of, sub_off, sub_mem = ctx.groups(label6, prm.n_min)
    mark(tag + "subgroups")
    ub = ctx.unbind(P, sub_off, sub_mem, prm.G, prm.eps, beta_E=prm.beta_E, n_min=prm.n_min) if nc > 0 else None
    mark(tag + "unbind")
    out.update(ellv=ellv, label6=label6, n_candidates=nc, sub_offsets=sub_off,
               sub_members=sub_mem, unbind=ub)
    return out


def stage_times(ev):
    """Milliseconds between consecutive stage markers."""
    torch.cuda.synchronize()
    return {ev[k][0]: ev[k - 1][1].elapsed_time(ev[k][1]) for k in range(1, len(ev))}
