"""CPU oracle of the phase-space halo-finder hot path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 reference written from the paper
(Elahi et al., VELOCIraptor, Sec. 2).  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the GPU library never does,
and the two share no code.

`libvr_ref.so` is built from `vr_ref.cpp` by :func:`build` (g++, no
fast-math, no FP contraction).  The functions below marshal numpy arrays into
the C calls and return numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vr_ref.cpp")
_LIB = os.path.join(_HERE, "libvr_ref.so")

BUILD_CMD = ["g++", "-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off",
             "-shared", "-fPIC", "-pthread", _SRC, "-o", _LIB]


def build() -> str:
    """Compile the oracle library in place and return its path."""
    subprocess.check_call(BUILD_CMD)
    return _LIB


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64),
                ("qx", C.c_void_p), ("qy", C.c_void_p), ("qz", C.c_void_p),
                ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("mass", C.c_void_p), ("mass_value", C.c_double),
                ("box", C.c_double), ("grid_bits", C.c_int32)]


class _CellParams(C.Structure):
    _fields_ = [("f_cell", C.c_double), ("ncell_floor", C.c_int32), ("ncell_div", C.c_int32),
                ("nbins", C.c_int32), ("split_rule", C.c_int32)]


class _EllParams(C.Structure):
    _fields_ = [("lo", C.c_double), ("width", C.c_double), ("nbins", C.c_int32), ("peak_min", C.c_int32),
                ("max_merge", C.c_int32), ("golden_iters", C.c_int32)]


# fine grid of 1024 bins of 1/32 on [-16, 16); merge to >= 32 in the fullest
# bin (factor <= 64); 48 golden-section steps
ELL_DEFAULTS = dict(lo=-16.0, width=1.0 / 32, nbins=1024, peak_min=32, max_merge=64, golden_iters=48)


class _UnbindParams(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("beta_E", C.c_double),
                ("frac_ref", C.c_double), ("n_min", C.c_int32), ("n_ref_min", C.c_int32),
                ("frame_type", C.c_int32), ("max_iter", C.c_int32)]


CELL_COLS = 28
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        vp, i64, i32, dbl, flt = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_float
        P = C.POINTER(_Particles)
        L.vr_ref_set_threads.argtypes = [C.c_int]
        L.vr_ref_quantize.argtypes = [i64, vp, vp, vp, dbl, i32, vp, vp, vp]
        L.vr_ref_ell2_grid.argtypes = [dbl, dbl, i32]
        L.vr_ref_ell2_grid.restype = dbl
        L.vr_ref_fof3d.argtypes = [P, dbl, vp]
        L.vr_ref_groups.argtypes = [i64, vp, i32, vp, vp, vp, vp]
        L.vr_ref_entropy.argtypes = [i32, vp]
        L.vr_ref_entropy.restype = dbl
        L.vr_ref_cell_moments.argtypes = [P, i32, vp, vp, C.POINTER(_CellParams), vp, vp, vp, vp,
                                          i64, vp, vp]
        L.vr_ref_local_vdensity.argtypes = [P, i32, vp, vp, vp, vp, i32, i32, vp, i64, vp, vp, vp,
                                            vp, vp]
        L.vr_ref_host_ellv.argtypes = [P, i32, vp, vp, dbl, vp]
        L.vr_ref_fof6d.argtypes = [P, vp, i32, vp, dbl, vp, flt, vp]
        L.vr_ref_fof_sub.argtypes = [P, vp, i32, vp, dbl, vp, flt, dbl, dbl, vp]
        L.vr_ref_fof3d_dm.argtypes = [P, dbl, vp, vp]
        L.vr_ref_assign_baryons.argtypes = [P, i32, vp, vp, vp, vp, dbl, dbl, vp]
        L.vr_ref_sub_grow.argtypes = [P, vp, i32, vp, vp, flt, dbl, dbl, dbl, dbl, dbl, dbl, dbl, i32, vp, vp, vp]
        L.vr_ref_unbind.argtypes = [P, i32, vp, vp, C.POINTER(_UnbindParams), vp, vp, vp, vp]
        L.vr_ref_ell_fit.argtypes = [i64, i32, vp, vp, vp, C.POINTER(_EllParams), vp, vp, vp, vp]
        L.vr_ref_ell_cost.argtypes = [i32, vp, vp, dbl, vp]
        L.vr_ref_ell_cost.restype = dbl
        L.vr_ref_ell_mean.argtypes = [dbl]
        L.vr_ref_ell_mean.restype = dbl
        L.vr_ref_ell_clean.argtypes = [i64, i32, vp, vp, vp, dbl, dbl, i32, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def set_threads(n: int) -> int:
    return lib().vr_ref_set_threads(int(n))


class Particles:
    """Host particle set: q (3,n) uint32, v (3,n) float32, optional mass (n,) float32."""

    def __init__(self, q, v, mass, mass_value, box, grid_bits):
        self.q = np.ascontiguousarray(q, dtype=np.uint32)
        self.v = None if v is None else np.ascontiguousarray(v, dtype=np.float32)
        self.mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float32)
        self.mass_value = float(mass_value)
        self.box = float(box)
        self.grid_bits = int(grid_bits)
        n = self.q.shape[1]
        s = _Particles()
        s.n = n
        s.qx, s.qy, s.qz = (self.q[d].ctypes.data_as(C.c_void_p) for d in range(3))
        if self.v is not None:
            s.vx, s.vy, s.vz = (self.v[d].ctypes.data_as(C.c_void_p) for d in range(3))
        s.mass = _p(self.mass)
        s.mass_value = self.mass_value
        s.box = self.box
        s.grid_bits = self.grid_bits
        self.s = s

    @property
    def n(self):
        return self.q.shape[1]


def quantize(x, box, grid_bits):
    x = np.ascontiguousarray(x, dtype=np.float32)
    n = x.shape[1]
    q = np.zeros((3, n), np.uint32)
    _check(lib().vr_ref_quantize(n, _p(x[0]), _p(x[1]), _p(x[2]), float(box), int(grid_bits),
                                 _p(q[0]), _p(q[1]), _p(q[2])), "quantize")
    return q


def ell2_grid(ell, box, grid_bits):
    return lib().vr_ref_ell2_grid(float(ell), float(box), int(grid_bits))


def fof3d(P: Particles, ellx):
    lab = np.zeros(P.n, np.int32)
    _check(lib().vr_ref_fof3d(C.byref(P.s), float(ellx), _p(lab)), "fof3d")
    return lab


def groups(label, n_min):
    label = np.ascontiguousarray(label, dtype=np.int32)
    n = label.shape[0]
    ng = np.zeros(1, np.int32)
    gof = np.zeros(n, np.int32)
    off = np.zeros(n + 1, np.int32)
    mem = np.zeros(max(n, 1), np.int32)
    _check(lib().vr_ref_groups(n, _p(label), int(n_min), _p(ng), _p(gof), _p(off), _p(mem)), "groups")
    g = int(ng[0])
    return g, gof, off[:g + 1].copy(), mem[:off[g]].copy()


def entropy(hist):
    h = np.ascontiguousarray(hist, dtype=np.float64)
    return lib().vr_ref_entropy(h.shape[0], _p(h))


def cell_moments(P: Particles, host_offsets, host_members, f_cell=0.01, ncell_floor=100,
                 ncell_div=8, nbins=16, split_rule=0):
    off = np.ascontiguousarray(host_offsets, dtype=np.int32)
    mem = np.ascontiguousarray(host_members, dtype=np.int32)
    nh = off.shape[0] - 1
    n = P.n
    vbar = np.full((3, n), np.nan, np.float32)
    sig = np.full((6, n), np.nan, np.float32)
    rho = np.full(n, np.nan, np.float32)
    cof = np.full(n, -1, np.int32)
    cp = _CellParams(f_cell, ncell_floor, ncell_div, nbins, split_rule)
    nc = np.zeros(1, np.int64)
    _check(lib().vr_ref_cell_moments(C.byref(P.s), nh, _p(off), _p(mem), C.byref(cp), _p(vbar),
                                     _p(sig), _p(rho), _p(cof), 0, None, _p(nc)), "cell_moments(count)")
    ncell = int(nc[0])
    table = np.zeros((max(ncell, 1), CELL_COLS), np.float64)
    _check(lib().vr_ref_cell_moments(C.byref(P.s), nh, _p(off), _p(mem), C.byref(cp), _p(vbar),
                                     _p(sig), _p(rho), _p(cof), ncell, _p(table), _p(nc)), "cell_moments")
    return dict(vbar=vbar, sigma=sig, rho_cell=rho, cell_of=cof, cells=table[:ncell])


def local_vdensity(P: Particles, host_offsets, host_members, vbar, sigma, n_se, n_v,
                   subset=None, want_sets=False, R_init=None):
    off = np.ascontiguousarray(host_offsets, dtype=np.int32)
    mem = np.ascontiguousarray(host_members, dtype=np.int32)
    nh = off.shape[0] - 1
    n = P.n
    vbar = np.ascontiguousarray(vbar, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    R = np.full(n, np.nan, np.float32) if R_init is None else np.array(R_init, np.float32)
    lnfl = np.full(n, np.nan)
    lnfbg = np.full(n, np.nan)
    sub = None if subset is None else np.ascontiguousarray(subset, dtype=np.int32)
    nproc = int(off[-1]) if sub is None else sub.shape[0]
    ns = np.zeros((max(nproc, 1), n_se), np.int32) if want_sets else None
    nv = np.zeros((max(nproc, 1), n_v), np.int32) if want_sets else None
    _check(lib().vr_ref_local_vdensity(C.byref(P.s), nh, _p(off), _p(mem), _p(vbar), _p(sigma),
                                       int(n_se), int(n_v), _p(sub), 0 if sub is None else sub.shape[0],
                                       _p(R), _p(lnfl), _p(lnfbg), _p(ns), _p(nv)), "local_vdensity")
    out = dict(R=R, lnfl=lnfl, lnfbg=lnfbg)
    if want_sets:
        out["nbr_s"] = ns[:nproc]
        out["nbr_v"] = nv[:nproc]
    return out


def host_ellv(P: Particles, host_offsets, host_members, alpha_v=1.25):
    off = np.ascontiguousarray(host_offsets, dtype=np.int32)
    mem = np.ascontiguousarray(host_members, dtype=np.int32)
    nh = off.shape[0] - 1
    out = np.zeros(max(nh, 1), np.float64)
    _check(lib().vr_ref_host_ellv(C.byref(P.s), nh, _p(off), _p(mem), float(alpha_v), _p(out)),
           "host_ellv")
    return out[:nh]


def fof6d(P: Particles, host_of, ellv_host, ellx_s, R=None, R_threshold=2.0):
    hof = np.ascontiguousarray(host_of, dtype=np.int32)
    ev = np.ascontiguousarray(ellv_host, dtype=np.float64)
    nh = ev.shape[0]
    if ev.shape[0] == 0:
        ev = np.ones(1)
    Rr = None if R is None else np.ascontiguousarray(R, dtype=np.float32)
    lab = np.zeros(P.n, np.int32)
    _check(lib().vr_ref_fof6d(C.byref(P.s), _p(hof), nh, _p(ev), float(ellx_s), _p(Rr),
                              float(R_threshold), _p(lab)), "fof6d")
    return lab


def fof_sub(P: Particles, host_of, n_hosts, vbar, ellx_s, L, L_threshold=2.5, Vr=2.0, cos_op=None,
            theta_op=math.pi / 10):
    """The paper's substructure linker (Sec. 2.2, Eq. linkingcriteria); label =
    smallest participant index of the component, -1 for non-participants."""
    hof = np.ascontiguousarray(host_of, dtype=np.int32)
    vb = np.ascontiguousarray(vbar, dtype=np.float32)
    Lr = np.ascontiguousarray(L, dtype=np.float32)
    c = math.cos(theta_op) if cos_op is None else float(cos_op)
    lab = np.zeros(P.n, np.int32)
    _check(lib().vr_ref_fof_sub(C.byref(P.s), _p(hof), int(n_hosts), _p(vb), float(ellx_s), _p(Lr),
                                float(L_threshold), float(Vr), c, _p(lab)), "fof_sub")
    return lab


def sub_grow(P: Particles, host_of, n_hosts, vbar, L, label1, ellx_s, L_threshold=2.5, gamma_L=1.0, gamma_x=2.0,
             Vr=2.0, gamma_V=1.0, theta_op=math.pi / 10, gamma_theta=1.0, f_merge=0.25, n_min=20):
    """Second, relaxed stage of the paper's linker: candidate groups of
    label1 grow into untagged outliers and join when strongly connected.
    Returns (label, growth rounds)."""
    hof = np.ascontiguousarray(host_of, dtype=np.int32)
    vb = np.ascontiguousarray(vbar, dtype=np.float32)
    Lr = np.ascontiguousarray(L, dtype=np.float32)
    l1 = np.ascontiguousarray(label1, dtype=np.int32)
    out = np.zeros(P.n, np.int32)
    nr = np.zeros(1, np.int32)
    c = math.cos(min(math.pi, gamma_theta * theta_op))
    _check(lib().vr_ref_sub_grow(C.byref(P.s), _p(hof), int(n_hosts), _p(vb), _p(Lr), float(L_threshold),
                                 float(gamma_L), float(ellx_s), float(gamma_x), float(Vr), float(gamma_V), c,
                                 float(f_merge), int(n_min), _p(l1), _p(out), _p(nr)), "sub_grow")
    return out, int(nr[0])


def fof3d_dm(P: Particles, ellx, is_baryon):
    """3D FOF of two species: baryons never link to each other (Sec. 2.1)."""
    ib = np.ascontiguousarray(is_baryon, dtype=np.uint8)
    lab = np.zeros(P.n, np.int32)
    _check(lib().vr_ref_fof3d_dm(C.byref(P.s), float(ellx), _p(ib), _p(lab)), "fof3d_dm")
    return lab


def assign_baryons(P: Particles, host_offsets, host_members, is_baryon, sub, ellx, sigma_v, out_init=None):
    """Baryons take the substructure label of the nearest dark-matter member
    of their host in phase space (Sec. 2.4, Eq. baryondist)."""
    off = np.ascontiguousarray(host_offsets, dtype=np.int32)
    mem = np.ascontiguousarray(host_members, dtype=np.int32)
    ib = np.ascontiguousarray(is_baryon, dtype=np.uint8)
    sb = np.ascontiguousarray(sub, dtype=np.int32)
    out = np.full(P.n, -7, np.int32) if out_init is None else np.array(out_init, np.int32)
    _check(lib().vr_ref_assign_baryons(C.byref(P.s), off.shape[0] - 1, _p(off), _p(mem), _p(ib), _p(sb),
                                       float(ellx), float(sigma_v), _p(out)), "assign_baryons")
    return out


def unbind(P: Particles, offsets, members, G, eps, beta_E=0.95, frac_ref=0.1, n_min=20,
           n_ref_min=10, frame_type=1, max_iter=100):
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    ng = off.shape[0] - 1
    n = P.n
    bound = np.zeros(n, np.uint8)
    phi = np.full(n, np.nan)
    iters = np.zeros(max(ng, 1), np.int32)
    margin = np.zeros(max(ng, 1), np.float64)
    up = _UnbindParams(G, eps, beta_E, frac_ref, n_min, n_ref_min, frame_type, max_iter)
    rc = lib().vr_ref_unbind(C.byref(P.s), ng, _p(off), _p(mem), C.byref(up), _p(bound), _p(phi),
                             _p(iters), _p(margin))
    if rc == -5:
        raise RuntimeError("oracle unbind did not converge within max_iter")
    _check(rc, "unbind")
    return dict(bound=bound, phi=phi, iters=iters[:ng], min_margin=margin[:ng])


def ell_fit(R, host_offsets, host_members, ell_init=None, **params):
    """Per-host skew-Gaussian fit of the binned R values and L = (R - Rbar) /
    sigma_R (Sec. 2.2, Eqs. skewgaus and ell).  Returns dict(fit (nh, 4):
    Rbar, sigma_R, s, A; status (nh,); merge (nh,); ell (n,) float32, NaN
    outside the hosts unless ell_init is given)."""
    R = np.ascontiguousarray(R, dtype=np.float32)
    off = np.ascontiguousarray(host_offsets, dtype=np.int32)
    mem = np.ascontiguousarray(host_members, dtype=np.int32)
    nh = off.shape[0] - 1
    ep = _EllParams(**{**ELL_DEFAULTS, **params})
    fit = np.zeros((max(nh, 1), 4))
    status = np.zeros(max(nh, 1), np.int32)
    merge = np.zeros(max(nh, 1), np.int32)
    ell = np.full(R.shape[0], np.nan, np.float32) if ell_init is None else np.array(ell_init, np.float32)
    _check(lib().vr_ref_ell_fit(R.shape[0], nh, _p(off), _p(mem), _p(R), C.byref(ep), _p(fit), _p(status),
                                _p(merge), _p(ell)), "ell_fit")
    return dict(fit=fit[:nh], status=status[:nh], merge=merge[:nh], ell=ell)


def ell_cost(x, w, c):
    """Cost and (a, p, q) of the log-model least-squares fit at peak c."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    apq = np.zeros(3)
    J = lib().vr_ref_ell_cost(x.shape[0], _p(x), _p(w), float(c), _p(apq))
    return J, apq


def ell_mean(ell_th):
    """Expected L of chance outliers above ell_th (closed form after Eq. ellsig)."""
    return lib().vr_ref_ell_mean(float(ell_th))


def ell_clean(ell, offsets, members, label, ell_th=2.5, beta=1.0, n_min=20):
    """Significance cleaning (Eq. ellsig).  Returns (label, removed): label a
    copy with removed members -1 and kept ones relabelled by their smallest
    index; removed[g] = members removed from group g (all when dissolved)."""
    ell = np.ascontiguousarray(ell, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    mem = np.ascontiguousarray(members, dtype=np.int32)
    lab = np.array(label, dtype=np.int32)
    ng = off.shape[0] - 1
    rem = np.zeros(max(ng, 1), np.int32)
    _check(lib().vr_ref_ell_clean(ell.shape[0], ng, _p(off), _p(mem), _p(ell), float(ell_th), float(beta),
                                  int(n_min), _p(lab), _p(rem)), "ell_clean")
    return lab, rem[:ng]
