"""Thin ctypes binding of libvr (include/vr.h).

Argument marshalling only: every step runs in the HIP kernels of libvr.so.
PyTorch supplies device memory and the current stream.  There is no fallback:
if libvr.so is missing, or no gfx950 device is visible, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvr.so")

VR_OK, VR_ERR_INVALID_ARG, VR_ERR_NO_DEVICE, VR_ERR_OUT_OF_MEMORY = 0, -1, -2, -3
VR_ERR_HIP, VR_ERR_NOT_CONVERGED, VR_ERR_UNSUPPORTED = -4, -5, -6
CELL_COLS = 28
NOALLOC_MAX_LABELS = 4194304

# Entry points declared in include/vr.h (checked by the CPU test-suite).
ENTRY_POINTS = (
    "vr_create", "vr_destroy", "vr_last_error", "vr_sync", "vr_workspace_bytes", "vr_new_snapshot",
    "vr_set_timing", "vr_kernel_time", "vr_tune", "vr_get_tune", "vr_autotune",
    "vr_quantize", "vr_fof3d", "vr_groups", "vr_cell_moments", "vr_local_vdensity",
    "vr_host_ellv", "vr_fof6d", "vr_fof_sub", "vr_sub_grow", "vr_fof3d_dm", "vr_assign_baryons",
    "vr_relabel_min", "vr_relabel_min_noalloc", "vr_select_members", "vr_unbind", "vr_ell_fit", "vr_ell_clean",
    "vr_rs_features", "vr_mlp_forward", "vr_mlp_grad", "vr_mlp_train_step", "vr_rs_select",
)

MLP_PARAMS = 9217
TUNE_KNOBS = ("unbind_tile", "unbind_jchunk", "unbind_bpc", "unbind_wide", "knn_leaf", "xcd_chunk")


class VrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libvr status {code}: {msg}")
        self.code = code


class _Particles(C.Structure):
    _fields_ = [("n", C.c_int64),
                ("qx", C.c_void_p), ("qy", C.c_void_p), ("qz", C.c_void_p),
                ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
                ("mass", C.c_void_p), ("mass_value", C.c_double),
                ("box", C.c_double), ("grid_bits", C.c_int32)]


class _CellParams(C.Structure):
    _fields_ = [("f_cell", C.c_double), ("ncell_floor", C.c_int32), ("ncell_div", C.c_int32),
                ("nbins", C.c_int32), ("split_rule", C.c_int32)]


class _UnbindParams(C.Structure):
    _fields_ = [("G", C.c_double), ("eps", C.c_double), ("beta_E", C.c_double),
                ("frac_ref", C.c_double), ("n_min", C.c_int32), ("n_ref_min", C.c_int32),
                ("frame_type", C.c_int32), ("max_iter", C.c_int32), ("persistent", C.c_int32),
                ("tile", C.c_int32)]


class _EllParams(C.Structure):
    _fields_ = [("lo", C.c_double), ("width", C.c_double), ("nbins", C.c_int32), ("peak_min", C.c_int32),
                ("max_merge", C.c_int32), ("golden_iters", C.c_int32)]


# R grid of the per-host fit: 1024 bins of 1/32 on [-16, 16), bin pairs merged
# until the fullest holds 32 (factor <= 64), 48 golden-section steps
ELL_PARAMS = dict(lo=-16.0, width=1.0 / 32, nbins=1024, peak_min=32, max_merge=64, golden_iters=48)


class _AdamParams(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


_lib = None


def load_library():
    """Load libvr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1902_01010_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl, flt, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_float, C.c_size_t
        P = C.POINTER(_Particles)
        L.vr_create.argtypes = [C.POINTER(vp), C.c_int, sz]
        L.vr_destroy.argtypes = [vp]
        L.vr_destroy.restype = None
        L.vr_last_error.argtypes = [vp]
        L.vr_last_error.restype = C.c_char_p
        L.vr_sync.argtypes = [vp, vp]
        L.vr_workspace_bytes.argtypes = [vp]
        L.vr_new_snapshot.argtypes = [vp]
        L.vr_workspace_bytes.restype = sz
        L.vr_set_timing.argtypes = [vp, C.c_int]
        L.vr_kernel_time.argtypes = [vp, C.c_char_p, C.POINTER(i64), C.POINTER(dbl), C.POINTER(dbl)]
        L.vr_tune.argtypes = [vp, C.c_char_p, C.c_int]
        L.vr_get_tune.argtypes = [vp, C.c_char_p, C.POINTER(C.c_int)]
        L.vr_autotune.argtypes = [vp, C.c_char_p, C.c_int]
        L.vr_quantize.argtypes = [vp, i64, vp, vp, vp, dbl, i32, vp, vp, vp, vp]
        L.vr_fof3d.argtypes = [vp, P, dbl, vp, vp]
        L.vr_groups.argtypes = [vp, i64, vp, i32, C.POINTER(i32), vp, vp, vp, vp]
        L.vr_cell_moments.argtypes = [vp, P, i32, vp, vp, C.POINTER(_CellParams), vp, vp, vp, vp,
                                      i64, vp, C.POINTER(i64), vp]
        L.vr_local_vdensity.argtypes = [vp, P, i32, vp, vp, vp, vp, i32, i32, vp, i64, vp, vp]
        L.vr_host_ellv.argtypes = [vp, P, i32, vp, vp, dbl, vp, vp]
        L.vr_fof6d.argtypes = [vp, P, vp, vp, i32, dbl, vp, flt, vp, vp]
        L.vr_fof_sub.argtypes = [vp, P, vp, i32, vp, dbl, vp, flt, dbl, dbl, vp, vp]
        L.vr_fof3d_dm.argtypes = [vp, P, dbl, vp, vp, vp]
        L.vr_assign_baryons.argtypes = [vp, P, i32, vp, vp, vp, vp, dbl, dbl, vp, dbl, vp, vp, vp]
        L.vr_relabel_min.argtypes = [vp, i64, vp, i32, vp, vp]
        L.vr_relabel_min_noalloc.argtypes = [vp, i64, vp, i32, vp, vp]
        L.vr_select_members.argtypes = [vp, i64, i32, vp, vp, vp, vp, vp, vp]
        L.vr_sub_grow.argtypes = [vp, P, vp, i32, vp, vp, flt, dbl, dbl, dbl, dbl, dbl, dbl, dbl, i32, vp, vp,
                                  C.POINTER(i32), vp]
        L.vr_unbind.argtypes = [vp, P, i32, vp, vp, C.POINTER(_UnbindParams), vp, vp, vp, vp]
        L.vr_ell_fit.argtypes = [vp, i64, i32, vp, vp, vp, C.POINTER(_EllParams), vp, vp, vp, vp, vp]
        L.vr_ell_clean.argtypes = [vp, i64, i32, vp, vp, vp, dbl, dbl, i32, vp, vp, vp]
        fp = C.POINTER(C.c_float)
        L.vr_rs_features.argtypes = [vp, P, i32, vp, vp, vp, vp, vp, i32, i32, fp, fp, vp, C.POINTER(i64), vp]
        L.vr_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
        L.vr_mlp_grad.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp]
        L.vr_mlp_train_step.argtypes = [vp, vp, vp, i64, vp, vp, vp, C.POINTER(_AdamParams), i32, vp, vp]
        L.vr_rs_select.argtypes = [vp, i64, vp, vp, flt, flt, vp, vp, C.POINTER(i64), vp]
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libvr takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libvr takes contiguous tensors")
    return C.c_void_p(t.data_ptr())


def _pm(t, k, output=False):
    """A per-particle k-vector field held as a (k, n) tensor, in the
    library's particle-major [n][k] layout.  A (k, n) view of [n][k] storage
    (what cell_moments returns) is used as it is; a component-major (k, n)
    array is copied into the library's layout (inputs only); a flat buffer
    of k n values is taken to be in that layout already.  The caller holds
    the result until the library call has been enqueued, so that a copy's
    memory is not handed out again before the kernels that read it."""
    if t is None:
        return None
    if t.dim() == 1 and t.numel() % k == 0:
        return t
    if t.dim() != 2 or t.shape[0] != k:
        raise ValueError(f"expected a ({k}, n) tensor, got {tuple(t.shape)}")
    tt = t.t()
    if not tt.is_contiguous():
        if output:
            raise ValueError("outputs must be (k, n) views of particle-major [n][k] storage")
        tt = tt.contiguous()
    return tt


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Particles:
    """Device particle set: q (3, n) int32 grid coordinates, v (3, n) float32,
    optional mass (n,) float32."""

    def __init__(self, q, v, mass, mass_value, box, grid_bits):
        self.q = q.contiguous()
        self.v = None if v is None else v.contiguous()
        self.mass = None if mass is None else mass.contiguous()
        self.mass_value = float(mass_value)
        self.box = float(box)
        self.grid_bits = int(grid_bits)
        s = _Particles()
        s.n = self.q.shape[1]
        s.qx, s.qy, s.qz = (C.c_void_p(self.q[d].data_ptr()) for d in range(3))
        if self.v is not None:
            s.vx, s.vy, s.vz = (C.c_void_p(self.v[d].data_ptr()) for d in range(3))
        s.mass = None if self.mass is None else C.c_void_p(self.mass.data_ptr())
        s.mass_value = self.mass_value
        s.box = self.box
        s.grid_bits = self.grid_bits
        self.s = s

    @property
    def n(self):
        return self.q.shape[1]

    @property
    def device(self):
        return self.q.device


class Context:
    """A libvr context on one device (workspace pool, autotune state)."""

    def __init__(self, device: int = 0, max_workspace_bytes: int = 0):
        self.lib = load_library()
        h = C.c_void_p()
        rc = self.lib.vr_create(C.byref(h), int(device), int(max_workspace_bytes))
        if rc != VR_OK:
            raise VrError(rc, self.lib.vr_last_error(None).decode())
        self.h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.vr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != VR_OK:
            raise VrError(rc, self.lib.vr_last_error(self.h).decode())

    def sync(self):
        self._check(self.lib.vr_sync(self.h, _stream()))

    def new_snapshot(self):
        """Forget state kept from calls on the previous particle set."""
        self._check(self.lib.vr_new_snapshot(self.h))

    def workspace_bytes(self):
        return int(self.lib.vr_workspace_bytes(self.h))

    def set_timing(self, enabled: bool):
        self._check(self.lib.vr_set_timing(self.h, 1 if enabled else 0))

    def tune(self, knob: str, value: int):
        self._check(self.lib.vr_tune(self.h, knob.encode(), int(value)))

    def autotune(self, cache_path=None, force=False):
        """Apply cached launch knobs for this GPU, or time the sweeps and write the cache."""
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.lib.vr_autotune(self.h, path, 1 if force else 0))
        return {k: self.get_tune(k) for k in TUNE_KNOBS}

    def get_tune(self, knob: str) -> int:
        v = C.c_int(0)
        self._check(self.lib.vr_get_tune(self.h, knob.encode(), C.byref(v)))
        return v.value

    def kernel_time(self, name: str):
        """(launches, total ms, algorithmic work units) accumulated for a kernel."""
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        work = C.c_double(0.0)
        self._check(self.lib.vr_kernel_time(self.h, name.encode(), C.byref(n), C.byref(ms), C.byref(work)))
        return n.value, ms.value, work.value

    # -- entry points -------------------------------------------------------
    def quantize(self, x, box, grid_bits=21):
        n = x.shape[1]
        q = torch.empty((3, n), dtype=torch.int32, device=x.device)
        x = x.contiguous()
        self._check(self.lib.vr_quantize(self.h, n, _ptr(x[0]), _ptr(x[1]), _ptr(x[2]), float(box),
                                         int(grid_bits), _ptr(q[0]), _ptr(q[1]), _ptr(q[2]), _stream()))
        return q

    def fof3d(self, P: Particles, ellx, label=None):
        if label is None:
            label = torch.empty(P.n, dtype=torch.int32, device=P.device)
        self._check(self.lib.vr_fof3d(self.h, C.byref(P.s), float(ellx), _ptr(label), _stream()))
        return label

    def groups(self, label, n_min):
        n = label.shape[0]
        dev = label.device
        ng = C.c_int32(0)
        gof = torch.empty(n, dtype=torch.int32, device=dev)
        off = torch.empty(n + 1, dtype=torch.int32, device=dev)
        mem = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        self._check(self.lib.vr_groups(self.h, n, _ptr(label), int(n_min), C.byref(ng), _ptr(gof),
                                       _ptr(off), _ptr(mem), _stream()))
        g = ng.value
        off = off[:g + 1]
        return g, gof, off, mem

    def cell_moments(self, P: Particles, host_offsets, host_members, f_cell=0.01, ncell_floor=100,
                     ncell_div=8, nbins=16, split_rule=0, want_table=True, out=None, want_rho=True,
                     want_cell_of=True):
        """want_rho / want_cell_of False: that output is not written (None)."""
        dev = P.device
        n = P.n
        nh = host_offsets.shape[0] - 1
        if out is None:
            # particle-major storage, returned as (3, n) and (6, n) views;
            # the float outputs share one NaN-filled allocation (one fill),
            # each part starting on a 256-byte boundary
            a = lambda k: -(-k // 64) * 64  # noqa: E731
            o1 = a(3 * n)
            o2 = a(o1 + 6 * n)
            buf = torch.full((o2 + (n if want_rho else 0),), float("nan"), device=dev)
            out = dict(vbar=buf[:3 * n].view(n, 3).t(),
                       sigma=buf[o1:o1 + 6 * n].view(n, 6).t(),
                       rho_cell=buf[o2:o2 + n] if want_rho else None,
                       cell_of=torch.full((n,), -1, dtype=torch.int32, device=dev) if want_cell_of else None)
        cp = _CellParams(f_cell, ncell_floor, ncell_div, nbins, split_rule)
        vb_l, sg_l = _pm(out["vbar"], 3, True), _pm(out["sigma"], 6, True)
        ncell = C.c_int64(0)
        cap = 0
        table = None
        if want_table:
            # an upper bound on the number of leaves: every leaf holds >= 1 member
            cap = int(host_members.shape[0]) if nh > 0 else 0
            table = torch.empty((max(cap, 1), CELL_COLS), dtype=torch.float64, device=dev)
        self._check(self.lib.vr_cell_moments(self.h, C.byref(P.s), nh, _ptr(host_offsets), _ptr(host_members),
                                             C.byref(cp), _ptr(vb_l), _ptr(sg_l),
                                             _ptr(out["rho_cell"]), _ptr(out["cell_of"]), cap,
                                             _ptr(table), C.byref(ncell), _stream()))
        out["n_cells"] = ncell.value
        if want_table:
            out["cells"] = table[:ncell.value]
        return out

    def local_vdensity(self, P: Particles, host_offsets, host_members, vbar, sigma, n_se, n_v,
                       subset=None, R=None):
        if R is None:
            R = torch.full((P.n,), float("nan"), device=P.device)
        nh = host_offsets.shape[0] - 1
        ns = 0 if subset is None else subset.shape[0]
        vb_l, sg_l = _pm(vbar, 3), _pm(sigma, 6)
        self._check(self.lib.vr_local_vdensity(self.h, C.byref(P.s), nh, _ptr(host_offsets),
                                               _ptr(host_members), _ptr(vb_l), _ptr(sg_l), int(n_se),
                                               int(n_v), _ptr(subset), ns, _ptr(R), _stream()))
        return R

    def host_ellv(self, P: Particles, host_offsets, host_members, alpha_v=1.25):
        nh = host_offsets.shape[0] - 1
        out = torch.empty(max(nh, 1), dtype=torch.float64, device=P.device)
        self._check(self.lib.vr_host_ellv(self.h, C.byref(P.s), nh, _ptr(host_offsets), _ptr(host_members),
                                          float(alpha_v), _ptr(out), _stream()))
        return out[:nh]

    def fof6d(self, P: Particles, host_of, ellv_host, ellx_s, R=None, R_threshold=2.0, label6=None):
        if label6 is None:
            label6 = torch.empty(P.n, dtype=torch.int32, device=P.device)
        self._check(self.lib.vr_fof6d(self.h, C.byref(P.s), _ptr(host_of), _ptr(ellv_host),
                                      int(ellv_host.shape[0]), float(ellx_s), _ptr(R), float(R_threshold),
                                      _ptr(label6), _stream()))
        return label6

    def fof_sub(self, P: Particles, host_of, n_hosts, vbar, ellx_s, L, L_threshold=2.5, Vr=2.0,
                theta_op=math.pi / 10, label=None):
        """The paper's substructure linker (speed ratio and opening angle about
        the local mean velocity vbar, over L >= L_threshold)."""
        if label is None:
            label = torch.empty(P.n, dtype=torch.int32, device=P.device)
        vb_l = _pm(vbar, 3)
        self._check(self.lib.vr_fof_sub(self.h, C.byref(P.s), _ptr(host_of), int(n_hosts), _ptr(vb_l),
                                        float(ellx_s), _ptr(L), float(L_threshold), float(Vr),
                                        math.cos(theta_op), _ptr(label), _stream()))
        return label

    def sub_grow(self, P: Particles, host_of, n_hosts, vbar, L, label1, ellx_s, L_threshold=2.5, gamma_L=1.0,
                 gamma_x=2.0, Vr=2.0, gamma_V=1.0, theta_op=math.pi / 10, gamma_theta=1.0, f_merge=0.25, n_min=20,
                 label=None):
        """The paper's relaxed second stage: candidate groups of label1 grow and
        join.  Returns (label, growth rounds)."""
        if label is None:
            label = torch.empty(P.n, dtype=torch.int32, device=P.device)
        nr = C.c_int32(0)
        vb_l = _pm(vbar, 3)
        self._check(self.lib.vr_sub_grow(self.h, C.byref(P.s), _ptr(host_of), int(n_hosts), _ptr(vb_l), _ptr(L),
                                         float(L_threshold), float(gamma_L), float(ellx_s), float(gamma_x),
                                         float(Vr), float(gamma_V), math.cos(min(math.pi, gamma_theta * theta_op)),
                                         float(f_merge), int(n_min), _ptr(label1), _ptr(label), C.byref(nr),
                                         _stream()))
        return label, nr.value

    def fof3d_dm(self, P: Particles, ellx, is_baryon, label=None):
        """3D FOF in which baryons (is_baryon != 0, uint8) never link to each other."""
        if label is None:
            label = torch.empty(P.n, dtype=torch.int32, device=P.device)
        self._check(self.lib.vr_fof3d_dm(self.h, C.byref(P.s), float(ellx), _ptr(is_baryon), _ptr(label), _stream()))
        return label

    def assign_baryons(self, P: Particles, host_offsets, host_members, is_baryon, sub, ellx, sigma_v, out=None,
                       ellv_host=None, alpha_v=1.25):
        """Baryons of each host take the substructure label of the nearest dark
        matter in phase space; dark matter copies its own.  sigma_v <= 0: the
        library computes it from ellv_host (the hosts' dark-matter-weighted
        mean of ellv / alpha_v).  Returns (out, sigma_v used)."""
        if out is None:
            out = torch.full((P.n,), -1, dtype=torch.int32, device=P.device)
        used = C.c_double(0.0)
        self._check(self.lib.vr_assign_baryons(self.h, C.byref(P.s), host_offsets.shape[0] - 1, _ptr(host_offsets),
                                               _ptr(host_members), _ptr(is_baryon), _ptr(sub), float(ellx),
                                               float(sigma_v), _ptr(ellv_host), float(alpha_v), C.byref(used),
                                               _ptr(out), _stream()))
        return out, used.value

    def relabel_min(self, label, min_size=1, out=None):
        """Canonical smallest-index labels of components with >= min_size members."""
        if out is None:
            out = torch.empty_like(label)
        self._check(self.lib.vr_relabel_min(self.h, label.shape[0], _ptr(label), int(min_size), _ptr(out), _stream()))
        return out

    def relabel_min_noalloc(self, label, min_size=1, out=None):
        """relabel_min through the entry point that allocates nothing (fixed
        library scratch; at most NOALLOC_MAX_LABELS labels)."""
        if out is None:
            out = torch.empty_like(label)
        self._check(self.lib.vr_relabel_min_noalloc(self.h, label.shape[0], _ptr(label), int(min_size), _ptr(out),
                                                    _stream()))
        return out

    def select_members(self, n, offsets, members, drop):
        """The groups' members without those flagged in drop: (offsets, members)."""
        ng = offsets.shape[0] - 1
        out_off = torch.zeros(ng + 1, dtype=torch.int32, device=offsets.device)
        out_mem = torch.empty(max(1, members.shape[0]), dtype=torch.int32, device=offsets.device)
        self._check(self.lib.vr_select_members(self.h, int(n), ng, _ptr(offsets), _ptr(members), _ptr(drop),
                                               _ptr(out_off), _ptr(out_mem), _stream()))
        return out_off, out_mem

    def unbind(self, P: Particles, offsets, members, G, eps, beta_E=0.95, frac_ref=0.1, n_min=20,
               n_ref_min=10, frame_type=1, max_iter=100, persistent=1, tile=0):
        ng = offsets.shape[0] - 1
        dev = P.device
        bound = torch.zeros(P.n, dtype=torch.uint8, device=dev)
        phi = torch.full((P.n,), float("nan"), dtype=torch.float64, device=dev)
        iters = torch.zeros(max(ng, 1), dtype=torch.int32, device=dev)
        up = _UnbindParams(G, eps, beta_E, frac_ref, n_min, n_ref_min, frame_type, max_iter, persistent, tile)
        self._check(self.lib.vr_unbind(self.h, C.byref(P.s), ng, _ptr(offsets), _ptr(members), C.byref(up),
                                       _ptr(bound), _ptr(phi), _ptr(iters), _stream()))
        return dict(bound=bound, phi=phi, iters=iters[:ng])

    # ---- normalised ratio L and cleaning ---------------------------------------
    def ell_fit(self, R, host_offsets, host_members, ell=None, **params):
        """Per-host skew-Gaussian fit of the binned R and L = (R - Rbar) / sigma_R.
        Returns dict(fit (nh, 4) float64: Rbar, sigma_R, s, A; status; merge;
        ell (n,) float32, NaN outside the hosts unless `ell` is given)."""
        nh = host_offsets.shape[0] - 1
        n = R.shape[0]
        dev = R.device
        ep = _EllParams(**{**ELL_PARAMS, **params})
        fit = torch.zeros((max(nh, 1), 4), dtype=torch.float64, device=dev)
        status = torch.zeros(max(nh, 1), dtype=torch.int32, device=dev)
        merge = torch.zeros(max(nh, 1), dtype=torch.int32, device=dev)
        if ell is None:
            ell = torch.full((n,), float("nan"), dtype=torch.float32, device=dev)
        self._check(self.lib.vr_ell_fit(self.h, n, nh, _ptr(host_offsets), _ptr(host_members), _ptr(R),
                                        C.byref(ep), _ptr(fit), _ptr(status), _ptr(merge), _ptr(ell), _stream()))
        return dict(fit=fit[:nh], status=status[:nh], merge=merge[:nh], ell=ell)

    def ell_clean(self, ell, offsets, members, label, ell_th=2.5, beta=1.0, n_min=20):
        """Significance cleaning of the groups; updates `label` in place and
        returns (label, removed per group)."""
        ng = offsets.shape[0] - 1
        removed = torch.zeros(max(ng, 1), dtype=torch.int32, device=ell.device)
        self._check(self.lib.vr_ell_clean(self.h, ell.shape[0], ng, _ptr(offsets), _ptr(members), _ptr(ell),
                                          float(ell_th), float(beta), int(n_min), _ptr(label), _ptr(removed),
                                          _stream()))
        return label, removed[:ng]

    # ---- learned surrogate of R ------------------------------------------------
    def rs_features(self, P: Particles, host_offsets, host_members, vbar, sigma, rho_cell, n_se=32,
                    cell_bits=9, shift=None, scale=None, feat=None):
        """(m, 12) BF16 feature rows (int16 tensor of bit patterns) of the host members."""
        nh = host_offsets.shape[0] - 1
        if feat is None:
            m = int(host_members.shape[0])
            feat = torch.empty((max(m, 1), 12), dtype=torch.int16, device=P.device)
        arr = C.c_float * 12
        sh = None if shift is None else arr(*[float(x) for x in shift])
        sc = None if scale is None else arr(*[float(x) for x in scale])
        rows = C.c_int64(0)
        vb_l, sg_l = _pm(vbar, 3), _pm(sigma, 6)
        self._check(self.lib.vr_rs_features(self.h, C.byref(P.s), nh, _ptr(host_offsets), _ptr(host_members),
                                            _ptr(vb_l), _ptr(sg_l), _ptr(rho_cell), int(n_se), int(cell_bits),
                                            sh, sc, _ptr(feat), C.byref(rows), _stream()))
        return feat[:rows.value]

    def mlp_forward(self, weights, feat, out=None):
        m = feat.shape[0]
        if out is None:
            out = torch.empty(max(m, 1), dtype=torch.float32, device=feat.device)
        self._check(self.lib.vr_mlp_forward(self.h, _ptr(weights), m, _ptr(feat), _ptr(out), _stream()))
        return out[:m]

    def mlp_grad(self, weights, feat, target, rows=None):
        """(gradient, loss) of the mean squared error over the batch."""
        m = feat.shape[0] if rows is None else rows.shape[0]
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=feat.device)
        loss = torch.empty(1, dtype=torch.float32, device=feat.device)
        self._check(self.lib.vr_mlp_grad(self.h, _ptr(weights), m, _ptr(feat), _ptr(rows), _ptr(target),
                                         _ptr(grad), _ptr(loss), _stream()))
        return grad, loss

    def mlp_train_step(self, weights, adam_state, feat, target, step, rows=None, lr=1e-3, beta1=0.9,
                       beta2=0.999, eps=1e-8, loss=None):
        m = feat.shape[0] if rows is None else rows.shape[0]
        ap = _AdamParams(lr, beta1, beta2, eps)
        self._check(self.lib.vr_mlp_train_step(self.h, _ptr(weights), _ptr(adam_state), m, _ptr(feat), _ptr(rows),
                                               _ptr(target), C.byref(ap), int(step), _ptr(loss), _stream()))
        return loss

    def rs_select(self, members, Rhat, R, R_threshold=2.0, margin=0.5, subset=None):
        """Writes R[members] = Rhat; returns the band's particle list."""
        m = members.shape[0]
        if subset is None:
            subset = torch.empty(max(m, 1), dtype=torch.int32, device=members.device)
        ns = C.c_int64(0)
        self._check(self.lib.vr_rs_select(self.h, m, _ptr(members), _ptr(Rhat), float(R_threshold), float(margin),
                                          _ptr(R), _ptr(subset), C.byref(ns), _stream()))
        return subset[:ns.value]
