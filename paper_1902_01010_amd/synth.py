"""Seeded synthetic workloads shaped like the paper's simulations.

The paper measures on SURFS N-body snapshots (L40N512, L210N1536, Table
"Simulation parameters"), which are not available here; these generators stand
in for them.  They only draw particles: positions (float32, length units,
inside a periodic box), velocities (float32, km/s) and masses.  They contain
none of the halo finder's arithmetic, and both the GPU path and the CPU oracle
consume their output.

Units: Mpc/h, km/s, Msun/h.  Every generator shuffles the particle order so
that index order carries no spatial structure.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import lambertw

RHO_CRIT = 2.7754e11     # critical density, h^2 Msun / Mpc^3
OMEGA_M = 0.3121         # matter density implied by the particle masses of the simulation table
G_GRAV = 4.30091e-9      # gravitational constant, Mpc (km/s)^2 / Msun
GRID_BITS = 21


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray            # (3, n) float32 positions in [0, box)
    v: np.ndarray            # (3, n) float32 velocities
    mass: np.ndarray | None  # (n,) float32, or None for uniform mass
    mass_value: float
    box: float
    grid_bits: int
    params: dict             # method parameters for this workload
    meta: dict               # generator bookkeeping (component counts, seeds)
    groups: tuple | None = None   # (offsets, members) for group-level workloads

    @property
    def n(self) -> int:
        return self.x.shape[1]


# ---------------------------------------------------------------------------
# Profile samplers

def _unit_vectors(rng, n):
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0, keepdims=True)
    return u


def _nfw_mu(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw_radii(rng, n, r200, c):
    """Radii of an NFW profile truncated at r200 (inverse enclosed mass via Lambert W)."""
    c = np.broadcast_to(np.asarray(c, np.float64), (n,))
    r200 = np.broadcast_to(np.asarray(r200, np.float64), (n,))
    mu = rng.random(n) * _nfw_mu(c)
    w = lambertw(-np.exp(-1.0 - mu), 0).real
    x = -1.0 / w - 1.0
    return x * (r200 / c)


def plummer_radii(rng, n, a, umax=0.985):
    """Radii of a Plummer sphere, truncated near 10a by capping the mass fraction."""
    u = rng.random(n) * umax
    return np.asarray(a) / np.sqrt(u ** (-2.0 / 3.0) - 1.0)


def power_law_sizes(rng, lo, hi, total, slope=0.9):
    """Integer sizes from dN/dlnN ~ N^-slope on [lo, hi], drawn until they sum
    to at least `total`; the last draw is truncated so the sum is exact."""
    out, acc = [], 0
    a, b = lo ** (-slope), hi ** (-slope)
    while acc < total:
        u = rng.random(4096)
        s = np.floor((a - u * (a - b)) ** (-1.0 / slope)).astype(np.int64)
        s = np.clip(s, lo, hi)
        cs = np.cumsum(s) + acc
        k = int(np.searchsorted(cs, total))
        if k < len(s):
            s = s[:k + 1].copy()
            s[-1] -= cs[k] - total
            out.append(s)
            acc = total
        else:
            out.append(s)
            acc = int(cs[-1])
    sizes = np.concatenate(out)
    return sizes[sizes > 0]


def _nfw_phi(r, m200, r200, c):
    """Potential of an NFW sphere truncated at r200 (for escape speeds)."""
    rs = r200 / c
    x = np.maximum(r, 1e-12) / rs
    k = G_GRAV * m200 / _nfw_mu(c)
    inside = -k * (np.log1p(x) / np.maximum(r, 1e-12) - np.log1p(c) / r200) - G_GRAV * m200 / r200
    return np.where(r <= r200, inside, -G_GRAV * m200 / np.maximum(r, 1e-12))


def _finish(name, rng, pos, vel, box, mass, mass_value, params, meta, groups_of=None, extra=None):
    n = pos.shape[1]
    perm = rng.permutation(n)
    for k, a in (extra or {}).items():
        meta[k] = a[perm]
    pos = np.mod(pos[:, perm], box)
    # float32 rounding can map a coordinate just below the box edge onto it
    x = pos.astype(np.float32)
    x[x >= np.float32(box)] = 0.0
    v = vel[:, perm].astype(np.float32)
    m = None if mass is None else mass[perm].astype(np.float32)
    groups = None
    if groups_of is not None:
        gid = groups_of[perm]
        order = np.lexsort((np.arange(n), gid))
        order = order[gid[order] >= 0]
        counts = np.bincount(gid[gid >= 0], minlength=int(gid.max()) + 1)
        offsets = np.zeros(len(counts) + 1, np.int32)
        offsets[1:] = np.cumsum(counts)
        groups = (offsets, order.astype(np.int32))
    return Workload(name, x, v, m, mass_value, float(box), GRID_BITS, params, meta, groups)


def mean_spacing_for_mass(m_p):
    """Cosmological mean inter-particle spacing for a particle mass."""
    return (m_p / (OMEGA_M * RHO_CRIT)) ** (1.0 / 3.0)


# ---------------------------------------------------------------------------
# Workloads

def isolated_halo(seed=1, n_host=100_000, n_sub=5, sub_range=(1000, 10000), box=1.0, m=1e8, n_subsub=0):
    """Single isolated halo: an NFW host (c=10, r200=0.3 Mpc/h at 1e5 particles)
    with Plummer subhalos (a = 5-15 kpc/h at radii 30-250 kpc/h), Gaussian
    velocities (host sigma 200, subhalo sigma 10-30 km/s, subhalo bulk
    N(0, 200) per axis), equal masses 1e8 Msun/h, 1 Mpc/h periodic box.
    n_subsub > 0 plants a sub-subhalo of that many particles in the largest
    subhalo: Plummer a = 0.2 a_sub at radius a_sub from its centre, moving at
    3 sigma_sub from its bulk velocity, dispersion 0.3 sigma_sub;
    meta["subsub"] flags its particles."""
    rng = np.random.default_rng(seed)
    scale = (n_host / 1e5) ** (1.0 / 3.0)
    r200, c = 0.3 * scale, 10.0
    centre = np.full((3, 1), 0.5 * box)
    r = nfw_radii(rng, n_host, r200, c)
    pos = [centre + _unit_vectors(rng, n_host) * r]
    vel = [rng.normal(0.0, 200.0, size=(3, n_host))]
    subs = []
    for _ in range(n_sub):
        ns = int(rng.integers(sub_range[0], sub_range[1] + 1))
        a = rng.uniform(0.005, 0.015) * scale
        rc = rng.uniform(0.030, 0.250) * scale
        sc = centre + _unit_vectors(rng, 1) * rc
        rr = plummer_radii(rng, ns, a)
        pos.append(sc + _unit_vectors(rng, ns) * rr)
        sig = rng.uniform(10.0, 30.0)
        bulk = rng.normal(0.0, 200.0, size=(3, 1))
        vel.append(bulk + rng.normal(0.0, sig, size=(3, ns)))
        subs.append(dict(n=ns, a=a, r=rc, sigma=sig, centre=sc[:, 0], bulk=bulk[:, 0]))
    flag = [np.zeros(sum(p_.shape[1] for p_ in pos), np.uint8)]
    if n_subsub > 0:
        big = max(subs, key=lambda d: d["n"])
        ssc = big["centre"][:, None] + _unit_vectors(rng, 1) * big["a"]
        pos.append(ssc + _unit_vectors(rng, n_subsub) * plummer_radii(rng, n_subsub, 0.2 * big["a"]))
        sdir = _unit_vectors(rng, 1)
        vel.append(big["bulk"][:, None] + 3.0 * big["sigma"] * sdir
                   + rng.normal(0.0, 0.3 * big["sigma"], size=(3, n_subsub)))
        flag.append(np.ones(n_subsub, np.uint8))
    pos = np.concatenate(pos, axis=1)
    vel = np.concatenate(vel, axis=1)
    spacing = mean_spacing_for_mass(m)
    params = dict(ellx=0.2 * spacing, n_se=32, n_v=8, R_threshold=2.0, alpha_v=1.25,
                  alpha_xs=0.5, eps=0.02 * spacing, G=G_GRAV, beta_E=0.95, n_min=20,
                  host_min=256)
    meta = dict(seed=seed, n_host=n_host, subhalos=subs, spacing=spacing)
    return _finish("isolated_halo", rng, pos, vel, box, None, m, params, meta, extra=dict(subsub=np.concatenate(flag)))


def cosmo_box(seed=2, n_side=256, box=None, halo_frac=0.45, sub_frac=0.10, n_max=None):
    """Synthetic cosmological box: a fraction of the particles in NFW halos
    whose sizes follow dN/dlnN ~ N^-0.9 on [20, n_max], each with Plummer
    subhalos holding 10% of its particles; the rest is a uniform background.
    Halo dispersion 300 (N/1e5)^(1/3) km/s, halo bulk N(0, 400), background
    N(0, 300).  The box keeps the mean spacing of 256^3 particles in 100 Mpc/h
    unless given."""
    rng = np.random.default_rng(seed)
    n_tot = n_side ** 3
    if box is None:
        box = 100.0 * n_side / 256.0
    if n_max is None:
        n_max = int(min(2_000_000, max(1000, 2_000_000 * n_tot / 256 ** 3)))
    m_p = OMEGA_M * RHO_CRIT * box ** 3 / n_tot
    sizes = power_law_sizes(rng, 20, n_max, int(round(halo_frac * n_tot)))
    nh = len(sizes)
    conc = rng.uniform(5.0, 15.0, nh)
    r200 = (3.0 * sizes * m_p / (4.0 * np.pi * 200.0 * RHO_CRIT)) ** (1.0 / 3.0)
    sig_h = 300.0 * (sizes / 1e5) ** (1.0 / 3.0)
    centres = rng.random((3, nh)) * box
    bulk = rng.normal(0.0, 400.0, size=(3, nh))
    # Subhalo components (part of their halo's particle count).
    s_host, s_size = [], []
    for h in np.nonzero(sub_frac * sizes >= 20)[0]:
        ss = power_law_sizes(rng, 20, int(sub_frac * sizes[h]), int(sub_frac * sizes[h]))
        ss = ss[ss >= 2]
        s_host.append(np.full(len(ss), h))
        s_size.append(ss)
    s_host = np.concatenate(s_host) if s_host else np.zeros(0, np.int64)
    s_size = np.concatenate(s_size) if s_size else np.zeros(0, np.int64)
    n_in_subs = np.bincount(s_host, weights=s_size, minlength=nh).astype(np.int64)
    n_nfw = sizes - n_in_subs
    # NFW part of every halo.
    hid = np.repeat(np.arange(nh), n_nfw)
    r = nfw_radii(rng, len(hid), r200[hid], conc[hid])
    pos_h = centres[:, hid] + _unit_vectors(rng, len(hid)) * r
    vel_h = bulk[:, hid] + rng.normal(size=(3, len(hid))) * sig_h[hid]
    # Plummer subhalos.
    ns = len(s_size)
    ha = s_host
    a = rng.uniform(0.005, 0.015, ns) * r200[ha] / 0.3
    rc = rng.uniform(0.1, 0.83, ns) * r200[ha]
    sc = centres[:, ha] + _unit_vectors(rng, ns) * rc
    sig_s = rng.uniform(10.0, 30.0, ns) * sig_h[ha] / 200.0
    sb = bulk[:, ha] + rng.normal(size=(3, ns)) * sig_h[ha]
    sid = np.repeat(np.arange(ns), s_size)
    rr = plummer_radii(rng, len(sid), a[sid])
    pos_s = sc[:, sid] + _unit_vectors(rng, len(sid)) * rr
    vel_s = sb[:, sid] + rng.normal(size=(3, len(sid))) * sig_s[sid]
    # Uniform background.
    nb = n_tot - int(sizes.sum())
    pos_b = rng.random((3, nb)) * box
    vel_b = rng.normal(0.0, 300.0, size=(3, nb))
    pos = np.concatenate([pos_h, pos_s, pos_b], axis=1)
    vel = np.concatenate([vel_h, vel_s, vel_b], axis=1)
    spacing = box / n_side
    params = dict(ellx=0.2 * spacing, n_se=32, n_v=8, R_threshold=2.0, alpha_v=1.25,
                  alpha_xs=0.5, eps=0.02 * spacing, G=G_GRAV, beta_E=0.95, n_min=20,
                  host_min=256)
    meta = dict(seed=seed, n_side=n_side, n_halos=nh, n_subhalos=ns, n_background=nb,
                m_p=m_p, spacing=spacing, n_max=n_max,
                halos=dict(size=sizes, r200=r200, c=conc, sigma=sig_h, centre=centres, bulk=bulk))
    # which component drew each particle: 0 halo (NFW), 1 subhalo (Plummer), 2 background
    comp = np.concatenate([np.zeros(len(hid), np.int8), np.ones(len(sid), np.int8), np.full(nb, 2, np.int8)])
    return _finish("cosmo_box", rng, pos, vel, box, None, m_p, params, meta, extra=dict(component=comp))


def two_species(seed=5, n_side=256, star_per_halo_dm=0.662, disc_frac=0.7, star_mass=0.1, dm=None):
    """Dark matter of cosmo_box(seed, n_side) plus star particles of mass
    star_mass m_p in its halos: per halo round(star_per_halo_dm N) stars, a
    fraction disc_frac in an exponential disc (radial scale 0.03 r200,
    height 0.1 of that, random orientation, rotation 150 km/s plus 20 km/s
    dispersion) and the rest a stellar halo on the halo's NFW profile with
    dispersion 0.8 sigma_host; stars move with the halo's bulk velocity.
    512^3 with the default ratio gives the 40M stars of that configuration.
    meta["is_baryon"] flags the stars; masses are per particle.  dm, when
    given, is that cosmo_box already generated."""
    if dm is None:
        dm = cosmo_box(seed=seed, n_side=n_side)
    rng = np.random.default_rng(seed + 1000)
    H = dm.meta["halos"]
    m_p = dm.meta["m_p"]
    nst = np.rint(star_per_halo_dm * H["size"]).astype(np.int64)
    nd = np.rint(disc_frac * nst).astype(np.int64)
    nsh = nst - nd
    # discs
    hd = np.repeat(np.arange(len(nst)), nd)
    h = 0.03 * H["r200"][hd]
    R = rng.gamma(2.0, 1.0, len(hd)) * h
    z = rng.laplace(0.0, 0.1, len(hd)) * h
    phi = rng.uniform(0, 2 * np.pi, len(hd))
    nrm = _unit_vectors(rng, len(nst))
    e1 = np.cross(nrm.T, np.where(np.abs(nrm[2:3].T) < 0.9, [[0, 0, 1.0]], [[1.0, 0, 0]]))
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(nrm.T, e1)
    a1, a2, an = e1[hd].T, e2[hd].T, nrm[:, hd]
    cph, sph = np.cos(phi), np.sin(phi)
    pos_d = H["centre"][:, hd] + a1 * (R * cph) + a2 * (R * sph) + an * z
    vel_d = H["bulk"][:, hd] + 150.0 * (-a1 * sph + a2 * cph) + rng.normal(0, 20.0, (3, len(hd)))
    # stellar halos
    hh = np.repeat(np.arange(len(nst)), nsh)
    r = nfw_radii(rng, len(hh), H["r200"][hh], H["c"][hh])
    pos_s = H["centre"][:, hh] + _unit_vectors(rng, len(hh)) * r
    vel_s = H["bulk"][:, hh] + rng.normal(size=(3, len(hh))) * (0.8 * H["sigma"][hh])
    box = dm.box
    pos = np.concatenate([dm.x.astype(np.float64), pos_d, pos_s], axis=1)
    vel = np.concatenate([dm.v.astype(np.float64), vel_d, vel_s], axis=1)
    n_dm, n_st = dm.n, len(hd) + len(hh)
    mass = np.concatenate([np.full(n_dm, m_p), np.full(n_st, star_mass * m_p)])
    isb = np.concatenate([np.zeros(n_dm, np.uint8), np.ones(n_st, np.uint8)])
    params = dict(dm.params)
    meta = dict(seed=seed, n_side=n_side, n_dm=n_dm, n_star=n_st, n_disc=len(hd), m_p=m_p,
                spacing=dm.meta["spacing"])
    return _finish("two_species", rng, pos, vel, box, mass, m_p, params, meta, extra=dict(is_baryon=isb))


def unbind_groups(seed=3, n_groups=50_000, n_max=2_000_000, box=100.0, m=1e8,
                  contam_frac=0.2, n_sub=5, sizes=None):
    """Groups for batched unbinding: C1-style NFW hosts (c = 10, r200 and
    sigma scaled by (N/1e5)^(1/3)) with Plummer subhalos of 1-10% of N, plus
    round(0.2 N) contaminants at twice the local escape speed.  Host sizes
    are drawn from dN/dlnN ~ N^-0.9 on [20, n_max], or taken from `sizes`
    (then n_groups = len(sizes)).  Returns the particle set and the
    (offsets, members) group table."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        a0, b0 = 20.0 ** -0.9, float(n_max) ** -0.9
        u = rng.random(n_groups)
        sizes = np.clip(np.floor((a0 - u * (a0 - b0)) ** (-1.0 / 0.9)), 20, n_max).astype(np.int64)
    else:
        sizes = np.asarray(sizes, dtype=np.int64)
        n_groups = len(sizes)
    scale = (sizes / 1e5) ** (1.0 / 3.0)
    r200, c = 0.3 * scale, 10.0
    sig = 200.0 * scale
    m200 = sizes * m
    centres = rng.random((3, n_groups)) * box
    # subhalo sizes (part of N)
    fr = rng.uniform(0.01, 0.1, size=(n_groups, n_sub))
    sub_n = np.floor(fr * sizes[:, None]).astype(np.int64)
    sub_n[sub_n < 20] = 0
    n_nfw = sizes - sub_n.sum(1)
    n_con = np.rint(contam_frac * sizes).astype(np.int64)
    gid_h = np.repeat(np.arange(n_groups), n_nfw)
    r = nfw_radii(rng, len(gid_h), r200[gid_h], c)
    pos_h = centres[:, gid_h] + _unit_vectors(rng, len(gid_h)) * r
    vel_h = rng.normal(size=(3, len(gid_h))) * sig[gid_h]
    # subhalos
    sg = np.repeat(np.arange(n_groups), n_sub)
    sn = sub_n.reshape(-1)
    keep = sn > 0
    sg, sn = sg[keep], sn[keep]
    nsb = len(sn)
    a = rng.uniform(0.005, 0.015, nsb) * scale[sg]
    rc = rng.uniform(0.030, 0.250, nsb) * scale[sg]
    sc = centres[:, sg] + _unit_vectors(rng, nsb) * rc
    ss = rng.uniform(10.0, 30.0, nsb) * scale[sg]
    sb = rng.normal(size=(3, nsb)) * sig[sg]
    sid = np.repeat(np.arange(nsb), sn)
    pos_s = sc[:, sid] + _unit_vectors(rng, len(sid)) * plummer_radii(rng, len(sid), a[sid])
    vel_s = sb[:, sid] + rng.normal(size=(3, len(sid))) * ss[sid]
    gid_s = sg[sid]
    # contaminants at twice the escape speed of the host profile
    gid_c = np.repeat(np.arange(n_groups), n_con)
    rcn = nfw_radii(rng, len(gid_c), r200[gid_c], c)
    pos_c = centres[:, gid_c] + _unit_vectors(rng, len(gid_c)) * rcn
    vesc = np.sqrt(-2.0 * _nfw_phi(rcn, m200[gid_c], r200[gid_c], c))
    vel_c = _unit_vectors(rng, len(gid_c)) * (2.0 * vesc)
    pos = np.concatenate([pos_h, pos_s, pos_c], axis=1)
    vel = np.concatenate([vel_h, vel_s, vel_c], axis=1)
    gid = np.concatenate([gid_h, gid_s, gid_c])
    is_con = np.concatenate([np.zeros(len(gid_h) + len(gid_s), bool), np.ones(len(gid_c), bool)])
    spacing = mean_spacing_for_mass(m)
    params = dict(eps=0.02 * spacing, G=G_GRAV, beta_E=0.95, n_min=20)
    meta = dict(seed=seed, n_groups=n_groups, sizes=sizes, n_contaminants=n_con,
                sum_n2=float(((sizes + n_con) ** 2).sum()))
    return _finish("unbind_groups", rng, pos, vel, box, None, m, params, meta,
                   groups_of=gid, extra=dict(is_contaminant=is_con))


def maxwellian_host(seed=7, n=4096, box=1.0, extent=0.2, sigma=150.0, m=1.0):
    """Uniform positions in a cube of side `extent` inside the box and
    isotropic Gaussian velocities: a smooth background with no substructure."""
    rng = np.random.default_rng(seed)
    pos = 0.5 * box + (rng.random((3, n)) - 0.5) * extent
    vel = rng.normal(0.0, sigma, size=(3, n))
    params = dict(sigma=sigma, extent=extent)
    return _finish("maxwellian", rng, pos, vel, box, None, m, params, dict(seed=seed))


def plummer_sphere(seed=8, n=20000, a=0.01, box=1.0, m=1.0, sigma=50.0):
    rng = np.random.default_rng(seed)
    r = plummer_radii(rng, n, a, umax=0.999)
    pos = 0.5 * box + _unit_vectors(rng, n) * r
    vel = rng.normal(0.0, sigma, size=(3, n))
    return _finish("plummer", rng, pos, vel, box, None, m, dict(a=a), dict(seed=seed))


def mlp_init(seed):
    """Seeded initial parameters of the 12-64-64-64-1 surrogate network in its
    flat FP32 layout (W1[12][64], b1, W2[64][64], b2, W3[64][64], b3, w4[64],
    b4): He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((12, 64), (64, 64), (64, 64)):
        lim = np.sqrt(6.0 / fan_in)
        parts += [rng.uniform(-lim, lim, (fan_in, fan_out)).ravel(), np.zeros(fan_out)]
    lim = np.sqrt(6.0 / 64)
    parts += [rng.uniform(-lim, lim, 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)
