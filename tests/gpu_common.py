"""Helpers shared by the GPU parity tests: one seeded workload feeds both the
HIP path (through the C ABI) and the CPU oracle."""
import numpy as np
import torch


def dev_tensor(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_particles(vr, q_dev, w):
    v = dev_tensor(w.v)
    m = None if w.mass is None else dev_tensor(w.mass)
    return vr.Particles(q_dev, v, m, w.mass_value, w.box, w.grid_bits)


def ref_particles(ref, w):
    q = ref.quantize(w.x, w.box, w.grid_bits)
    return ref.Particles(q, w.v, w.mass, w.mass_value, w.box, w.grid_bits)


def both(ctx, vr, ref, w):
    """(GPU particles, oracle particles), each side quantising on its own."""
    x = dev_tensor(w.x)
    q = ctx.quantize(x, w.box, w.grid_bits)
    return gpu_particles(vr, q, w), ref_particles(ref, w)


def R_agrees(Rg, Re, thr=2.0, where=None):
    """The GPU's R against the oracle's: |dR| <= 1e-4 max(1, |R|), NaN and
    +inf alike, classes equal outside the tolerance band.  Returns whether
    the classes also agree inside the band (only then may the oracle's own
    downstream chain be compared with the GPU's exactly)."""
    Rg = np.asarray(Rg, np.float64)
    Re = np.asarray(Re, np.float64)
    if where is not None:
        Rg, Re = Rg[where], Re[where]
    assert (np.isnan(Rg) == np.isnan(Re)).all()
    assert (np.isposinf(Rg) == np.isposinf(Re)).all()
    fin = np.isfinite(Re)
    err = np.abs(Rg[fin] - Re[fin]) / np.maximum(1.0, np.abs(Re[fin]))
    assert err.size == 0 or err.max() <= 1e-4, err.max()
    near = np.abs(Re - thr) <= 1e-4 * max(1.0, abs(thr))
    differ = (Rg >= thr) != (Re >= thr)
    assert not (differ & ~near).any()
    return not differ.any()
