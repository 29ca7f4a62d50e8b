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
