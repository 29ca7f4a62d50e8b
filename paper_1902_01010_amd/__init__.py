"""MI355X-native hot path of the VELOCIraptor phase-space halo finder.

`paper_1902_01010_amd.vr` is the thin ctypes binding of the HIP library
`libvr.so` (C ABI declared in include/vr.h); `synth` holds the seeded
synthetic workloads.  Importing the package loads nothing; the binding loads
the library on first use and raises if it is missing.
"""
