"""Deep Potential energy / force / virial evaluation on MI355X (gfx950).

The compute path is libdpmi.so (HIP kernels behind the C ABI of
include/dpmi.h); ``_lib`` binds it with ctypes and ``model.DPModel`` wraps it
for torch tensors.  ``synth`` generates the seeded synthetic workloads.
Submodules are imported on demand so that ``synth`` works without a GPU.
"""
__all__ = ["synth", "model", "build"]
