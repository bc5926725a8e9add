"""H-matrix assembly and application for 3D elastodynamic Green's tensors on MI355X.

The compute path lives in the C-ABI shared library ``libhmat.so`` (HIP kernels
for gfx950 plus host orchestration); :mod:`paper_1706_09384_amd.hmat` is a thin
ctypes binding with the same entry points.  :mod:`paper_1706_09384_amd.workloads`
generates the synthetic point clouds and right-hand sides.
"""
__all__ = ["hmat", "workloads"]
