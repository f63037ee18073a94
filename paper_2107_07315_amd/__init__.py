"""MI355X (gfx950) SPH particle loop for neutron stars with a solid crust.

The compute path is libsph.so (HIP kernels behind the C ABI in include/sph.h); the Python
binding in paper_2107_07315_amd.sph only marshals arguments.  Importing the package does not
touch the GPU.
"""
__all__ = ["sph"]
