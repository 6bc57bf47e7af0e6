"""MI355X (gfx950) radiance-bucket lookup of "Radiance Textures for
Rasterizing Ray-Traced Data" (arXiv 2301.01719).

The compute path is libradtex.so (HIP kernels behind the C ABI of
include/radtex.h); `radtex` is its ctypes binding.  Importing the package
does not load the library; `from paper_2301_01719_amd import radtex` does,
and raises if it has not been built.
"""
__all__ = ["radtex", "workloads", "build"]
