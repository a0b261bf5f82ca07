"""MI355X straightest-geodesic exponential map (gfx950 HIP kernels behind a C ABI).

`paper_2603_15780_amd.sg` is the ctypes binding of libsg.so; importing this
package does not load the library.
"""
__all__ = ["sg", "build"]
