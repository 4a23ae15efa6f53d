"""fntrs: FNT-based Reed-Solomon erasure coding over GF(65537) for AMD MI355X.

The coding path lives in the HIP library libfntrs.so (C ABI in
include/fntrs.h); ``paper_0907_1788_amd.fntrs`` is its Python binding and
``paper_0907_1788_amd.synth`` the seeded input generators.  Importing this
package loads nothing; the binding loads the library on first use.
"""
__all__ = ["fntrs", "synth", "build"]
