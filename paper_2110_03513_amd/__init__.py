"""MI355X-native binned componentwise boosting (CWB / ACWB / HCWB).

The numeric work runs in HIP kernels for gfx950 inside ``libcwb.so``; this
package is a thin ctypes binding (``paper_2110_03513_amd.cwb``) plus the
seeded synthetic-input generators (``paper_2110_03513_amd.datagen``).
Importing the package does not load the library; ``cwb.lib()`` does, and it
raises if the library has not been built.
"""
__all__ = ["cwb", "datagen"]
