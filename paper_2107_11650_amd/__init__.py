"""MI355X-native separable low-rank Hankel (SHLR) reconstruction.

The package is imported lazily: ``paper_2107_11650_amd.inputs`` (seeded
synthetic phantoms and masks) needs only NumPy, while
``paper_2107_11650_amd.shlr`` loads the HIP shared library ``libshlr.so`` and
raises if it is missing.
"""

__all__ = ["inputs", "shlr"]
