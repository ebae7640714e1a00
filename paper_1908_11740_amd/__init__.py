"""MI355X (gfx950) implementation of the MBR filter step of the
partition-based in-memory spatial join of Tsitsigkos et al. (arXiv 1908.11740).

The join itself runs in the HIP library ``libsj.so`` behind the C ABI declared
in ``include/sj.h``; ``paper_1908_11740_amd.sj`` is the thin ctypes binding to
it.  Importing this package does not load the library; the first call into
``sj`` does, and raises if the library is missing.
"""
__all__ = ["sj", "datagen"]
