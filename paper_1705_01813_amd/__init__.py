"""KNN-graph-supported k-means (Deng & Zhao, arXiv 1705.01813) on MI355X.

The compute path is the HIP library ``libknnkm.so`` (kernels for gfx950 behind a
C ABI declared in ``include/knnkm.h``).  ``knnkm`` is the thin ctypes binding;
importing this package does not load the library, so the input generators in
``datagen`` can be used on machines without a GPU.
"""

__all__ = ["knnkm", "datagen"]
