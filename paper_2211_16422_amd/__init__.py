"""MI355X (gfx950) implementation of the HyperOMS hot path (arXiv 2211.16422):
Eq. 1 hypervector encoding and open-window Hamming top-1 search, behind the
C ABI of libhyperoms (include/hyperoms.h).

Import :mod:`paper_2211_16422_amd.hyperoms` for the binding; it raises if the
native library has not been built.
"""
