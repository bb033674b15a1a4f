"""Seeded synthetic spectra shaped like the workloads of the HyperOMS evaluation
(Section 4.1, Table 1): raw fragment peaks, precursor m/z and charge for a
spectral library (references plus decoys) and for query spectra.

This module is shared by the oracle and by the GPU path. It only draws random
inputs; it holds none of the method's arithmetic (no filtering, binning,
quantisation, encoding or search).
"""
from .spectra import (  # noqa: F401
    Generated,
    RawSpectra,
    WORKLOADS,
    Workload,
    make_references,
    make_decoys,
    make_queries,
    make_workload,
    make_training_queries,
    concat,
    subset,
)
