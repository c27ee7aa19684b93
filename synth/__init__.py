"""Seeded synthetic inputs shared by the HIP path's callers and the oracle.

This package holds *inputs only*: workload constants, a synthetic PDF grid,
query points, batched-integral specifications and initial network weights.
It contains none of the method's arithmetic (no random-number generator of
the method, no grid map, no interpolation, no integrand, no training step),
so that the GPU path and the oracle, which both consume these inputs, share
no computation.
"""
from .configs import C0, C1, C2, C3, C4, C5, C6, C7, FLAVOURS
from .pdfgrid import synthetic_pdf_grid, synthetic_pdf_replicas, nonuniform_pdf_grid, PdfGridData
from .queries import pdf_queries, fk_points
from .batch import batch_specs, BatchSpec
from .flowinit import he_init_segments
from .alphas import synthetic_alphas, AlphasTable

__all__ = [
    "C0", "C1", "C2", "C3", "C4", "C5", "C6", "C7", "FLAVOURS",
    "synthetic_pdf_grid", "synthetic_pdf_replicas", "nonuniform_pdf_grid", "PdfGridData", "pdf_queries", "fk_points",
    "batch_specs", "BatchSpec", "he_init_segments", "synthetic_alphas", "AlphasTable",
]
