"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

Holds data generation only (no solver arithmetic)."""
from .problems import (QPProblem, config1, config2, config4_instance, config4_sizes,
                       config5, tiny, random_iterate, round_to_bf16, band_dose_matrix,
                       random_sparse, ragged_lines, sqp_sequence, irregular_bands, long_rows)

__all__ = ["QPProblem", "config1", "config2", "config4_instance", "config4_sizes",
           "config5", "tiny", "random_iterate", "round_to_bf16", "band_dose_matrix",
           "random_sparse", "ragged_lines", "sqp_sequence", "irregular_bands", "long_rows"]
