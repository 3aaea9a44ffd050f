"""FP64 CPU oracle of the EDAC-SPH hot path (test infrastructure only)."""
