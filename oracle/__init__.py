"""CPU FP64 oracle of multilevel spectral domain decomposition (test infrastructure only)."""
