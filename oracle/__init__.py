"""CPU FP64 oracle (test infrastructure; never imported by the GPU package)."""
