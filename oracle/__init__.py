"""CPU FP64 oracle for the HDD path (test infrastructure only)."""
