"""FP64 CPU oracle of the improved 3D color-gradient LB model (test infrastructure only)."""
