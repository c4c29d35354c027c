"""FP64 CPU oracle for local bundle adjustment (test infrastructure only)."""
