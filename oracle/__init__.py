"""FP64 CPU oracle for bundle adjustment: test infrastructure only."""
