"""FP64 CPU oracle for the pROST per-frame hot path (test infrastructure only)."""
