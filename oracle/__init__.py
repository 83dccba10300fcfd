"""FP64 CPU oracle for the RBSOG force and pressure evaluation (test infrastructure only)."""
