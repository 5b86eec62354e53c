"""MI355X-native two-level block preconditioned Jacobi-Davidson (BPJD) eigensolver."""
