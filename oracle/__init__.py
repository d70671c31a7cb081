"""Serial CPU oracle for sparse-matrix assembly: test infrastructure only."""
