"""CPU oracle for the FCIQMC hot path (test infrastructure only)."""
