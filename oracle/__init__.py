"""CPU oracle (test infrastructure only; see oracle.c for what it computes)."""
