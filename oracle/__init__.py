"""Plain FP64 CPU oracle (test infrastructure; see oracle.c for the contract)."""
