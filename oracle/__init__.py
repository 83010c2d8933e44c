"""FP64 CPU reference oracle (test infrastructure; see oracle.c for the definitions)."""
