"""FP64 CPU oracle of the PAMD hot path -- test infrastructure only (see oracle.py)."""
