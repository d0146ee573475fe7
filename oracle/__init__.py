"""FP64 brute-force oracle (test infrastructure only; see ``oracle.py``)."""
