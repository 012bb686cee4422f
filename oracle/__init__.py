"""CPU oracle (test infrastructure only; see oracle.py and hough_oracle.c)."""
