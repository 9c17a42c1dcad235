"""CPU oracle for the SO(3) FFT (test infrastructure only; see oracle.py)."""
