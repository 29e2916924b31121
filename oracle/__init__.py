"""Plain FP64 CPU oracle of the hybrid LU-QR solver: test infrastructure only."""
