"""FP64 CPU oracle of the matrix-profile join (numpy + C/OpenMP).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and bench.py's
CPU-baseline leg may import this package; the product path never does.
"""
