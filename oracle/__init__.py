"""FP64 CPU oracle of the MLPF forward pass (test infrastructure only: tests, smoke check and the
benchmark's CPU-baseline leg may use it; the product path never does)."""
