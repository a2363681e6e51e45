"""FP64 CPU oracle (test infrastructure only; see mimo_oracle)."""
