"""FP64 CPU oracle (test infrastructure only; see ghom_oracle)."""
