"""FP64 CPU oracle (test infrastructure only; see ttm_oracle)."""
