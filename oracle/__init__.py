"""FP64 CPU oracle (test infrastructure only; see parafac2_oracle)."""
