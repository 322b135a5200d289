"""Plain FP64 CPU oracle (test infrastructure only; see cpm_oracle)."""
