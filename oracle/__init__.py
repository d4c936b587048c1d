"""CPU oracle (test infrastructure only; see cmm_oracle)."""
