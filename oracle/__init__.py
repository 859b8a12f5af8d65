"""CPU oracle (test infrastructure only; see mphf_oracle)."""
