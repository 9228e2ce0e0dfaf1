"""CPU FP64 oracle (test infrastructure only; see fsa_oracle)."""
