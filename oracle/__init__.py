"""CPU FP64 oracle (test infrastructure only; see teuk_oracle)."""
