"""CPU FP64 oracle (test infrastructure only; see spai_oracle's header)."""
