"""CPU oracle (test infrastructure only; see mg_oracle's header)."""
