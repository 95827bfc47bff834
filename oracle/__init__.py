"""CPU checker for the Poisson path (test infrastructure only; see poisson_oracle)."""
