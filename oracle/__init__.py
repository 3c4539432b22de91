"""FP64 CPU oracle (test infrastructure): see dsl_oracle."""
