"""FP64 CPU oracle of the APM gravity solve -- test infrastructure only (see
apm_oracle's module docstring).  The product path never imports this package."""
