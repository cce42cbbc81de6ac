"""Physical constants of the oracle (test infrastructure)."""

C0 = 299_792_458.0  # speed of light in vacuum, m/s (the paper's c in eqs. (4), (12))
