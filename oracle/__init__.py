"""CPU oracle of the SHLR iteration (test infrastructure only; never product code)."""
