"""Oracle package -- test infrastructure only (see hermite_oracle.py)."""
