"""Independent references used to pin the oracle (tests only)."""
