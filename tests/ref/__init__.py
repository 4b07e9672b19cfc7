"""Independent reference routines used by the tests to pin the oracle."""
