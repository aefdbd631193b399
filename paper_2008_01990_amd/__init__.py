"""MI355X-native structured divide-and-conquer tridiagonal eigensolver."""
