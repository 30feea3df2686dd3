"""MI355X-native MR-STAT matrix-free Jacobian products (placeholder; binding added below)."""
