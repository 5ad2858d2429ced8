"""Placeholder; the binding is filled in with the C-ABI library."""
