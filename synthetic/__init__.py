"""Seeded synthetic workloads (input fields only)."""
