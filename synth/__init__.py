"""Seeded synthetic workloads shared by the GPU path and the oracle."""
