"""Workload definitions for the benchmark (inputs only; no solver arithmetic)."""
