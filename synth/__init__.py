"""Seeded synthetic inputs shared by the tests and the benchmark (no cipher code)."""
from . import gen, workloads  # noqa: F401
