"""Seeded synthetic inputs (networks, queries, workloads) shared by the CPU
oracle and the GPU library.  No path-count arithmetic lives here."""
from .hin import HIN, Constraint, Query, Relation  # noqa: F401
