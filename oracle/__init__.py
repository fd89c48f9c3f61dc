"""CPU oracle for the partitioned reduction (test infrastructure only)."""
from .oracle import Oracle, arrival_constraints, get  # noqa: F401
