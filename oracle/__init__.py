"""CPU oracle for the partitioned reduction (test infrastructure only)."""
from .oracle import Oracle, get  # noqa: F401
