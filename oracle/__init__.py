"""Plain FP64 CPU oracle (test infrastructure only; never used by the product path)."""
from .oracle import Oracle, build, lib_path  # noqa: F401
