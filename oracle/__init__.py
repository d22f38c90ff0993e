"""CPU oracle for the ISM pressure solve: test infrastructure only (see ism_oracle)."""
from . import ism_oracle  # noqa: F401
