"""Seeded synthetic inputs shared by the oracle tests and the HIP path."""
from .scenes import Problem, Scene, make, pack, CONFIGS  # noqa: F401
