"""Seeded synthetic inputs (thermal multiphase Jacobians) shared by tests and benchmarks."""
from .problem import CONFIGS, Problem, make_problem, build_model, bsr_matvec  # noqa: F401
