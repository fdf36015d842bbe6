"""Seeded synthetic inputs for the transit search (light curves, templates,
grids).  Shared by the CPU oracle's tests and by the GPU path; holds none of
the search's own arithmetic."""

from . import transit, workloads  # noqa: F401
from .workloads import Workload, Injection  # noqa: F401
