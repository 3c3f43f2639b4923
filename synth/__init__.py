"""Seeded synthetic inputs (no SSIM arithmetic); shared by tests and bench."""
from .workloads import *  # noqa: F401,F403
