"""Seeded synthetic inputs for the Core-AFD loop.

This module builds input samples only.  It holds none of the decomposition's
arithmetic (no grid values, no selection, no remainder update); the oracle and
the GPU path both receive the arrays it returns.  Every generator is
deterministic in (config, item) through numpy's SeedSequence/PCG64.
"""
from .generate import *  # noqa: F401,F403
from .generate import __all__  # noqa: F401
