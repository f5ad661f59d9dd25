"""Seeded synthetic grain maps and parameter draws.

The one module shared by the oracle side and the GPU side of the test suite and
the benchmark.  It draws random inputs and labels pixels by the physical
definitions of the diagrams it samples; it holds none of the objective, gradient
or assignment arithmetic that is being tested.
"""
from .maps import *  # noqa: F401,F403
from .points import power_points  # noqa: F401
