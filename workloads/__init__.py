"""Seeded synthetic inputs for the inaccessibility-measure-field (IMF) workloads.

This package only draws inputs: designs, fixtures, tool shapes and orientation
sets.  It holds none of the method's arithmetic, so both the oracle tests and the
HIP path can use it without sharing any computation.
"""
from .gen import *  # noqa: F401,F403
