"""Seeded synthetic inputs for the Couette workloads.

This module holds only parameter draws and random numbers: no part of the method's arithmetic.
Both the CPU oracle (through the tests) and the GPU path take their inputs from here.
"""
from .cases import *  # noqa: F401,F403
