"""Model descriptions, the model blob, and seeded synthetic inputs.

Shared by the GPU library's users and by the FP64 reference checks; holds none of the
physics step's arithmetic.
"""
from . import inputs, model, robots  # noqa: F401
from .model import Model  # noqa: F401
