"""Seeded synthetic placement instances.

This module only draws random numbers and lays them out in arrays; it holds
none of the placement method's arithmetic (no density, no transform, no
wirelength).  Both the FP64 oracle tests and the GPU path consume its output.
"""
from .instances import (  # noqa: F401
    Instance,
    make_instance,
    make_config,
    serving_pool,
    serving_requests,
    serving_stream,
    CONFIGS,
)
