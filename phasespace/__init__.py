"""Seeded synthetic phase-space inputs shared by the oracle, the tests and the bench.

This package holds no matrix-element arithmetic: it only draws massless
momenta (RAMBO), applies the jet cuts of the paper (section 2.2, eqs. cuts) and
draws helicity patterns for the Monte Carlo helicity mode,
so that the oracle and the HIP path consume the very same momentum buffers.
"""
from .rambo import (  # noqa: F401
    rambo_massless,
    apply_cuts,
    generate_events,
    random_helicities,
    rambo_uniforms,
    Kinematics,
    KIN_C1,
    KIN_C2,
    KIN_C5,
)
