"""Seeded synthetic input fields shared by the tests, the smoke check and the
benchmark.  Holds no step of the compression method: only the random fields
that stand in for the paper's scientific datasets and the error bounds taken
relative to their value range."""
from .fields import (batch_arena, batch_specs, batch_field, batch_field_device, climate_steps, climate_steps_device, grf_3d, rel_eb,  # noqa: F401
                     sinusoid_1d, value_range)
