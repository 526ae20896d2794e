"""Seeded synthetic inputs (morphologies and cable coefficients) shared by the
FP64 oracle and the GPU library.  numpy only; no step of the solve lives here."""
from .trees import (CableSystem, Forest, assemble, cable_values, full_binary_forest, grow_level_forest,
                    grow_random_forest)
from . import configs

__all__ = ["CableSystem", "Forest", "assemble", "cable_values", "full_binary_forest", "grow_level_forest",
           "grow_random_forest", "configs"]
