"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package produces *data only*: mechanism tables (compositions, Arrhenius
parameters, thermodynamic and transport constants), initial fields (mass
fractions and temperature), random state batches for kernel tests and the
workload descriptions.  It contains none of the integration method's arithmetic
(no rates, no enthalpy-temperature relation, no quadrature, no solves): each
consumer converts these inputs with its own code.
"""
from .mechanism import make_mechanism, mlp_init, ELEMENT_MASSES, R_U, R_CAL, P_ATM
from .fields import (flame_1d, flame_2d, ensemble_flames, random_cell_batch,
                     random_helmholtz_problem)
from .configs import CONFIGS, config

__all__ = [
    "make_mechanism", "mlp_init", "ELEMENT_MASSES", "R_U", "R_CAL", "P_ATM",
    "flame_1d", "flame_2d", "ensemble_flames", "random_cell_batch",
    "random_helmholtz_problem", "CONFIGS", "config",
]
