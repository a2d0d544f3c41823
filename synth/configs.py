"""The five synthetic workloads (sizes and scheme parameters only).

Each entry names a mechanism recipe, a grid, a step size and the SDC scheme
parameters.  ``scheme`` is one of "misdc", "misdcq", "cisdcq"; ``nu`` is the
number of nested iterations per sweep of the concurrent scheme.
"""

CONFIGS = {
    # 1-D periodic flame, serial MISDC, 3 Gauss-Lobatto nodes, 4 sweeps, 10 steps
    "flame1d_64": dict(
        mech=dict(n_species=9, n_reactions=21, seed=0), dim=1, n=(64,), dx=(0.01,),
        u=(100.0,), dt=5e-5, n_nodes=3, sweeps=4, steps=10, scheme="misdc", nu=1,
        ic_seed=101),
    # 2-D periodic 256x256 flame, concurrent MISDC, 5 nodes, 6 sweeps
    "flame2d_256": dict(
        mech=dict(n_species=9, n_reactions=21, seed=0), dim=2, n=(256, 256),
        dx=(0.01, 0.01), u=(100.0, 0.0), dt=5e-5, n_nodes=5, sweeps=6, steps=1,
        scheme="cisdcq", nu=1, ic_seed=102),
    # 2-D 512x512, 53 species / 325 reactions with a rate-constant spread
    "flame2d_512_n53": dict(
        mech=dict(n_species=53, n_reactions=325, seed=1, rate_spread=(1e-2, 1e9)),
        dim=2, n=(512, 512), dx=(0.005, 0.005), u=(100.0, 0.0), dt=2.5e-5,
        n_nodes=5, sweeps=6, steps=1, scheme="cisdcq", nu=1, ic_seed=103),
    # 64 independent 1-D flames of uneven length with a 10x spread of step sizes
    "ensemble64": dict(
        mech=dict(n_species=9, n_reactions=21, seed=0), dim=1, n_flames=64,
        len_range=(128, 4096), dx=(0.01,), u=(100.0,), dt=5e-6, dt_spread=10.0,
        n_nodes=3, sweeps=4, steps=1, scheme="cisdcq", nu=1, ens_seed=5),
}


def config(name, **overrides):
    c = dict(CONFIGS[name])
    c.update(overrides)
    return c
