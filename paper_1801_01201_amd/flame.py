"""Flame workloads on the GPU: handles for a mechanism and a grid, the
initial state, and the integrator.  Thin wrappers over the C ABI; all
arithmetic runs in the library's kernels.
"""
import numpy as np

from . import native as nat

# Length of the backward-Euler reaction solve that relaxes the synthetic
# initial composition onto the fast chemical manifold (s).
RELAX_TIME = 1.0


class Mechanism:
    def __init__(self, mech):
        self.desc = mech
        self.N = int(mech["N"])
        self.handle = nat.misdc_mech_create(mech)

    def close(self):
        if self.handle:
            nat.misdc_mech_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Grid:
    def __init__(self, dim=None, n=None, dx=None, u=None, ensemble=None):
        if ensemble is not None:
            lengths, dxs, us = ensemble
            self.handle = nat.misdc_grid_create_ensemble(lengths, dxs, us)
            self.cells = int(np.sum(lengths))
        else:
            self.handle = nat.misdc_grid_create(dim, n, dx, u)
            self.cells = int(np.prod(n))

    def close(self):
        if self.handle:
            nat.misdc_grid_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def initial_state(mech, Y, T, relax_time=RELAX_TIME, stream=None):
    """State (N+1, cells) on the device from synthetic (Y, T) device tensors:
    h = enthalpy(Y, T), then one constant-enthalpy backward-Euler reaction
    solve of length ``relax_time`` started from Y.  Returns (state, iters)."""
    import torch
    N = mech.N
    n = T.numel()
    Yc = Y.reshape(N, n).contiguous()
    state = torch.empty((N + 1, n), dtype=torch.float64, device=Y.device)
    nat.misdc_enthalpy(mech.handle, n, Yc, T.reshape(n).contiguous(), state[N], stream)
    state[:N].copy_(Yc)
    c = torch.full((n,), float(relax_time), dtype=torch.float64, device=Y.device)
    iters = torch.empty(n, dtype=torch.int32, device=Y.device)
    bY = Yc.clone()
    nat.misdc_reaction_solve_batch(mech.handle, n, bY, state[N], c, state[:N], None, None, iters,
                                   stream=stream)
    return state, iters


class Integrator:
    def __init__(self, mech, grid, **opts):
        self.mech, self.grid = mech, grid
        self.opts = nat.make_opts(**opts)
        self.handle = nat.misdc_integ_create(mech.handle, grid.handle, self.opts)

    def step(self, state, dt, dt_per_flame=None, stream=None):
        """One step; ``dt_per_flame`` (device tensor, one dt per flame of an
        ensemble grid) replaces the scalar ``dt``."""
        nat.misdc_step(self.handle, state, dt, dt_per_flame, stream)

    def begin(self, state, dt, dt_per_flame=None, stream=None):
        """Open a step (I1-I4) to be advanced one sweep at a time."""
        nat.misdc_step_begin(self.handle, state, dt, dt_per_flame, stream)

    def sweep(self, stream=None):
        """One more correction sweep of the open step."""
        nat.misdc_sweep(self.handle, stream)

    def end(self, stream=None):
        """Write the open step's result into its state."""
        nat.misdc_step_end(self.handle, stream)

    def autotune(self, state, dt, dt_per_flame=None, reps=3, stream=None):
        return nat.misdc_autotune(self.handle, state, dt, dt_per_flame, reps, stream)

    def set_guess(self, net, sweeps=0):
        """Start the reaction solves of the first ``sweeps`` sweeps (0: all)
        from the learned guess where it has the smaller residual (``net``: a
        ``GuessNet``, or None)."""
        nat.misdc_integ_set_guess(self.handle, net.handle if net is not None else None, sweeps)

    def record(self, buf, max_tasks):
        """Record the reaction problems of later steps into ``buf`` (device,
        float64, max_tasks * (2N + 2) * cells); max_tasks 0 stops."""
        nat.misdc_integ_record(self.handle, buf, max_tasks)

    def recorded(self):
        return nat.misdc_integ_recorded(self.handle)

    def set_streams(self, diffusion_stream=None, reaction_stream=None):
        """Issue the diffusion and reaction tasks on the caller's streams
        (None: the integrator's own)."""
        nat.misdc_set_streams(self.handle, diffusion_stream, reaction_stream)

    def tune(self):
        return nat.misdc_get_tune(self.handle)

    def set_tune(self, cg_variant, cg_blocks, cyclic, serialize, cu_split=0, stagger=0, fused=0):
        nat.misdc_set_tune(self.handle, cg_variant, cg_blocks, cyclic, serialize, cu_split,
                           stagger, fused)

    def stats(self):
        return nat.misdc_get_stats(self.handle)

    def newton_histogram(self, sweep):
        return nat.misdc_get_newton_histogram(self.handle, sweep)

    def close(self):
        if self.handle:
            nat.misdc_integ_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GuessNet:
    """Dense network of the learned Newton guess, (N+2) -> H -> H -> (N+1),
    held by the library (parameters, Adam state and work buffers on the
    device)."""

    def __init__(self, n_species, hidden=256, precision="bf16"):
        self.N = int(n_species)
        self.sizes = [self.N + 2, hidden, hidden, self.N + 1]
        self.handle = nat.misdc_mlp_create(self.N + 2, hidden, self.N + 1, precision)

    def param_count(self):
        return nat.misdc_mlp_param_count(self.handle)

    def set_params(self, flat):
        nat.misdc_mlp_set_params(self.handle, flat)

    def params(self):
        return nat.misdc_mlp_get_params(self.handle)

    def set_normalization(self, in_mu, in_sd, out_sd):
        nat.misdc_mlp_set_normalization(self.handle, in_mu, in_sd, out_sd)

    def close(self):
        if self.handle:
            nat.misdc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
