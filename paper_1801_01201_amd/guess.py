"""Training data and training of the learned Newton guess (the network runs
in the library; this module only moves device arrays between its calls).

Typical use::

    net = GuessNet(N)                              # (N+2) -> 256 -> 256 -> (N+1)
    net.set_params(initial_params)
    data = record_problems(mech, grid, states, dt, integ_opts)   # from real steps
    train(mech, net, *data, epochs=5)
    integ.set_guess(net)
"""
import numpy as np

from . import native as nat
from .flame import Integrator


def pack_params(layers):
    """Flat FP32 parameter vector in the library's layer order (W1, b1, W2,
    b2, ...; each W row-major, inputs by outputs) from a list of (W, b)."""
    return np.concatenate([np.concatenate([np.asarray(W, dtype=np.float32).ravel(),
                                           np.asarray(b, dtype=np.float32).ravel()])
                           for W, b in layers])


def record_problems(mech, grid, states, dt, **integ_opts):
    """Reaction problems (b_Y, h, c, Y*) of one step from each device state
    in ``states`` (each N+1 x cells, advanced in place), recorded by the
    integrator.  Returns device tensors b_Y (N, P), h (P), c (P), Y* (N, P)."""
    import torch
    N = mech.N
    n = grid.cells
    tasks = None
    parts = []
    for st in states:
        integ = Integrator(mech, grid, **integ_opts)
        nu = integ.opts.nu if integ.opts.scheme == nat.SCHEME["cisdcq"] else 1
        tasks = integ.opts.n_sweeps * nu * (integ.opts.n_nodes - 1)
        buf = torch.empty(tasks * (2 * N + 2) * n, dtype=torch.float64, device=st.device)
        integ.record(buf, tasks)
        integ.step(st, dt)
        got = integ.recorded()
        integ.close()
        parts.append(buf.view(tasks, 2 * N + 2, n)[:got])
    rec = torch.cat(parts)
    bY = rec[:, :N].permute(1, 0, 2).reshape(N, -1).contiguous()
    h = rec[:, N].reshape(-1).contiguous()
    c = rec[:, N + 1].reshape(-1).contiguous()
    Ys = rec[:, N + 2:].permute(1, 0, 2).reshape(N, -1).contiguous()
    return bY, h, c, Ys


def train(mech, net, bY, h, c, Ys, epochs=5, batch=4096, lr=2e-3, seed=0):
    """The library sets the network's normalisation from the data (means and
    standard deviations of the features and targets) and writes the
    normalised pairs in shuffled order, then trains on them.  Returns the
    per-epoch loss (host)."""
    import torch
    n = h.numel()
    N = net.N
    x = torch.empty((n, N + 2), dtype=torch.float32, device=h.device)
    t = torch.empty((n, N + 1), dtype=torch.float32, device=h.device)
    nat.misdc_mlp_prepare_training(mech.handle, net.handle, n, bY, h, c, Ys, seed, x, t)
    hist = torch.empty(epochs, dtype=torch.float32, device=h.device)
    nat.misdc_mlp_train(net.handle, n, x, t, batch, epochs, lr, hist)
    return hist.cpu().numpy()
