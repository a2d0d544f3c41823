"""GPU parity of the learned Newton guess: the network's forward pass,
gradients and Adam step (the library's MFMA kernels) against the NumPy
oracle in the same rounding mode, training progress, and the guess inside
the reaction solve and the integrator.

Tolerances (per tensor, max |gpu - ref| / max |ref|): 1e-2 with bfloat16
operands (the oracle rounds at the same points but accumulates in FP64; a
BF16 rounding of a hidden activation may fall on the other side, 2^-8
relative), 1e-5 with FP32 operands.
"""
import numpy as np
import pytest

import synth
from oracle import chemistry as ch
from oracle import mlp as om

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
TOL = {"bf16": 1e-2, "fp32": 1e-5}


@pytest.fixture(scope="module")
def nat():
    from paper_1801_01201_amd import native
    native.lib()
    return native


@pytest.fixture(scope="module")
def mech9():
    return synth.make_mechanism(9, 21, 0)


@pytest.fixture(scope="module")
def mh(nat, mech9):
    from paper_1801_01201_amd.flame import Mechanism
    m = Mechanism(mech9)
    yield m
    m.close()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def _net(nat, sizes, precision, seed):
    from paper_1801_01201_amd.flame import GuessNet
    rng = np.random.Generator(np.random.PCG64(seed))
    params = synth.mlp_init(sizes, seed)
    params = [(W, (rng.standard_normal(W.shape[1]) * 0.1).astype(np.float32).astype(np.float64))
              for W, _ in params]
    net = GuessNet(sizes[0] - 2, sizes[1], precision)
    net.set_params(om.pack(params).astype(np.float32))
    return net, params


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("B", [1, 77, 1000])
def test_forward_parity(nat, precision, B):
    sizes = [11, 256, 256, 10]
    net, params = _net(nat, sizes, precision, 3)
    rng = np.random.Generator(np.random.PCG64(B))
    X = rng.standard_normal((B, 11)).astype(np.float32).astype(np.float64)
    y = torch.empty((B, 10), dtype=torch.float32, device="cuda")
    nat.misdc_mlp_forward(net.handle, B, dev(X, torch.float32), y)
    ref = om.forward(params, X, precision)[-1]
    assert rel(host(y), ref) <= TOL[precision]
    net.close()


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
@pytest.mark.parametrize("sizes,B", [([11, 256, 256, 10], 333), ([55, 256, 256, 54], 129),
                                     ([11, 256, 256, 10], 4096)])
def test_gradient_parity(nat, precision, sizes, B):
    net, params = _net(nat, sizes, precision, 5)
    rng = np.random.Generator(np.random.PCG64(7))
    X = rng.standard_normal((B, sizes[0])).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((B, sizes[-1])).astype(np.float32).astype(np.float64)
    g = torch.empty(net.param_count(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    nat.misdc_mlp_gradients(net.handle, B, dev(X, torch.float32), dev(T, torch.float32), g, loss)
    grads, L = om.gradients(params, X, T, precision)
    got = om.unpack(host(g), sizes)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(got, grads)):
        assert rel(gW, rW) <= TOL[precision], (l, "W", rel(gW, rW))
        assert rel(gb, rb) <= TOL[precision], (l, "b", rel(gb, rb))
    assert abs(float(host(loss)[0]) - L) <= TOL[precision] * L
    net.close()


def test_gradients_deterministic(nat):
    sizes = [11, 256, 256, 10]
    net, params = _net(nat, sizes, "bf16", 9)
    rng = np.random.Generator(np.random.PCG64(1))
    X = dev(rng.standard_normal((5000, 11)), torch.float32)
    T = dev(rng.standard_normal((5000, 10)), torch.float32)
    g1 = torch.empty(net.param_count(), dtype=torch.float32, device="cuda")
    g2 = torch.empty_like(g1)
    nat.misdc_mlp_gradients(net.handle, 5000, X, T, g1)
    nat.misdc_mlp_gradients(net.handle, 5000, X, T, g2)
    assert torch.equal(g1, g2)
    net.close()


def test_adam_step_parity(nat):
    sizes = [11, 256, 256, 10]
    net, params = _net(nat, sizes, "fp32", 11)
    rng = np.random.Generator(np.random.PCG64(2))
    X = rng.standard_normal((64, 11)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((64, 10)).astype(np.float32).astype(np.float64)
    g = torch.empty(net.param_count(), dtype=torch.float32, device="cuda")
    p = params
    m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    for t in (1, 2, 3):
        nat.misdc_mlp_gradients(net.handle, 64, dev(X, torch.float32), dev(T, torch.float32), g)
        gr = om.unpack(host(g), sizes)
        nat.misdc_mlp_adam_step(net.handle, g, 1e-3)
        p, m, v = om.adam_step(p, gr, m, v, t, 1e-3)
    got = om.unpack(net.params().astype(np.float64), sizes)
    for (W, b), (rW, rb) in zip(got, p):
        assert np.abs(W - rW).max() <= 1e-6
        assert np.abs(b - rb).max() <= 1e-6
    net.close()


def test_training_fits_a_teacher(nat):
    """Training on the GPU (forward, gradients, Adam) fits the outputs of a
    fixed random teacher network of the same shape: the loss falls by an
    order of magnitude."""
    sizes = [11, 256, 256, 10]
    teacher = synth.mlp_init(sizes, 21)
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((32768, 11))
    Y = om.forward(teacher, X)[-1]
    Y = Y / Y.std()
    net, _ = _net(nat, sizes, "bf16", 22)
    x, t = dev(X, torch.float32), dev(Y, torch.float32)
    g = torch.empty(net.param_count(), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    nat.misdc_mlp_gradients(net.handle, 32768, x, t, g, loss)
    l0 = float(host(loss)[0])
    hist = torch.empty(20, dtype=torch.float32, device="cuda")
    nat.misdc_mlp_train(net.handle, 32768, x, t, 1024, 20, 1e-3, hist)
    nat.misdc_mlp_gradients(net.handle, 32768, x, t, g, loss)
    l1 = float(host(loss)[0])
    assert np.all(np.isfinite(host(hist)))
    assert l1 < 0.1 * l0, (l0, l1)
    net.close()


def test_guess_leaves_roots_unchanged(nat, mech9, mh):
    """Whatever the network predicts (here: untrained), the solve converges
    to the oracle's root, and a cell takes the learned guess only where its
    residual is smaller."""
    from paper_1801_01201_amd.flame import GuessNet
    n = 500
    Yb, Tb, c, Yg = synth.random_cell_batch(mech9, n, seed=31)
    h = ch.enthalpy(mech9, Yb, Tb)
    net, _ = _net(nat, [11, 256, 256, 10], "bf16", 33)
    Y = dev(Yg)
    choice = torch.zeros(n, dtype=torch.int32, device="cuda")
    nat.misdc_reaction_guess_mlp(mh.handle, net.handle, n, dev(Yb), dev(h), dev(c), Y, choice)
    it = torch.empty(n, dtype=torch.int32, device="cuda")
    nat.misdc_reaction_solve_batch(mh.handle, n, dev(Yb), dev(h), dev(c), Y, None, None, it)
    Yr, Tr, itr = ch.reaction_solve(mech9, c, Yb, h, Yg)
    assert np.all(host(it) > 0)
    assert np.abs(host(Y) - Yr).max() <= 1e-11
    ch_ = host(choice)
    assert set(np.unique(ch_)) <= {0, 1}
    net.close()


def _record_problems(nat, mh, mech9, seeds, nx, ny, dt):
    """Reaction problems (b_Y, h, c, Y*) of one CISDCQ step of flames with
    the given initial-condition seeds, recorded by the integrator."""
    from paper_1801_01201_amd.flame import Grid, Integrator, initial_state
    g = Grid(2, [nx, ny], [0.01, 0.01], [100.0, 0.0])
    n = nx * ny
    tasks = 6 * 4
    out = []
    for s in seeds:
        Y, T = synth.flame_2d(mech9, nx, ny, seed=s)
        st, _ = initial_state(mh, dev(Y.reshape(9, -1)), dev(T.ravel()))
        integ = Integrator(mh, g, n_nodes=5, sweeps=6, scheme="cisdcq")
        buf = torch.empty(tasks * 20 * n, dtype=torch.float64, device="cuda")
        integ.record(buf, tasks)
        integ.step(st, dt)
        assert integ.recorded() == tasks
        integ.close()
        out.append(buf.view(tasks, 20, n))
    g.close()
    rec = torch.cat(out)                         # (tasks, 20, n)
    bY = rec[:, :9].permute(1, 0, 2).reshape(9, -1).contiguous()
    hh = rec[:, 9].reshape(-1).contiguous()
    cc = rec[:, 10].reshape(-1).contiguous()
    Ys = rec[:, 11:].permute(1, 0, 2).reshape(9, -1).contiguous()
    return bY, hh, cc, Ys


def train_guess_net(nat, mh, net, bY, hh, cc, Ys, epochs=30, batch=4096, lr=2e-3, seed=0):
    """Normalisation from the data and shuffled, normalised pairs (one
    library call), then GPU training on them."""
    n = hh.numel()
    N = net.N
    x = torch.empty((n, N + 2), dtype=torch.float32, device="cuda")
    t = torch.empty((n, N + 1), dtype=torch.float32, device="cuda")
    nat.misdc_mlp_prepare_training(mh.handle, net.handle, n, bY, hh, cc, Ys, seed, x, t)
    hist = torch.empty(epochs, dtype=torch.float32, device="cuda")
    nat.misdc_mlp_train(net.handle, n, x, t, batch, epochs, lr, hist)
    return host(hist)


def test_learned_guess_in_the_integrator(nat, mech9, mh):
    """Train on the reaction problems of flames with initial-condition seeds
    200..203 (64 x 64), then step the benchmark's flame (held out) with and
    without the learned guess: the states agree to the Newton tolerance, the
    learned guess is taken in some cells, and the trained network predicts
    the held-out increments far better than the zero increment."""
    from paper_1801_01201_amd.flame import GuessNet, Grid, Integrator, initial_state
    dt = 5e-5
    bY, hh, cc, Ys = _record_problems(nat, mh, mech9, [200, 201, 202, 203], 64, 64, dt)
    net = GuessNet(9, 256, "bf16")
    net.set_params(om.pack(synth.mlp_init(net.sizes, 7)).astype(np.float32))
    hist = train_guess_net(nat, mh, net, bY, hh, cc, Ys, epochs=20)
    assert hist[-1] < 0.7 * hist[0], hist       # hist[0]: already after one epoch
    # held-out problems: prediction error vs the zero increment
    hb, hhb, hcc, hYs = _record_problems(nat, mh, mech9, [102], 64, 64, dt)
    n = hhb.numel()
    x = torch.empty((n, 11), dtype=torch.float32, device="cuda")
    t = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    y = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    nat.misdc_mlp_features(mh.handle, net.handle, n, hb, hhb, hcc, x)
    nat.misdc_mlp_targets(mh.handle, net.handle, n, hb, hhb, hYs, t)
    nat.misdc_mlp_forward(net.handle, n, x, y)
    err_net = float(((y - t) ** 2).mean())
    err_zero = float((t ** 2).mean())
    assert err_net < 0.2 * err_zero, (err_net, err_zero)
    # the held-out flame stepped with and without the guess
    Y, T = synth.flame_2d(mech9, 64, 64)
    g = Grid(2, [64, 64], [0.01, 0.01], [100.0, 0.0])
    outs, stats = [], []
    for use in (False, True):
        st, _ = initial_state(mh, dev(Y.reshape(9, -1)), dev(T.ravel()))
        integ = Integrator(mh, g, n_nodes=5, sweeps=6, scheme="cisdcq")
        if use:
            integ.set_guess(net)
        integ.step(st, dt)
        stats.append(integ.stats())
        outs.append(host(st))
        integ.close()
    g.close()
    assert stats[0]["newton_failed"] == 0 and stats[1]["newton_failed"] == 0
    assert stats[1]["newton_guess_learned"] > 0
    a, b = outs
    err = float((np.abs(a - b).max(axis=1) / np.abs(a).max(axis=1)).max())
    assert err <= 1e-10, err
    print("newton iterations per cell: plain %.4f learned %.4f (learned guess taken in %d of %d)"
          % (stats[0]["newton_iters"] / stats[0]["newton_solves"],
             stats[1]["newton_iters"] / stats[1]["newton_solves"],
             stats[1]["newton_guess_learned"], stats[1]["newton_solves"]))
    net.close()


def _relaxation_problems(nat, mh, mech9, seeds, nx, ny):
    """Cold-start reaction problems: the synthetic flame states b with
    c = 1 s (the relaxation that prepares an initial state), solved from
    the plain guess Y = b.  Returns (b_Y, h, c, Y*, iterations)."""
    from paper_1801_01201_amd.flame import RELAX_TIME
    bs, hs, Ys, its = [], [], [], []
    for s in seeds:
        Y, T = synth.flame_2d(mech9, nx, ny, seed=s)
        n = nx * ny
        b = dev(Y.reshape(9, -1))
        h = torch.empty(n, dtype=torch.float64, device="cuda")
        nat.misdc_enthalpy(mh.handle, n, b, dev(T.ravel()), h)
        Yo = b.clone()
        it = torch.empty(n, dtype=torch.int32, device="cuda")
        c = torch.full((n,), RELAX_TIME, dtype=torch.float64, device="cuda")
        nat.misdc_reaction_solve_batch(mh.handle, n, b, h, c, Yo, None, None, it)
        bs.append(b), hs.append(h), Ys.append(Yo), its.append(it)
    b = torch.cat(bs, dim=1).contiguous()
    h = torch.cat(hs).contiguous()
    return b, h, torch.full_like(h, RELAX_TIME), torch.cat(Ys, dim=1).contiguous(), torch.cat(its)


def test_learned_guess_cold_start_gain(nat, mech9, mh):
    """Where the plain guess is poor (cold starts: the 1 s relaxation of a
    synthetic composition, started from b), the learned guess cuts the
    Newton iterations; the roots stay the oracle-checked ones of the plain
    solve (same unique root, Newton tolerance)."""
    from paper_1801_01201_amd.flame import GuessNet
    bY, hh, cc, Ys, it_train = _relaxation_problems(nat, mh, mech9, [200, 201, 202, 203], 64, 64)
    assert bool((it_train > 0).all())
    net = GuessNet(9, 256, "bf16")
    net.set_params(om.pack(synth.mlp_init(net.sizes, 7)).astype(np.float32))
    train_guess_net(nat, mh, net, bY, hh, cc, Ys, epochs=40, batch=2048)
    hb, hhb, hcc, hYs, it_plain = _relaxation_problems(nat, mh, mech9, [102], 64, 64)
    n = hhb.numel()
    Y = hb.clone()
    choice = torch.zeros(n, dtype=torch.int32, device="cuda")
    nat.misdc_reaction_guess_mlp(mh.handle, net.handle, n, hb, hhb, hcc, Y, choice)
    it = torch.empty(n, dtype=torch.int32, device="cuda")
    nat.misdc_reaction_solve_batch(mh.handle, n, hb, hhb, hcc, Y, None, None, it)
    itp, itl = host(it_plain), host(it)
    assert np.all(itl > 0)
    assert np.abs(host(Y) - host(hYs)).max() <= 1e-11
    taken = float(host(choice).mean())
    print("cold start: newton iterations per cell plain %.3f learned %.3f (learned guess taken "
          "in %.1f %% of cells)" % (itp.mean(), itl.mean(), 100 * taken))
    assert itl.mean() < 0.8 * itp.mean()
    net.close()
