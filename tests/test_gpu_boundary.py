"""GPU tests of the C ABI's contract around the step: the caller's streams
(misdc_set_streams), unconverged solves reported as MISDC_ENOTCONV
(misdc_get_stats, misdc_step_end), calls refused while a step is open, and
the training-set preparation of the learned guess (statistics against a
NumPy computation from the oracle's temperature, and the shuffle)."""
import numpy as np
import pytest

import synth
from oracle import chemistry as ch

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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
    return t.detach().cpu().numpy()


def _state(mh, mech9, nx, ny):
    from paper_1801_01201_amd.flame import initial_state
    Y, T = synth.flame_2d(mech9, nx, ny)
    st, _ = initial_state(mh, dev(Y.reshape(9, -1)), dev(T.ravel()))
    return st


def test_caller_streams_give_the_same_step(nat, mech9, mh):
    """A step on two torch streams equals the step on the integrator's own
    streams bit for bit (CISDCQ-2, so both streams carry work), also when
    the step is ordered after work on a third stream and after switching
    back to the integrator's streams."""
    from paper_1801_01201_amd.flame import Grid, Integrator
    g = Grid(2, [40, 32], [0.01, 0.01], [100.0, 0.0])
    dt = 5e-5
    integ = Integrator(mh, g, n_nodes=5, sweeps=3, nu=2, scheme="cisdcq")
    st0 = _state(mh, mech9, 40, 32)
    ref = st0.clone()
    integ.step(ref, dt)
    ref = host(ref)
    sd, sr, sc = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    integ.set_streams(sd, sr)
    st = st0.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(sc):
        st.mul_(1.0)                      # work on the caller's stream before the step
        integ.step(st, dt, stream=sc)
        out = st.clone()                  # ordered after the step on the same stream
    sc.synchronize()
    assert np.array_equal(host(out), ref)
    assert integ.stats()["converged"]
    # refused: the same stream twice, and a CU split of the caller's reaction stream
    with pytest.raises(nat.MisdcError) as e:
        integ.set_streams(sd, sd)
    assert e.value.code == nat.MISDC_EINVAL
    t = integ.tune()
    with pytest.raises(nat.MisdcError) as e:
        integ.set_tune(t["cg_variant"], t["cg_blocks"], t["cyclic"], 0, 2, 1)
    assert e.value.code == nat.MISDC_EINVAL
    # serialised onto the caller's diffusion stream, then back to its own
    integ.set_tune(t["cg_variant"], t["cg_blocks"], t["cyclic"], 1, 0, 0)
    st = st0.clone()
    integ.step(st, dt)
    assert np.array_equal(host(st), ref)
    integ.set_tune(t["cg_variant"], t["cg_blocks"], t["cyclic"], 0, 0, 1)
    integ.set_streams(None, None)
    st = st0.clone()
    integ.step(st, dt)
    assert np.array_equal(host(st), ref)
    # a step open: the streams cannot change
    integ.begin(st, dt)
    with pytest.raises(nat.MisdcError) as e:
        integ.set_streams(sd, sr)
    assert e.value.code == nat.MISDC_ESTATE
    integ.sweep()
    integ.end()
    integ.close()
    g.close()


def test_caller_streams_graph_replay(nat, mech9, mh):
    """The captured step replays on the caller's streams with the same
    result as eager execution."""
    from paper_1801_01201_amd.flame import Grid, Integrator
    g = Grid(2, [24, 20], [0.01, 0.01], [100.0, 0.0])
    dt = 5e-5
    st0 = _state(mh, mech9, 24, 20)
    eager = Integrator(mh, g, n_nodes=5, sweeps=2, nu=1, scheme="cisdcq")
    ref = st0.clone()
    eager.step(ref, dt)
    ref = host(ref)
    eager.close()
    integ = Integrator(mh, g, n_nodes=5, sweeps=2, nu=1, scheme="cisdcq", use_graph=True)
    sd, sr = torch.cuda.Stream(), torch.cuda.Stream()
    integ.set_streams(sd, sr)
    work = st0.clone()
    for rep in range(3):
        work.copy_(st0)
        integ.step(work, dt)
        assert np.array_equal(host(work), ref), rep
    integ.close()
    g.close()


def test_unconverged_newton_reported(nat, mech9, mh):
    """With one Newton iteration allowed the solves cannot converge: the
    step still runs, misdc_get_stats fills the counts and returns
    MISDC_ENOTCONV, and a step ended by misdc_step_end returns it too."""
    from paper_1801_01201_amd.flame import Grid, Integrator
    g = Grid(2, [24, 20], [0.01, 0.01], [100.0, 0.0])
    newton = nat.newton_opts(maxit=1)
    integ = Integrator(mh, g, n_nodes=3, sweeps=2, nu=1, scheme="cisdcq", newton=newton)
    st = _state(mh, mech9, 24, 20)
    integ.step(st, 5e-5)
    s = integ.stats()
    assert not s["converged"]
    assert s["newton_failed"] > 0
    code = nat.lib().misdc_get_stats(integ.handle, nat.C.byref(nat.misdc_stats()))
    assert code == nat.MISDC_ENOTCONV
    assert "Newton" in nat.lib().misdc_last_error().decode()
    integ.begin(st, 5e-5)
    integ.sweep()
    with pytest.raises(nat.MisdcError) as e:
        integ.end()
    assert e.value.code == nat.MISDC_ENOTCONV
    # the step is closed all the same
    integ.begin(st, 5e-5)
    integ.sweep()
    with pytest.raises(nat.MisdcError):
        integ.end()
    integ.close()
    # the default limits converge from a fresh state: OK from both calls
    st = _state(mh, mech9, 24, 20)
    integ = Integrator(mh, g, n_nodes=3, sweeps=2, nu=1, scheme="cisdcq")
    integ.begin(st, 5e-5)
    integ.sweep()
    integ.end()
    assert integ.stats()["converged"]
    integ.close()
    g.close()


def test_unconverged_diffusion_reported(nat, mech9, mh):
    """A diffusion solve stopped at its iteration limit (cg_maxit = 2 with a
    tolerance no two iterations reach) counts in cg_failed and makes
    misdc_get_stats return MISDC_ENOTCONV."""
    from paper_1801_01201_amd.flame import Grid, Integrator
    g = Grid(2, [40, 32], [0.01, 0.01], [100.0, 0.0])
    integ = Integrator(mh, g, n_nodes=3, sweeps=1, nu=1, scheme="cisdcq", cg_maxit=2,
                       cg_rtol=1e-14)
    st = _state(mh, mech9, 40, 32)
    integ.step(st, 5e-5)
    s = integ.stats()
    assert s["cg_failed"] > 0 and not s["converged"]
    integ.close()
    g.close()


def test_guess_and_record_refused_while_a_step_is_open(nat, mech9, mh):
    from paper_1801_01201_amd.flame import Grid, Integrator
    g = Grid(2, [24, 20], [0.01, 0.01], [100.0, 0.0])
    integ = Integrator(mh, g, n_nodes=3, sweeps=1, nu=1, scheme="cisdcq")
    st = _state(mh, mech9, 24, 20)
    buf = torch.empty(4 * 20 * 480, dtype=torch.float64, device="cuda")
    integ.begin(st, 5e-5)
    for call in (lambda: integ.set_guess(None), lambda: integ.record(buf, 4),
                 lambda: integ.record(buf, 0)):
        with pytest.raises(nat.MisdcError) as e:
            call()
        assert e.value.code == nat.MISDC_ESTATE
    integ.sweep()
    integ.end()
    integ.record(buf, 4)                  # accepted once the step is ended
    integ.record(buf, 0)
    integ.set_guess(None)
    integ.close()
    g.close()


def test_training_set_statistics_and_shuffle(nat, mech9, mh):
    """misdc_mlp_prepare_training: the normalisation it sets equals the
    means and sample standard deviations of the raw features (b_Y, T_b from
    the oracle's temperature, ln c) and targets computed in NumPy, with the
    stated floors (checked through misdc_mlp_features and _targets, which
    apply it); its rows are the same rows in another order; another seed
    gives another order."""
    from paper_1801_01201_amd.flame import GuessNet
    rng = np.random.Generator(np.random.PCG64(11))
    n = 5000
    Y, T = synth.flame_2d(mech9, 100, 50)
    bY = np.ascontiguousarray(Y.reshape(9, -1))
    h = ch.enthalpy(mech9, bY, T.ravel())
    Ys = np.clip(bY + 1e-3 * rng.standard_normal(bY.shape) * bY, 0.0, None)
    c = 10.0 ** rng.uniform(-6, -4, n)
    Tb = ch.temperature(mech9, bY, h)
    Ts = ch.temperature(mech9, Ys, h)
    feats = np.vstack([bY, Tb[None], np.log(c)[None]]).T           # n x 11
    targs = np.vstack([Ys - bY, (Ts - Tb)[None]]).T                 # n x 10
    mu = feats.mean(0)
    sd = np.maximum(feats.std(0, ddof=1), np.maximum(1e-3 * np.abs(mu), 1e-6))
    osd = np.maximum(targs.std(0, ddof=1), 1e-30)
    x_ref = ((feats - mu.astype(np.float32)) / sd.astype(np.float32))
    t_ref = targs / osd.astype(np.float32)
    net = GuessNet(9, 32, "fp32")
    dbY, dh, dc, dYs = dev(bY), dev(h), dev(c), dev(Ys)
    x = torch.empty((n, 11), dtype=torch.float32, device="cuda")
    t = torch.empty((n, 10), dtype=torch.float32, device="cuda")
    nat.misdc_mlp_prepare_training(mh.handle, net.handle, n, dbY, dh, dc, dYs, 3, x, t)
    xs, ts = host(x).astype(np.float64), host(t).astype(np.float64)
    # the same normalisation applied in problem order
    x1 = torch.empty_like(x)
    t1 = torch.empty_like(t)
    nat.misdc_mlp_features(mh.handle, net.handle, n, dbY, dh, dc, x1)
    nat.misdc_mlp_targets(mh.handle, net.handle, n, dbY, dh, dYs, t1)
    xp, tp = host(x1).astype(np.float64), host(t1).astype(np.float64)
    assert np.abs(xp - x_ref).max() <= 2e-4 * max(1.0, np.abs(x_ref).max())
    assert np.abs(tp - t_ref).max() <= 2e-4 * np.abs(t_ref).max()
    # shuffled rows: a permutation of the ordered ones, not the identity
    key = np.lexsort(xp.T[::-1])
    keys = np.lexsort(xs.T[::-1])
    assert np.array_equal(xp[key], xs[keys])
    assert np.array_equal(tp[key], ts[keys])
    assert not np.array_equal(xp, xs)
    x2 = torch.empty_like(x)
    t2 = torch.empty_like(t)
    nat.misdc_mlp_prepare_training(mh.handle, net.handle, n, dbY, dh, dc, dYs, 4, x2, t2)
    assert not np.array_equal(host(x2), xs)
    net.close()
