"""Host-side checks of the C ABI library: it loads, exports every declared
symbol, computes the SDC tables on the host, and rejects bad arguments
before touching the GPU (none of these tests needs a device)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle.coefficients import sdc_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "misdc.h")


@pytest.fixture(scope="module")
def nat():
    from paper_1801_01201_amd import native
    native.lib()
    return native


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(misdc_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(nat):
    lib = C.CDLL(nat.LIB_PATH)
    declared = _declared_functions()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(nat.EXPORTED) == declared


@pytest.mark.parametrize("n_nodes", range(2, 10))
@pytest.mark.parametrize("qi", ["lu", "be"])
@pytest.mark.parametrize("qe", ["cumulative", "literal"])
def test_host_tables_match_oracle(nat, n_nodes, qi, qe):
    a = nat.misdc_sdc_tables(n_nodes, qi, qe)
    b = sdc_tables(n_nodes, qi, qe)
    for k in ("tau", "Q", "QI", "QE"):
        ulps = np.abs(a[k] - b[k]) / np.spacing(np.maximum(np.abs(b[k]), 1e-300))
        assert np.all(ulps <= 2), (k, ulps.max())


def test_node_to_node_weights_are_differences_of_Q(nat):
    for n_nodes in (3, 5, 7):
        a = nat.misdc_sdc_tables(n_nodes)
        Q, S = a["Q"], a["S"]
        np.testing.assert_allclose(S[0], Q[0], atol=1e-16)
        np.testing.assert_allclose(S[1:], Q[1:] - Q[:-1], atol=2e-16)


def test_table_arguments_rejected(nat):
    with pytest.raises(nat.MisdcError) as e:
        nat.misdc_sdc_tables(1)
    assert e.value.code == nat.MISDC_EINVAL
    with pytest.raises(nat.MisdcError):
        nat.misdc_sdc_tables(10)
    rc = nat.lib().misdc_sdc_tables(5, 7, 0, None, None, None, None, None)
    assert rc == nat.MISDC_EINVAL


def test_grid_arguments_rejected(nat):
    for dim, n, dx, u in [(3, [8, 8], [0.1, 0.1], [0, 0]), (1, [2], [0.1], [0.0]),
                          (2, [8, 8], [0.1, -1.0], [0, 0]), (1, [8], [0.1], [np.inf])]:
        with pytest.raises(nat.MisdcError) as e:
            nat.misdc_grid_create(dim, n, dx, u)
        assert e.value.code == nat.MISDC_EINVAL
    with pytest.raises(nat.MisdcError):
        nat.misdc_grid_create_ensemble([64, 3], [0.1, 0.1], [1.0, 1.0])


def test_mechanism_validation_before_device(nat):
    m = synth.make_mechanism(9, 21, 0)
    bad = dict(m)
    bad["W"] = m["W"].copy()
    bad["W"][2] = -1.0
    with pytest.raises(nat.MisdcError) as e:
        nat.misdc_mech_create(bad)
    assert e.value.code == nat.MISDC_EINVAL
    bad = dict(m)
    bad["react"] = m["react"].copy()
    bad["react"][0, 0] = m["bath"]            # the bath may not react
    with pytest.raises(nat.MisdcError):
        nat.misdc_mech_create(bad)
    bad = dict(m)
    bad["prod"] = m["prod"].copy()
    bad["prod"][0] = [-1, -1]                 # no product
    with pytest.raises(nat.MisdcError):
        nat.misdc_mech_create(bad)
    bad = dict(m)
    bad["W"] = m["W"].copy()
    bad["W"][int(m["react"][0, 0])] *= 1.5    # unbalanced reaction
    with pytest.raises(nat.MisdcError) as e:
        nat.misdc_mech_create(bad)
    assert "balanced" in str(e.value)


def test_null_handles_rejected(nat):
    lib = nat.lib()
    assert lib.misdc_step(None, None, 1.0, None, None) == nat.MISDC_EINVAL
    assert lib.misdc_integ_create(None, None, None, C.byref(C.c_void_p())) == nat.MISDC_EINVAL
    assert lib.misdc_reaction_solve_batch(None, 1, None, None, None, None, None, None, None,
                                          None, None) == nat.MISDC_EINVAL
    assert lib.misdc_get_stats(None, None) == nat.MISDC_EINVAL
    assert lib.misdc_get_tune(None, None) == nat.MISDC_EINVAL
    assert lib.misdc_set_tune(None, None) == nat.MISDC_EINVAL
    assert lib.misdc_autotune(None, None, 1.0, None, 1, None, None) == nat.MISDC_EINVAL
    assert lib.misdc_step_begin(None, None, 1.0, None, None) == nat.MISDC_EINVAL
    assert lib.misdc_sweep(None, None) == nat.MISDC_EINVAL
    assert lib.misdc_step_end(None, None) == nat.MISDC_EINVAL
    assert lib.misdc_set_streams(None, None, None) == nat.MISDC_EINVAL
    assert lib.misdc_mlp_prepare_training(None, None, 4, None, None, None, None, 0, None, None,
                                          None) == nat.MISDC_EINVAL
    assert lib.misdc_integ_set_guess(None, None, 0) == nat.MISDC_EINVAL
    assert lib.misdc_integ_record(None, None, 0) == nat.MISDC_EINVAL
    o = nat.misdc_opts_default()
    assert (o.n_nodes, o.n_sweeps, o.nu, o.scheme) == (5, 6, 1, 2)
    assert o.use_graph == 0


def _header_struct_fields(name):
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    m = re.search(r"typedef struct\s*\{([^{}]*)\}\s*" + name + r"\s*;", text)
    assert m, name
    fields = []
    for decl in m.group(1).split(";"):
        decl = decl.strip()
        if not decl:
            continue
        fields.append(re.findall(r"([A-Za-z_][A-Za-z_0-9]*)\s*(?:\[[^\]]*\])?\s*$", decl)[0])
    return fields


@pytest.mark.parametrize("name", ["misdc_tune", "misdc_opts", "misdc_newton_opts", "misdc_stats"])
def test_binding_structs_match_header(nat, name):
    """The Python binding's ctypes structures list the header's fields in
    the header's order (the C ABI passes them by pointer)."""
    cls = getattr(nat, name)
    assert [f[0] for f in cls._fields_] == _header_struct_fields(name)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more it exits with a message
    before touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_generated_reaction_solve_compiles_on_the_host(nat):
    """The source of the reaction solve generated for the 9-species
    mechanism (every reaction written out with its constants) compiles for
    gfx950 with hiprtc, without a GPU; a mechanism beyond the generated
    kernel's species limit is refused."""
    mech = synth.make_mechanism(9, 21, 0)
    src = nat.misdc_mech_generate(mech, compile=True)
    assert 'extern "C" __global__' in src and "newton_spec" in src
    for j in range(mech["R"]):
        assert f"// reaction {j}\n" in src
    big = synth.make_mechanism(53, 325, 1)
    with pytest.raises(nat.MisdcError) as e:
        nat.misdc_mech_generate(big)
    assert e.value.code == nat.MISDC_EUNSUPPORTED
