"""The diffusion solve that allocates nothing (misdc_diffusion_solve_noalloc,
called through the C ABI) against misdc_diffusion_solve, which allocates its
workspace: the same result bit for bit and the same iteration count, on two
calls in a row with the second on a smaller grid (the shared scratch keeps
the first call's contents), on a 1-D grid, at the largest grid the scratch
holds (256 x 256 at 9 species), and a grid too large for it refused before
any work."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nat():
    from paper_1801_01201_amd import native
    native.lib()
    return native


@pytest.fixture(scope="module")
def mh(nat):
    from paper_1801_01201_amd.flame import Mechanism
    m = Mechanism(synth.make_mechanism(9, 21, 0))
    yield m
    m.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _solve(nat, fn, mh, g, c, T, rhs, y0):
    y = y0.clone()
    it = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    code = fn(mh.handle, g, float(c), T.data_ptr(), rhs.data_ptr(), y.data_ptr(), 1, 1e-13, 0,
              it.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert code == nat.MISDC_OK, nat.lib().misdc_last_error().decode()
    torch.cuda.synchronize()
    return y.cpu().numpy(), int(it.cpu()[0])


@pytest.mark.parametrize("shapes", [[(256, 256), (37, 29)], [(64, 96), (20, 24)],
                                    [(4096,), (64,)]])
def test_noalloc_matches_allocating_solve(nat, mh, shapes):
    lib = nat.lib()
    for k, shape in enumerate(shapes):
        dim = len(shape)
        n = list(shape)[::-1]
        g = nat.misdc_grid_create(dim, n, [0.01] * dim, [100.0, -40.0][:dim])
        T, rhs = synth.random_helmholtz_problem(shape, 10, seed=20 + k)
        Td, rd = dev(T.ravel()), dev(rhs.reshape(10, -1))
        y0 = dev(rhs.reshape(10, -1) * 0.9)         # an initial guess in y
        ref, it_ref = _solve(nat, lib.misdc_diffusion_solve, mh, g, 1.2e-5, Td, rd, y0)
        got, it_got = _solve(nat, lib.misdc_diffusion_solve_noalloc, mh, g, 1.2e-5, Td, rd, y0)
        assert np.array_equal(got, ref), shape
        assert it_got == it_ref, (shape, it_got, it_ref)
        nat.misdc_grid_destroy(g)


def test_noalloc_refuses_grids_beyond_its_scratch(nat, mh):
    lib = nat.lib()
    g = nat.misdc_grid_create(2, [512, 512], [0.01, 0.01], [0.0, 0.0])
    y = torch.zeros((10, 4), dtype=torch.float64, device="cuda")
    code = lib.misdc_diffusion_solve_noalloc(mh.handle, g, 1e-5, y.data_ptr(), y.data_ptr() + 8,
                                             y.data_ptr() + 16, 0, 0.0, 0, None, None)
    assert code == nat.MISDC_EINVAL
    assert "scratch" in lib.misdc_last_error().decode()
    nat.misdc_grid_destroy(g)
