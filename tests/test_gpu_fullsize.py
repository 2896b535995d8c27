"""Parity at the benchmark's full size and launch configuration: 8192 x 8192
FP32, periodic 2D box stencils of order 1..4, every path, checked on sampled
windows (the oracle's light-cone windows, including corners and edges)."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, torch_cuda

pytestmark = pytest.mark.gpu

DIMS = (8192, 8192)
STEPS = 6
WINDOWS = [(0, 0), (0, 8192 - 16), (8192 - 16, 0), (8192 - 16, 8192 - 16), (4000, 5000), (63, 64 * 77 - 8)]


@pytest.fixture(scope="module")
def grid0():
    return inputs.grid(DIMS, seed=201)


@pytest.mark.parametrize("path", [st.PATH_GATHER, st.PATH_MFMA, st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_fullsize_windows(grid0, path, r):
    torch = torch_cuda()
    c = inputs.coefficients(2, r, st.BOX, seed=2100 + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    plan = st.Plan(DIMS, r, st.BOX, c, boundary=st.BC_PERIODIC, dtype=st.F32, path=path)
    x = torch.from_numpy(grid0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), STEPS)
    torch.cuda.synchronize()
    tol = error_bound(ce, 2, r, st.BOX, st.F32, path, STEPS, 1.0)
    for lo in WINDOWS:
        want = oracle.window(grid0, ce, r, st.BOX, st.BC_PERIODIC, STEPS, lo, (16, 16))
        got = res[lo[0]:lo[0] + 16, lo[1]:lo[1] + 16].cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= tol, (lo, np.abs(got - want).max(), tol)
    plan.close()


@pytest.mark.parametrize("r,tb", [(1, 12), (1, 4), (2, 6), (3, 4), (4, 3)])
def test_fullsize_windows_time_blocked(grid0, r, tb):
    """Time-blocked gather at full size: STEPS = 6 is a partial last launch
    for every time block here except 6 and 3."""
    torch = torch_cuda()
    c = inputs.coefficients(2, r, st.BOX, seed=2100 + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    plan = st.Plan(DIMS, r, st.BOX, c, boundary=st.BC_PERIODIC, dtype=st.F32, time_block=tb)
    assert plan.info["time_block"] == tb
    x = torch.from_numpy(grid0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), STEPS)
    torch.cuda.synchronize()
    tol = error_bound(ce, 2, r, st.BOX, st.F32, st.PATH_GATHER, STEPS, 1.0)
    for lo in WINDOWS:
        want = oracle.window(grid0, ce, r, st.BOX, st.BC_PERIODIC, STEPS, lo, (16, 16))
        got = res[lo[0]:lo[0] + 16, lo[1]:lo[1] + 16].cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= tol, (lo, np.abs(got - want).max(), tol)
    plan.close()
