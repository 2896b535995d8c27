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


# ---------------------------------------------------------------- 3D, 512^3
DIMS3 = (512, 512, 512)
STEPS3 = 3
WINDOWS3 = [(0, 0, 0), (0, 504, 0), (504, 0, 504), (504, 504, 504), (250, 17, 300), (33, 260, 8)]


@pytest.fixture(scope="module")
def grid3():
    return inputs.grid(DIMS3, seed=301, dtype=np.float64)


@pytest.mark.parametrize("dtype", [st.F32, st.F64])
@pytest.mark.parametrize("shape,r", [(st.STAR, 1), (st.STAR, 2), (st.STAR, 3), (st.STAR, 4), (st.BOX, 1),
                                     (st.BOX, 3), (st.BOX, 4)])
@pytest.mark.parametrize("path", [st.PATH_AUTO, st.PATH_GATHER, st.PATH_MFMA])
def test_fullsize_3d_windows(grid3, dtype, shape, r, path):
    """512^3, zero halo, the configuration of the 3D benchmark (stars r = 1..4,
    the 27-point box) and the serving mix's large boxes, on sampled 8^3
    windows including corners and faces."""
    if dtype == st.F64 and shape == st.BOX and r > 2 and path == st.PATH_MFMA:
        pytest.skip("FP64 3D boxes beyond r = 2 have no outer-product kernel (AUTO takes the gather)")
    torch = torch_cuda()
    c = inputs.coefficients(3, r, shape, seed=3100 + 10 * shape + r, dtype=np.float64)
    ce = eff_coeffs(c, dtype)
    a0 = grid3 if dtype == st.F64 else grid3.astype(np.float32)
    plan = st.Plan(DIMS3, r, shape, c, boundary=st.BC_ZERO, dtype=dtype, path=path)
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), STEPS3)
    torch.cuda.synchronize()
    tol = error_bound(ce, 3, r, shape, dtype, plan.info["path"], STEPS3, 1.0)
    for lo in WINDOWS3:
        want = oracle.window(a0, ce, r, shape, st.BC_ZERO, STEPS3, lo, (8, 8, 8))
        got = res[lo[0]:lo[0] + 8, lo[1]:lo[1] + 8, lo[2]:lo[2] + 8].cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= tol, (lo, np.abs(got - want).max(), tol)
    plan.close()
    del x, res
    torch.cuda.empty_cache()


@pytest.mark.parametrize("path", [st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3])
@pytest.mark.parametrize("r", [2, 3, 4])
def test_fullsize_3d_split_box(grid3, path, r):
    """FP32 3D boxes of order 2-4 on the split-precision outer products
    (band fragments from the LDS table) at 512^3, zero halo, on the sampled
    8^3 windows against the FP64 oracle with the split bound."""
    torch = torch_cuda()
    c = inputs.coefficients(3, r, st.BOX, seed=3100 + 10 * st.BOX + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = grid3.astype(np.float32)
    plan = st.Plan(DIMS3, r, st.BOX, c, boundary=st.BC_ZERO, dtype=st.F32, path=path)
    assert plan.info["path"] == path and plan.info["mfma_lines"] == (2 * r + 1) ** 2
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), STEPS3)
    torch.cuda.synchronize()
    tol = error_bound(ce, 3, r, st.BOX, st.F32, path, STEPS3, 1.0)
    for lo in WINDOWS3:
        want = oracle.window(a0, ce, r, st.BOX, st.BC_ZERO, STEPS3, lo, (8, 8, 8))
        got = res[lo[0]:lo[0] + 8, lo[1]:lo[1] + 8, lo[2]:lo[2] + 8].cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= tol, (lo, np.abs(got - want).max(), tol)
    plan.close()
    del x, res
    torch.cuda.empty_cache()


@pytest.mark.parametrize("path,tb", [(st.PATH_AUTO, 0), (st.PATH_GATHER, 0), (st.PATH_MFMA, 0),
                                     (st.PATH_GATHER, 5), (st.PATH_GATHER, 8)])
def test_fullsize_512_fp64_star(path, tb):
    """The 512^2 FP64 five-point star (centre 0.5, neighbours 0.125, zero halo,
    10 steps) on every path the latency benchmark times, against the oracle
    on the whole grid."""
    torch = torch_cuda()
    c = np.zeros((3, 3))
    c[1, 1] = 0.5
    c[0, 1] = c[2, 1] = c[1, 0] = c[1, 2] = 0.125
    a0 = inputs.grid((512, 512), seed=101, dtype=np.float64)
    plan = st.Plan((512, 512), 1, st.STAR, c, boundary=st.BC_ZERO, dtype=st.F64, path=path, time_block=tb)
    x = torch.from_numpy(a0).cuda()
    got = plan.run_steps(x, torch.empty_like(x), 10).cpu().numpy()
    want = oracle.run(a0, c, 1, st.STAR, st.BC_ZERO, 10)
    tol = error_bound(c, 2, 1, st.STAR, st.F64, st.PATH_GATHER, 10, 1.0)
    assert np.abs(got - want).max() <= tol
    plan.close()


# ------------------------------------------------- mixed precision, full size
# The split-precision configurations at their benchmark shapes (zero halo):
# 2D box r = 2 at 4096^2 and 3D star r = 4 at 384^3, BF16 and FP16 hi/lo
# operands with FP32 accumulation, on sampled light-cone windows (corners,
# faces, interior) against the FP64 oracle with the split bound.
@pytest.mark.parametrize("path", [st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3])
def test_fullsize_mixed_2d_4096(path):
    torch = torch_cuda()
    dims, r, steps = (4096, 4096), 2, 4
    c = inputs.coefficients(2, r, st.BOX, seed=4100, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = inputs.grid(dims, seed=401)
    plan = st.Plan(dims, r, st.BOX, c, boundary=st.BC_ZERO, dtype=st.F32, path=path)
    assert plan.info["path"] == path
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), steps)
    torch.cuda.synchronize()
    tol = error_bound(ce, 2, r, st.BOX, st.F32, path, steps, 1.0)
    for lo in [(0, 0), (0, 4080), (4080, 0), (4080, 4080), (0, 2000), (2048, 4080), (1999, 3001)]:
        want = oracle.window(a0, ce, r, st.BOX, st.BC_ZERO, steps, lo, (16, 16))
        got = res[lo[0]:lo[0] + 16, lo[1]:lo[1] + 16].cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= tol, (lo, np.abs(got - want).max(), tol)
    plan.close()


@pytest.mark.parametrize("path", [st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3])
def test_fullsize_mixed_3d_384(path):
    torch = torch_cuda()
    dims, r, steps = (384, 384, 384), 4, 3
    c = inputs.coefficients(3, r, st.STAR, seed=4200, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = inputs.grid(dims, seed=402)
    plan = st.Plan(dims, r, st.STAR, c, boundary=st.BC_ZERO, dtype=st.F32, path=path)
    assert plan.info["path"] == path
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), steps)
    torch.cuda.synchronize()
    tol = error_bound(ce, 3, r, st.STAR, st.F32, path, steps, 1.0)
    for lo in [(0, 0, 0), (376, 376, 376), (0, 376, 0), (376, 0, 376), (190, 0, 100), (0, 190, 190),
               (200, 150, 376), (123, 231, 77)]:
        want = oracle.window(a0, ce, r, st.STAR, st.BC_ZERO, steps, lo, (8, 8, 8))
        got = res[lo[0]:lo[0] + 8, lo[1]:lo[1] + 8, lo[2]:lo[2] + 8].cpu().numpy().astype(np.float64)
        assert np.abs(got - want).max() <= tol, (lo, np.abs(got - want).max(), tol)
    plan.close()
    del x, res
    torch.cuda.empty_cache()
