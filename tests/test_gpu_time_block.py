"""GPU parity of time-blocked plans (T Jacobi steps per launch on overlapped
tiles in LDS) against the CPU FP64 oracle: every radius, both shapes, both
boundaries and dtypes, time blocks from 2 to the largest built, step counts
that leave a partial last launch, ragged and tiny extents, integer data
bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, torch_cuda

pytestmark = pytest.mark.gpu

TMAX = {(st.F32, 1): 12, (st.F32, 2): 6, (st.F32, 3): 4, (st.F32, 4): 3,
        (st.F64, 1): 8, (st.F64, 2): 4, (st.F64, 3): 2, (st.F64, 4): 2}


def _run(a0, c, r, shape, bc, dtype, tb, steps):
    torch = torch_cuda()
    plan = st.Plan(a0.shape, r, shape, c, boundary=bc, dtype=dtype, time_block=tb)
    assert plan.info["time_block"] == max(tb, 1)
    x = torch.from_numpy(a0).cuda()
    y = torch.empty_like(x)
    res = plan.run_steps(x, y, steps)
    torch.cuda.synchronize()
    launches = -(-steps // max(tb, 1))
    assert (res is x) == (launches % 2 == 0)
    out = res.cpu().numpy().astype(np.float64)
    plan.close()
    return out


def _case(dims, r, shape, bc, dtype, tb, steps, seed):
    c = inputs.coefficients(2, r, shape, seed=seed, dtype=np.float64)
    ce = eff_coeffs(c, dtype)
    a0 = inputs.grid(dims, seed=seed + 1, dtype=np.float32 if dtype == st.F32 else np.float64)
    want = oracle.run(a0, ce, r, shape, bc, steps)
    got = _run(a0, c, r, shape, bc, dtype, tb, steps)
    tol = error_bound(ce, 2, r, shape, dtype, st.PATH_GATHER, steps, np.abs(a0).max())
    err = np.abs(got - want).max()
    assert err <= tol, f"max err {err:.3e} > bound {tol:.3e}"


@pytest.mark.parametrize("dtype", [st.F32, st.F64])
@pytest.mark.parametrize("shape", [st.BOX, st.STAR])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", [st.BC_ZERO, st.BC_PERIODIC])
@pytest.mark.parametrize("dims", [(100, 77), (96, 132)])
def test_time_block_parity(dtype, shape, r, bc, dims):
    tmax = TMAX[(dtype, r)]
    for tb in sorted({2, tmax}):
        _case(dims, r, shape, bc, dtype, tb, 2 * tb + 1, seed=1000 + 10 * r + bc)


@pytest.mark.parametrize("dtype", [st.F32, st.F64])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [st.BOX, st.STAR])
def test_time_block_every_step_count(dtype, r, shape):
    """Grids whose column extent takes direct-to-LDS windows run one kernel
    per step count: every time block from 2 to the largest, in runs whose
    last launch fuses T - 1 steps (2T - 1 steps) or one step (T + 1; the
    one-step gather)."""
    for tb in range(2, TMAX[(dtype, r)] + 1):
        for bc in (st.BC_ZERO, st.BC_PERIODIC):
            for steps in (2 * tb - 1, tb + 1):
                _case((70, 132), r, shape, bc, dtype, tb, steps, seed=1050 + 10 * r + tb)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [st.BOX, st.STAR])
@pytest.mark.parametrize("dims", [(70, 132), (520, 1040)])
def test_time_block_f64_tile_rows(r, shape, dims):
    """FP64 direct-to-LDS time blocks on 16-row tiles (grids of fewer 32 x 64
    tiles than CUs: 70 x 132) and 32-row tiles (520 x 1040, 289 tiles): the
    largest time block, bit for bit against one step per launch and within
    the oracle's bound, on a run ending in a one-step launch."""
    tb = TMAX[(st.F64, r)]
    c = inputs.coefficients(2, r, shape, seed=1150 + r, dtype=np.float64)
    a0 = inputs.grid(dims, seed=1151, dtype=np.float64)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        got = _run(a0, c, r, shape, bc, st.F64, tb, tb + 1)
        assert np.array_equal(got, _run(a0, c, r, shape, bc, st.F64, 1, tb + 1))
        want = oracle.run(a0, c, r, shape, bc, tb + 1)
        tol = error_bound(c, 2, r, shape, st.F64, st.PATH_GATHER, tb + 1, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol


@pytest.mark.parametrize("dims", [(1, 1), (5, 3), (3, 70), (70, 2), (9, 9), (1, 4), (5, 8), (70, 4), (3, 68)])
@pytest.mark.parametrize("r", [1, 3])
def test_time_block_small_extents(dims, r):
    """Windows much larger than the grid: periodic wraps many times, zero
    halo keeps re-zeroing almost the whole window."""
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        for dtype in (st.F32, st.F64):
            _case(dims, r, st.BOX, bc, dtype, TMAX[(dtype, r)], 5, seed=1100 + r)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", [st.F32, st.F64])
def test_time_block_integer_bit_exact(r, dtype):
    c = inputs.int_coefficients(2, r, st.BOX, seed=1200 + r)
    s = float(np.abs(c).sum())
    tb = TMAX[(dtype, r)]
    limit = 2.0 ** 24 if dtype == st.F32 else 2.0 ** 53
    steps = 1
    while steps < tb + 1 and 8 * s ** (steps + 1) < limit:
        steps += 1
    a0 = inputs.int_grid((70, 132), seed=1210 + r, dtype=np.float32 if dtype == st.F32 else np.float64)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        want = oracle.run(a0, c, r, st.BOX, bc, steps)
        got = _run(a0, c, r, st.BOX, bc, dtype, tb, steps)
        assert np.array_equal(got, want)


def test_time_block_apply_is_one_step():
    torch = torch_cuda()
    c = inputs.coefficients(2, 2, st.BOX, seed=1300, dtype=np.float64)
    a0 = inputs.grid((64, 64), seed=1301)
    plan = st.Plan((64, 64), 2, st.BOX, c, time_block=4)
    x = torch.from_numpy(a0).cuda()
    y = torch.empty_like(x)
    plan.apply(x, y)
    torch.cuda.synchronize()
    want = oracle.run(a0, eff_coeffs(c, st.F32), 2, st.BOX, st.BC_ZERO, 1)
    tol = error_bound(eff_coeffs(c, st.F32), 2, 2, st.BOX, st.F32, st.PATH_GATHER, 1, 1.0)
    assert np.abs(y.cpu().numpy().astype(np.float64) - want).max() <= tol


def test_batch_rejects_time_blocked_plan():
    torch = torch_cuda()
    c = inputs.coefficients(2, 1, st.BOX, seed=1400, dtype=np.float64)
    plan = st.Plan((32, 32), 1, st.BOX, c, time_block=2)
    x, y = torch.zeros(32, 32, device="cuda"), torch.zeros(32, 32, device="cuda")
    with pytest.raises(st.StencilError) as e:
        st.Batch([plan], [x], [y])
    assert e.value.status == st.EUNSUPPORTED


# ------------------------------------------------------------------- 3D
def _run3(a0, c, shape, bc, dtype, tb, steps, r=1):
    torch = torch_cuda()
    plan = st.Plan(a0.shape, r, shape, c, boundary=bc, dtype=dtype, path=st.PATH_GATHER, time_block=tb)
    assert plan.info["time_block"] == max(tb, 1)
    x = torch.from_numpy(a0).cuda()
    y = torch.empty_like(x)
    res = plan.run_steps(x, y, steps)
    torch.cuda.synchronize()
    launches = -(-steps // max(tb, 1))
    assert (res is x) == (launches % 2 == 0)
    out = res.cpu().numpy()
    plan.close()
    return out


TB3 = [(st.F32, st.STAR, 1), (st.F32, st.BOX, 1), (st.F32, st.STAR, 2), (st.F32, st.STAR, 3), (st.F32, st.STAR, 4),
       (st.F64, st.STAR, 1), (st.F64, st.BOX, 1)]


@pytest.mark.parametrize("dtype,shape,r", TB3)
@pytest.mark.parametrize("bc", [st.BC_ZERO, st.BC_PERIODIC])
@pytest.mark.parametrize("dims", [(19, 35, 68), (8, 16, 64), (5, 3, 4), (1, 1, 4), (33, 17, 132), (9, 40, 32),
                                  (70, 66, 136), (9, 256, 260), (40, 130, 512)])
def test_time_block_3d_parity(dtype, shape, r, bc, dims):
    """3D time blocks (two steps per launch; streaming plane rings on planes
    of 32 or more (j, k) tiles -- the last two extents here -- and for FP32
    stars of order 2 to 4 (8-column window margins beyond order 2), whole
    windows otherwise): against the oracle, and bit for bit
    against one step per launch (the same per-point tap order), on runs with
    a last launch of two steps and of one, over several tiles and chunks with
    ragged tails."""
    c = inputs.coefficients(3, r, shape, seed=1500 + len(dims) + r, dtype=np.float64)
    ce = eff_coeffs(c, dtype)
    a0 = inputs.grid(dims, seed=1501, dtype=np.float32 if dtype == st.F32 else np.float64)
    for steps in (2, 5):
        got = _run3(a0, c, shape, bc, dtype, 2, steps, r)
        assert np.array_equal(got, _run3(a0, c, shape, bc, dtype, 1, steps, r))
        want = oracle.run(a0, ce, r, shape, bc, steps)
        tol = error_bound(ce, 3, r, shape, dtype, st.PATH_GATHER, steps, np.abs(a0).max())
        err = np.abs(got.astype(np.float64) - want).max()
        assert err <= tol, f"max err {err:.3e} > bound {tol:.3e}"


@pytest.mark.parametrize("dtype,shape,r", TB3)
def test_time_block_3d_integer_bit_exact(dtype, shape, r):
    c = inputs.int_coefficients(3, r, shape, seed=1600 + r)
    a0 = inputs.int_grid((21, 37, 72), seed=1601, dtype=np.float32 if dtype == st.F32 else np.float64)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        assert np.array_equal(_run3(a0, c, shape, bc, dtype, 2, 4, r).astype(np.float64),
                              oracle.run(a0, c, r, shape, bc, 4))


@pytest.mark.parametrize("shape,r", [(st.STAR, 1), (st.STAR, 2), (st.BOX, 1)])
@pytest.mark.parametrize("dims", [(64, 384, 384), (48, 320, 324)])
def test_time_block_3d_stream_two_per_cu(shape, r, dims):
    """FP32 streaming plans whose workgroups hold one level-1 block per thread
    and run at most two per CU, on planes of 72 / 60 (j, k) tiles where the
    launch re-cuts the chunks: bit for bit against one step per launch and
    within the oracle's bound, on runs ending in a two-step and a one-step
    launch."""
    c = inputs.coefficients(3, r, shape, seed=2700 + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = inputs.grid(dims, seed=2701, dtype=np.float32)
    for steps in (4, 3):
        got = _run3(a0, c, shape, st.BC_ZERO, st.F32, 2, steps, r)
        assert np.array_equal(got, _run3(a0, c, shape, st.BC_ZERO, st.F32, 1, steps, r))
        want = oracle.run(a0, ce, r, shape, st.BC_ZERO, steps)
        tol = error_bound(ce, 3, r, shape, st.F32, st.PATH_GATHER, steps, np.abs(a0).max())
        err = np.abs(got.astype(np.float64) - want).max()
        assert err <= tol, f"max err {err:.3e} > bound {tol:.3e}"


def _run_mfma(a0, c, bc, tb, steps, r):
    torch = torch_cuda()
    plan = st.Plan(a0.shape, r, st.BOX, c, boundary=bc, dtype=st.F32, path=st.PATH_MFMA, time_block=tb)
    assert plan.info["time_block"] == max(tb, 1) and plan.info["path"] == st.PATH_MFMA
    x = torch.from_numpy(a0).cuda()
    y = torch.empty_like(x)
    res = plan.run_steps(x, y, steps)
    torch.cuda.synchronize()
    out = res.cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", [st.BC_ZERO, st.BC_PERIODIC])
@pytest.mark.parametrize("dims", [(37, 20), (70, 252), (45, 500), (130, 744), (300, 1000), (1, 8), (5, 4)])
def test_mfma_time_block_2d(r, bc, dims):
    """Two steps per launch on the FP32 box outer products (n = 4 blocks):
    bit for bit against one step per launch on the same kernels, and within
    the oracle's bound, on runs ending in a two-step and a one-step launch;
    extents below, at and across the 248-column strips and the 16-row blocks,
    and degenerate ones."""
    c = inputs.coefficients(2, r, st.BOX, seed=2800 + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = inputs.grid(dims, seed=2801, dtype=np.float32)
    for steps in (2, 5):
        got = _run_mfma(a0, c, bc, 2, steps, r)
        assert np.array_equal(got, _run_mfma(a0, c, bc, 1, steps, r))
        want = oracle.run(a0, ce, r, st.BOX, bc, steps)
        tol = error_bound(ce, 2, r, st.BOX, st.F32, st.PATH_MFMA, steps, np.abs(a0).max())
        err = np.abs(got.astype(np.float64) - want).max()
        assert err <= tol, f"max err {err:.3e} > bound {tol:.3e}"


@pytest.mark.parametrize("r", [2, 4])
def test_mfma_time_block_2d_integer_bit_exact(r):
    c = inputs.int_coefficients(2, r, st.BOX, seed=2900 + r)
    a0 = inputs.int_grid((83, 520), seed=2901, dtype=np.float32)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        assert np.array_equal(_run_mfma(a0, c, bc, 2, 3, r).astype(np.float64), oracle.run(a0, c, r, st.BOX, bc, 3))


def test_mfma_time_block_2d_misaligned_buffer_rejected():
    torch = torch_cuda()
    c = inputs.coefficients(2, 2, st.BOX, seed=3000, dtype=np.float64)
    plan = st.Plan((16, 16), 2, st.BOX, c, path=st.PATH_MFMA, time_block=2)
    base = torch.zeros(16 * 16 + 1, device="cuda")
    x = base[1:].view(16, 16)  # 4-byte offset
    y = torch.zeros(16, 16, device="cuda")
    with pytest.raises(st.StencilError) as e:
        plan.run_steps(x, y, 2)
    assert e.value.status == st.EINVAL
    torch.cuda.synchronize()
    plan.close()


def test_time_block_3d_misaligned_buffer_rejected():
    torch = torch_cuda()
    c = inputs.coefficients(3, 1, st.STAR, seed=1700, dtype=np.float64)
    plan = st.Plan((8, 8, 8), 1, st.STAR, c, path=st.PATH_GATHER, time_block=2)
    base = torch.zeros(8 * 8 * 8 + 1, device="cuda")
    x = base[1:].view(8, 8, 8)  # 4-byte offset
    y = torch.zeros(8, 8, 8, device="cuda")
    with pytest.raises(st.StencilError) as e:
        plan.run_steps(x, y, 2)
    assert e.value.status == st.EINVAL
    torch.cuda.synchronize()
    plan.close()
