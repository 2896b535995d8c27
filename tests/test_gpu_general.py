"""GPU parity of GENERAL stencils: the 2D outer-product path covers the
nonzero weights with a minimum set of axis-parallel lines (Section 3.5) --
lines along i and along j mixed -- and must match the oracle (which sums all
(2r+1)^2 taps) on sparse irregular patterns, bit for bit on integers."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, torch_cuda

pytestmark = pytest.mark.gpu


def patterns(r):
    w = 2 * r + 1
    z = np.zeros((w, w), dtype=bool)
    out = {}
    m = z.copy(); m[r, :] = True; m[:, r] = True; m[0, 0] = True; out["cross_plus_corner"] = m
    m = z.copy(); m[0, :] = True; out["one_row_off_centre"] = m
    m = z.copy(); m[:, w - 1] = True; out["one_column_edge"] = m
    m = z.copy(); m[w - 1, :] = True; m[:, 0] = True; out["l_shape"] = m
    m = z.copy(); np.fill_diagonal(m, True); out["diagonal"] = m
    m = z.copy(); m[::2, ::2] = True; out["checker"] = m
    m = z.copy(); m[1, 2 * r - 1] = True; out["single"] = m
    rng = np.random.default_rng(77 + r)
    out["random_sparse"] = rng.random((w, w)) < 0.25
    out["full"] = ~z
    out["empty"] = z
    return out


def _coeffs(mask, seed, integer=False):
    rng = np.random.default_rng(seed)
    if integer:
        v = rng.integers(-2, 3, size=mask.shape).astype(np.float64)
        v[v == 0] = 1.0
    else:
        v = rng.uniform(0.05, 1.0, size=mask.shape)
        v = v / max(1e-30, float((v * mask).sum()))
    return np.where(mask, v, 0.0)


# FP32 n = 4 blocks on direct-to-LDS windows (column extent a multiple of 4),
# the 16x16 fallback on ragged extents, FP64 16x16
@pytest.mark.parametrize("dims", [(150, 203), (100, 260)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype,block_n", [(st.F32, 0), (st.F32, 16), (st.F64, 0)])
@pytest.mark.parametrize("bc", [st.BC_ZERO, st.BC_PERIODIC])
def test_general_cover_parity(dims, r, dtype, block_n, bc):
    torch = torch_cuda()
    a0 = inputs.grid(dims, seed=1500 + r, dtype=np.float32 if dtype == st.F32 else np.float64)
    for name, mask in patterns(r).items():
        c = _coeffs(mask, 1600 + r)
        plan = st.Plan(dims, r, st.GENERAL, c, boundary=bc, dtype=dtype, path=st.PATH_MFMA, block_n=block_n)
        rows, cols = st.line_cover(c, r)
        assert plan.info["mfma_lines"] <= max(len(rows) + len(cols), int(mask.any(axis=0).sum()))
        x = torch.from_numpy(a0).cuda()
        got = plan.run_steps(x, torch.empty_like(x), 2).cpu().numpy().astype(np.float64)
        ce = eff_coeffs(c, dtype)
        want = oracle.run(a0, ce, r, st.BOX, bc, 2)
        tol = error_bound(ce, 2, r, st.BOX, dtype, st.PATH_MFMA, 2, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol, (name, np.abs(got - want).max(), tol)
        plan.close()


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dims", [(96, 70), (64, 132)])
def test_general_cover_integer_bit_exact(r, dims):
    torch = torch_cuda()
    a0 = inputs.int_grid(dims, seed=1700 + r)
    for name, mask in patterns(r).items():
        c = _coeffs(mask, 1800 + r, integer=True)
        s = float(np.abs(c).sum())
        steps = 2 if 8 * s * s < 2.0 ** 24 else 1
        for bc in (st.BC_ZERO, st.BC_PERIODIC):
            plan = st.Plan(a0.shape, r, st.GENERAL, c, boundary=bc, dtype=st.F32, path=st.PATH_MFMA)
            x = torch.from_numpy(a0).cuda()
            got = plan.run_steps(x, torch.empty_like(x), steps).cpu().numpy().astype(np.float64)
            assert np.array_equal(got, oracle.run(a0, c, r, st.BOX, bc, steps)), (name, bc)
            plan.close()


@pytest.mark.parametrize("r", [1, 3])
def test_general_pure_shift_every_offset(r):
    """A single weight 1 at C^g[a][b] shifts the grid by (a - r, b - r); the
    cover is one line, along i or along j (orientation of Eq. (12) and (14))."""
    torch = torch_cuda()
    a0 = inputs.grid((64, 80), seed=1900 + r)
    w = 2 * r + 1
    for a in range(w):
        for b in range(w):
            c = np.zeros((w, w))
            c[a, b] = 1.0
            plan = st.Plan(a0.shape, r, st.GENERAL, c, boundary=st.BC_PERIODIC, dtype=st.F32, path=st.PATH_MFMA)
            assert plan.info["mfma_lines"] == 1
            x = torch.from_numpy(a0).cuda()
            got = plan.run_steps(x, torch.empty_like(x), 1).cpu().numpy()
            assert np.array_equal(got, np.roll(a0, shift=(r - a, r - b), axis=(0, 1))), (a, b)
            plan.close()


# The gather path of GENERAL stencils walks the nonzero taps only (direct-to-
# LDS windows: column extent a multiple of 4 and wider than 64 FP32 columns;
# other extents take the tiled all-tap gather kernel).
@pytest.mark.parametrize("dims", [(150, 260), (37, 516), (100, 203), (48, 64)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", [st.F32, st.F64])
@pytest.mark.parametrize("bc", [st.BC_ZERO, st.BC_PERIODIC])
def test_general_sparse_gather_parity(dims, r, dtype, bc):
    torch = torch_cuda()
    a0 = inputs.grid(dims, seed=2000 + r, dtype=np.float32 if dtype == st.F32 else np.float64)
    for name, mask in patterns(r).items():
        c = _coeffs(mask, 2100 + r)
        plan = st.Plan(dims, r, st.GENERAL, c, boundary=bc, dtype=dtype, path=st.PATH_GATHER)
        assert plan.info["taps"] == int(mask.sum())
        x = torch.from_numpy(a0).cuda()
        got = plan.run_steps(x, torch.empty_like(x), 2).cpu().numpy().astype(np.float64)
        ce = eff_coeffs(c, dtype)
        want = oracle.run(a0, ce, r, st.BOX, bc, 2)
        tol = error_bound(ce, 2, r, st.BOX, dtype, st.PATH_GATHER, 2, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol, (name, np.abs(got - want).max(), tol)
        plan.close()


@pytest.mark.parametrize("r", [1, 4])
def test_general_sparse_gather_shift_and_integer(r):
    """Single weight 1 at C^g[a][b]: the nonzero-tap gather shifts the grid by
    (a - r, b - r) exactly; integer patterns match the oracle bit for bit."""
    torch = torch_cuda()
    a0 = inputs.grid((40, 264), seed=2200 + r)
    w = 2 * r + 1
    for a in range(w):
        for b in range(w):
            c = np.zeros((w, w))
            c[a, b] = 1.0
            plan = st.Plan(a0.shape, r, st.GENERAL, c, boundary=st.BC_PERIODIC, dtype=st.F32, path=st.PATH_GATHER)
            x = torch.from_numpy(a0).cuda()
            got = plan.run_steps(x, torch.empty_like(x), 1).cpu().numpy()
            assert np.array_equal(got, np.roll(a0, shift=(r - a, r - b), axis=(0, 1))), (a, b)
            plan.close()
    ai = inputs.int_grid((96, 260), seed=2300 + r)
    for name, mask in patterns(r).items():
        c = _coeffs(mask, 2400 + r, integer=True)
        s = float(np.abs(c).sum())
        steps = 2 if 8 * s * s < 2.0 ** 24 else 1
        for bc in (st.BC_ZERO, st.BC_PERIODIC):
            plan = st.Plan(ai.shape, r, st.GENERAL, c, boundary=bc, dtype=st.F32, path=st.PATH_GATHER)
            x = torch.from_numpy(ai).cuda()
            got = plan.run_steps(x, torch.empty_like(x), steps).cpu().numpy().astype(np.float64)
            assert np.array_equal(got, oracle.run(ai, c, r, st.BOX, bc, steps)), (name, bc)
            plan.close()
