"""GPU tests of the batched launch (many grids of uneven sizes per launch).

A grid advanced inside a batch runs the same kernel body, with the same
arithmetic, as the grid alone, so its result must be bitwise equal to the
plan's own run_steps; the single runs are themselves checked against the
CPU FP64 oracle elsewhere, and here once more for a few members."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, torch_cuda

pytestmark = pytest.mark.gpu

BF, FH = st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3

# (dims, r, shape, bc, dtype, path): DMA-eligible and ragged extents, 2D and 3D
MIXED = [
    ((64, 64), 1, st.BOX, st.BC_ZERO, st.F64, st.PATH_GATHER),
    ((100, 36), 2, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_MFMA),
    ((77, 45), 2, st.BOX, st.BC_ZERO, st.F32, st.PATH_MFMA),
    ((128, 128), 2, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_MFMA),
    ((300, 260), 4, st.BOX, st.BC_ZERO, st.F32, st.PATH_MFMA),
    ((90, 64), 3, st.STAR, st.BC_ZERO, st.F32, st.PATH_MFMA),
    ((64, 200), 1, st.BOX, st.BC_PERIODIC, st.F32, BF),
    ((33, 17), 2, st.BOX, st.BC_ZERO, st.F32, FH),
    ((48, 48), 4, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_GATHER),
    ((96, 96), 3, st.STAR, st.BC_ZERO, st.F64, st.PATH_MFMA),
    ((8, 8, 8), 1, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_GATHER),
    ((20, 33, 64), 2, st.STAR, st.BC_ZERO, st.F32, st.PATH_MFMA),
    ((17, 40, 70), 1, st.BOX, st.BC_ZERO, st.F64, st.PATH_MFMA),
    ((40, 24, 32), 4, st.STAR, st.BC_PERIODIC, st.F32, BF),
    ((16, 16, 16), 1, st.BOX, st.BC_ZERO, st.F32, FH),
    ((35, 30, 66), 3, st.STAR, st.BC_ZERO, st.F64, st.PATH_GATHER),
    ((64, 64, 64), 4, st.STAR, st.BC_ZERO, st.F32, st.PATH_GATHER),
    ((14, 30, 64), 3, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_AUTO),
    ((11, 19, 70), 4, st.BOX, st.BC_ZERO, st.F32, st.PATH_MFMA),
]


def _member(torch, spec, seed):
    dims, r, shape, bc, dt, path = spec
    c = inputs.coefficients(len(dims), r, shape, seed=seed, dtype=np.float64)
    ndt = np.float64 if dt == st.F64 else np.float32
    a0 = inputs.grid(dims, seed=seed + 1, dtype=ndt)
    plan = st.Plan(dims, r, shape, c, boundary=bc, dtype=dt, path=path)
    x = torch.from_numpy(a0).cuda()
    return plan, c, a0, x, torch.empty_like(x)


def _alone(torch, plan, a0, steps):
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), steps)
    torch.cuda.synchronize()
    return res.cpu().numpy()


@pytest.mark.parametrize("steps", [1, 2, 5])
def test_mixed_batch_equals_alone(steps):
    torch = torch_cuda()
    ms = [_member(torch, spec, 7000 + 10 * k) for k, spec in enumerate(MIXED)]
    batch = st.Batch([m[0] for m in ms], [m[3] for m in ms], [m[4] for m in ms])
    info = batch.info()
    assert 1 < info["groups"] <= len(MIXED)
    idx = batch.run_steps(steps)
    torch.cuda.synchronize()
    assert idx == steps % 2
    for k, (plan, c, a0, x, y) in enumerate(ms):
        got = (x if idx == 0 else y).cpu().numpy()
        want = _alone(torch, plan, a0, steps)
        assert np.array_equal(got, want), f"member {k} {MIXED[k]}"
    # a few members against the oracle as well
    for k in (1, 4, 10, 13, 17, 18):
        plan, c, a0, x, y = ms[k]
        dims, r, shape, bc, dt, path = MIXED[k]
        got = (x if idx == 0 else y).cpu().numpy().astype(np.float64)
        ce = eff_coeffs(c, dt)
        want = oracle.run(a0.astype(np.float64), ce, r, shape, bc, steps)
        tol = error_bound(ce, len(dims), r, shape, dt, path, steps, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol
    batch.close()


def test_many_small_grids_one_group():
    """The paper-scale case: many small FP64 grids of one stencil kind."""
    torch = torch_cuda()
    rng = np.random.default_rng(7100)
    specs = []
    for k in range(60):
        n0, n1 = (int(v) for v in rng.integers(24, 160, size=2))
        specs.append(((n0, n1), 2, st.BOX, st.BC_PERIODIC, st.F64, st.PATH_MFMA))
    ms = [_member(torch, spec, 7200 + 3 * k) for k, spec in enumerate(specs)]
    batch = st.Batch([m[0] for m in ms], [m[3] for m in ms], [m[4] for m in ms])
    assert batch.info()["groups"] == 1
    idx = batch.run_steps(3)
    torch.cuda.synchronize()
    for plan, c, a0, x, y in ms:
        assert np.array_equal((x if idx == 0 else y).cpu().numpy(), _alone(torch, plan, a0, 3))
    batch.close()


def test_repeated_runs_continue_the_trajectory():
    """Graph replays of one batch continue from the state they left."""
    torch = torch_cuda()
    ms = [_member(torch, spec, 7300 + 10 * k) for k, spec in enumerate(MIXED[:6])]
    batch = st.Batch([m[0] for m in ms], [m[3] for m in ms], [m[4] for m in ms])
    for _ in range(3):
        assert batch.run_steps(4) == 0
    torch.cuda.synchronize()
    for plan, c, a0, x, y in ms:
        assert np.array_equal(x.cpu().numpy(), _alone(torch, plan, a0, 12))
    batch.close()


def test_batch_rejects_overlapping_buffers():
    torch = torch_cuda()
    c = inputs.coefficients(2, 1, st.BOX, seed=1, dtype=np.float64)
    plan = st.Plan((32, 32), 1, st.BOX, c)
    big = torch.zeros(3 * 32 * 32, device="cuda")
    a = big[: 32 * 32].view(32, 32)
    b = big[32 * 32: 2 * 32 * 32].view(32, 32)
    with pytest.raises(st.StencilError) as e:
        st.Batch([plan, plan], [a, b], [b, a])
    assert e.value.status == st.EALIAS


def test_batch_general_nonzero_tap_gather():
    """GENERAL members (2D and 3D) on the nonzero-tap gather in one batch with a box member:
    each equals its own launch and the oracle."""
    torch = torch_cuda()
    d3 = np.zeros((9, 9, 9)); d3[np.arange(9), np.arange(9), np.arange(9)] = 0.1
    specs = [((130, 264), 4, np.float32, st.F32, np.eye(9)),
             ((70, 132), 2, np.float64, st.F64, np.eye(5)[::-1] * 0.3),
             ((96, 516), 3, np.float32, st.F32, None),
             ((14, 40, 64), 4, np.float32, st.F32, d3)]
    ms = []
    for k, (dims, r, ndt, dt, c) in enumerate(specs):
        shape = st.BOX if c is None else st.GENERAL
        if c is None:
            c = inputs.coefficients(len(dims), r, st.BOX, seed=7300, dtype=np.float64)
        a0 = inputs.grid(dims, seed=7310 + k, dtype=ndt)
        plan = st.Plan(dims, r, shape, c, boundary=st.BC_PERIODIC, dtype=dt, path=st.PATH_GATHER)
        x = torch.from_numpy(a0).cuda()
        ms.append((plan, c, a0, x, torch.empty_like(x), r, dt))
    batch = st.Batch([m[0] for m in ms], [m[3] for m in ms], [m[4] for m in ms])
    idx = batch.run_steps(3)
    torch.cuda.synchronize()
    for plan, c, a0, x, y, r, dt in ms:
        got = (x if idx == 0 else y).cpu().numpy()
        assert np.array_equal(got, _alone(torch, plan, a0, 3))
        ce = eff_coeffs(c, dt)
        want = oracle.run(a0.astype(np.float64), ce, r, st.BOX, st.BC_PERIODIC, 3)
        tol = error_bound(ce, a0.ndim, r, st.BOX, dt, st.PATH_GATHER, 3, np.abs(a0).max())
        assert np.abs(got.astype(np.float64) - want).max() <= tol
    batch.close()


# Plans the library time-blocks (AUTO on 2D grids wider than 64 columns with a
# column extent that is a multiple of 4, 3D order-1 grids of at most 64^3
# points or planes of many tiles), with plain ones beside them.
TB_MIXED = [
    ((200, 136), 1, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_AUTO),
    ((150, 260), 2, st.STAR, st.BC_ZERO, st.F32, st.PATH_AUTO),
    ((96, 132), 3, st.BOX, st.BC_ZERO, st.F32, st.PATH_AUTO),
    ((120, 200), 4, st.STAR, st.BC_PERIODIC, st.F32, st.PATH_AUTO),
    ((130, 136), 1, st.STAR, st.BC_ZERO, st.F64, st.PATH_AUTO),
    ((520, 1040), 1, st.BOX, st.BC_PERIODIC, st.F64, st.PATH_AUTO),
    ((100, 100), 2, st.BOX, st.BC_ZERO, st.F64, st.PATH_AUTO),
    ((16, 24, 32), 1, st.STAR, st.BC_ZERO, st.F32, st.PATH_AUTO),
    ((8, 256, 260), 1, st.STAR, st.BC_PERIODIC, st.F32, st.PATH_AUTO),
    ((20, 30, 64), 1, st.BOX, st.BC_ZERO, st.F64, st.PATH_AUTO),
    ((77, 45), 2, st.BOX, st.BC_ZERO, st.F32, st.PATH_MFMA),
    ((64, 64), 1, st.BOX, st.BC_ZERO, st.F64, st.PATH_GATHER),
    ((90, 62), 2, st.STAR, st.BC_PERIODIC, st.F32, st.PATH_AUTO),
]


@pytest.mark.parametrize("steps", [1, 2, 3, 7, 10, 17])
def test_time_blocked_batch_equals_alone(steps):
    """Grids whose plans the library time-blocked advance up to T steps per
    batched launch (a schedule whose launch count has the parity of the step
    count); every grid ends in buffer steps % 2, bit for bit equal to its
    plan's own run_steps, and within the oracle's bound."""
    torch = torch_cuda()
    ms = [_member(torch, spec, 7500 + 10 * k) for k, spec in enumerate(TB_MIXED)]
    assert sum(m[0].info["time_block"] > 1 for m in ms) >= 9
    batch = st.Batch([m[0] for m in ms], [m[3] for m in ms], [m[4] for m in ms])
    idx = batch.run_steps(steps)
    torch.cuda.synchronize()
    assert idx == steps % 2
    for k, (plan, c, a0, x, y) in enumerate(ms):
        got = (x if idx == 0 else y).cpu().numpy()
        assert np.array_equal(got, _alone(torch, plan, a0, steps)), f"member {k} {TB_MIXED[k]}"
    for k in (0, 5, 8):
        plan, c, a0, x, y = ms[k]
        dims, r, shape, bc, dt, path = TB_MIXED[k]
        got = (x if idx == 0 else y).cpu().numpy().astype(np.float64)
        ce = eff_coeffs(c, dt)
        want = oracle.run(a0.astype(np.float64), ce, r, shape, bc, steps)
        tol = error_bound(ce, len(dims), r, shape, dt, st.PATH_GATHER, steps, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol
    batch.close()


def test_time_blocked_batch_repeated_runs():
    """Graph replays of a batch with time-blocked classes continue the
    trajectory: three runs of 6 steps (T = 8: two launches of 3; T = 2: four
    launches, 2 + 2 + 1 + 1) equal one of 18."""
    torch = torch_cuda()
    ms = [_member(torch, spec, 7600 + 10 * k) for k, spec in enumerate(TB_MIXED[:7])]
    batch = st.Batch([m[0] for m in ms], [m[3] for m in ms], [m[4] for m in ms])
    for _ in range(3):
        assert batch.run_steps(6) == 0
    torch.cuda.synchronize()
    for plan, c, a0, x, y in ms:
        assert np.array_equal(x.cpu().numpy(), _alone(torch, plan, a0, 18))
    batch.close()
