"""GPU tests of the autotuner: the winner is the fastest measured candidate,
the cache returns it again without measuring, and the tuned plan is correct."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,r,shape,dtype", [
    ((256, 320), 2, st.BOX, st.F32),
    ((128, 200), 3, st.STAR, st.F32),
    ((96, 96), 1, st.BOX, st.F64),
    ((40, 48, 64), 2, st.STAR, st.F32),
    ((24, 36, 40), 1, st.BOX, st.F64),
])
def test_autotune_picks_fastest_and_caches(tmp_path, dims, r, shape, dtype):
    torch = torch_cuda()
    c = inputs.coefficients(len(dims), r, shape, seed=9000 + r, dtype=np.float64)
    cache = str(tmp_path / "tune.txt")
    knobs, ms, rows = st.autotune(dims, r, shape, c, boundary=st.BC_ZERO, dtype=dtype, cache=cache)
    assert len(rows) >= 2
    assert all(row["status"] == st.OK and row["ms_per_step"] > 0 for row in rows)
    fastest = min(rows, key=lambda row: row["ms_per_step"])
    assert ms == fastest["ms_per_step"]
    assert knobs == {k: fastest[k] for k in ("path", "lines", "block_n", "chunk", "time_block", "reg_rows",
                                             "tile_width")}
    assert knobs["path"] in (st.PATH_GATHER, st.PATH_MFMA)  # no split paths unless allowed
    again, ms2, rows2 = st.autotune(dims, r, shape, c, boundary=st.BC_ZERO, dtype=dtype, cache=cache)
    assert again == knobs and rows2 == [] and abs(ms2 - ms) < 1e-6
    # the tuned plan is correct
    ndt = np.float64 if dtype == st.F64 else np.float32
    a0 = inputs.grid(dims, seed=9100 + r, dtype=ndt)
    plan = st.Plan(dims, r, shape, c, boundary=st.BC_ZERO, dtype=dtype, **knobs)
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), 3)
    torch.cuda.synchronize()
    ce = eff_coeffs(c, dtype)
    want = oracle.run(a0.astype(np.float64), ce, r, shape, st.BC_ZERO, 3)
    tol = error_bound(ce, len(dims), r, shape, dtype, knobs["path"], 3, np.abs(a0).max())
    assert np.abs(res.cpu().numpy().astype(np.float64) - want).max() <= tol


def test_autotune_split_only_when_allowed():
    torch_cuda()
    c = inputs.coefficients(2, 2, st.BOX, seed=9200, dtype=np.float64)
    knobs, ms, rows = st.autotune((128, 256), 2, st.BOX, c, allow_split=True, force=True)
    paths = {row["path"] for row in rows}
    assert {st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3} <= paths
    knobs, ms, rows = st.autotune((128, 256), 2, st.BOX, c, path=st.PATH_GATHER)
    assert {row["path"] for row in rows} == {st.PATH_GATHER}


@pytest.mark.parametrize("chunk", [16, 48, 200])
def test_chunk_knob_keeps_results(chunk):
    """Every chunk length gives the same (bitwise) result as the default."""
    torch = torch_cuda()
    for dims, r, shape, path in (((300, 260), 2, st.BOX, st.PATH_MFMA), ((70, 45, 68), 2, st.STAR, st.PATH_GATHER),
                                 ((300, 256), 1, st.BOX, st.PATH_MFMA_BF16X3)):
        c = inputs.coefficients(len(dims), r, shape, seed=9300 + r, dtype=np.float64)
        a0 = inputs.grid(dims, seed=9301, dtype=np.float32)
        outs = []
        for ch in (0, chunk):
            plan = st.Plan(dims, r, shape, c, path=path, chunk=ch)
            x = torch.from_numpy(a0).cuda()
            outs.append(plan.run_steps(x, torch.empty_like(x), 3).cpu().numpy())
        assert np.array_equal(outs[0], outs[1])


def test_autotune_tries_register_and_workgroup_tiles():
    """A 2D FP32 box whose winner is the n = 4 outer products: the tuner then
    measures the other register (rows per wave) x workgroup (columns) tiles."""
    torch_cuda()
    c = inputs.coefficients(2, 4, st.BOX, seed=9400, dtype=np.float64)
    knobs, ms, rows = st.autotune((512, 1024), 4, st.BOX, c, path=st.PATH_MFMA, block_n=4, force=True)
    tiles = {(row["reg_rows"], row["tile_width"]) for row in rows}
    assert {(8, 256), (32, 256), (8, 128), (16, 128), (32, 128)} <= tiles
    assert all(row["status"] == st.OK for row in rows)
