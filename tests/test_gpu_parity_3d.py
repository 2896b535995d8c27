"""GPU parity of the 3D paths against the CPU FP64 oracle (elementwise).

Extents span two 32 x 64 (j, k) workgroup tiles with ragged tails and two
chunks of planes along i (chunk boundaries exercise the warm-up of the
plane ring); edge cases: extents of 1 and below the stencil width, integer
data (bit-exact) and pure shifts along each axis (orientation)."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, run_gpu, torch_cuda

pytestmark = pytest.mark.gpu

BF, FH = st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3


def combos():
    out = []
    for r in (1, 2, 3, 4):
        for dt in (st.F32, st.F64):
            out.append((st.PATH_GATHER, dt, st.BOX, r))
            out.append((st.PATH_GATHER, dt, st.STAR, r))
            out.append((st.PATH_MFMA, dt, st.STAR, r))
            if r <= 2 or dt == st.F32:
                out.append((st.PATH_MFMA, dt, st.BOX, r))
        for p in (BF, FH):
            out.append((p, st.F32, st.STAR, r))
            out.append((p, st.F32, st.BOX, r))
    return out


COMBOS = combos()


def _case(dims, r, shape, bc, dtype, path, steps, seed):
    c = inputs.coefficients(3, r, shape, seed=seed, dtype=np.float64)
    ce = eff_coeffs(c, dtype)
    a0 = inputs.grid(dims, seed=seed + 1, dtype=np.float32 if dtype == st.F32 else np.float64)
    want = oracle.run(a0, ce, r, shape, bc, steps)
    got = run_gpu(a0, c, r, shape, bc, dtype, path, steps)
    tol = error_bound(ce, 3, r, shape, dtype, path, steps, np.abs(a0).max())
    err = np.abs(got - want).max()
    assert err <= tol, f"max err {err:.3e} > bound {tol:.3e}"


@pytest.mark.parametrize("path,dtype,shape,r", COMBOS)
@pytest.mark.parametrize("bc", [st.BC_ZERO, st.BC_PERIODIC])
def test_random_ragged(path, dtype, shape, r, bc):
    _case((37, 45, 77), r, shape, bc, dtype, path, 2, seed=100 + 10 * r + bc)


@pytest.mark.parametrize("path,dtype,shape,r", [c for c in COMBOS if c[3] in (1, 4) or c[2] == st.BOX])
@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 2, 5), (1, 40, 70), (20, 1, 1), (9, 33, 3)])
def test_small_extents(path, dtype, shape, r, dims):
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        _case(dims, r, shape, bc, dtype, path, 2, seed=200 + r)


@pytest.mark.parametrize("path,dtype,shape,r", COMBOS)
def test_integer_bit_exact(path, dtype, shape, r):
    c = inputs.int_coefficients(3, r, shape, seed=300 + r)
    s = float(np.abs(c).sum())
    limit = 6.0e4 if path in (BF, FH) else 2.0 ** 24
    steps = 2 if 8 * s * s < limit else 1
    a0 = inputs.int_grid((18, 40, 70), seed=310 + r, dtype=np.float32 if dtype == st.F32 else np.float64)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        want = oracle.run(a0, c, r, shape, bc, steps)
        got = run_gpu(a0, c, r, shape, bc, dtype, path, steps)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("path,dtype,shape,r", [c for c in COMBOS if c[3] in (1, 2)])
@pytest.mark.parametrize("offset", [(1, 0, 0), (0, -1, 0), (0, 0, 1), (-1, 0, 0), (1, 1, -1)])
def test_pure_shift_orientation(path, dtype, shape, r, offset):
    if shape == st.STAR and sum(1 for v in offset if v) > 1:
        pytest.skip("off-axis offset is not a star tap")
    c = inputs.shift_coefficients(3, r, offset)
    if path in (BF, FH):
        a0 = inputs.int_grid((19, 35, 66), seed=400, lo=-30000, hi=30000)
    else:
        a0 = inputs.grid((19, 35, 66), seed=400, dtype=np.float32 if dtype == st.F32 else np.float64)
    got = run_gpu(a0, c, r, shape, st.BC_PERIODIC, dtype, path, 1)
    want = np.roll(a0.astype(np.float64), shift=tuple(-o for o in offset), axis=(0, 1, 2))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape,r", [(st.BOX, 3), (st.STAR, 2), (st.BOX, 1)])
def test_auto_path(shape, r):
    c = inputs.coefficients(3, r, shape, seed=500, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = inputs.grid((30, 33, 65), seed=501)
    got = run_gpu(a0, c, r, shape, st.BC_ZERO, st.F32, st.PATH_AUTO, 2)
    want = oracle.run(a0, ce, r, shape, st.BC_ZERO, 2)
    assert np.abs(got - want).max() <= error_bound(ce, 3, r, shape, st.F32, st.PATH_MFMA, 2, 1.0)


@pytest.mark.parametrize("path,dtype,shape,r", COMBOS)
@pytest.mark.parametrize("dims", [(21, 45, 132), (9, 40, 64), (5, 3, 4), (34, 1, 8), (7, 20, 66)])
def test_dma_plane_extents(path, dtype, shape, r, dims):
    """k extents that are multiples of the 16-byte vector take the
    direct-to-LDS plane windows (double-buffered across planes)."""
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        _case(dims, r, shape, bc, dtype, path, 2, seed=600 + r)


@pytest.mark.parametrize("path,dtype,shape,r", [c for c in COMBOS if c[3] in (1, 2)])
def test_dma_plane_integer_bit_exact(path, dtype, shape, r):
    c = inputs.int_coefficients(3, r, shape, seed=610 + r)
    s = float(np.abs(c).sum())
    limit = 6.0e4 if path in (BF, FH) else 2.0 ** 24
    steps = 2 if 8 * s * s < limit else 1
    a0 = inputs.int_grid((20, 37, 68), seed=620 + r, dtype=np.float32 if dtype == st.F32 else np.float64)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        assert np.array_equal(run_gpu(a0, c, r, shape, bc, dtype, path, steps),
                              oracle.run(a0, c, r, shape, bc, steps))


@pytest.mark.parametrize("shape,r", [(st.STAR, 1), (st.STAR, 2), (st.STAR, 3), (st.STAR, 4),
                                     (st.BOX, 1), (st.BOX, 2), (st.BOX, 3), (st.BOX, 4)])
@pytest.mark.parametrize("dims", [(37, 45, 77), (21, 45, 132)])
def test_mfma_fp32_block_edges(shape, r, dims):
    """FP32 outer products on n = 4 blocks (default) and on 16x16 blocks
    (block_n = 16), synchronous and direct-to-LDS staging (k extent 77 / 132)."""
    c = inputs.coefficients(3, r, shape, seed=700 + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    a0 = inputs.grid(dims, seed=701 + r)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        want = oracle.run(a0, ce, r, shape, bc, 3)
        tol = error_bound(ce, 3, r, shape, st.F32, st.PATH_MFMA, 3, np.abs(a0).max())
        for bn in ((0, 16) if shape == st.STAR or r <= 2 else (0,)):
            got = run_gpu(a0, c, r, shape, bc, st.F32, st.PATH_MFMA, 3, block_n=bn)
            assert np.abs(got - want).max() <= tol, (bn, bc, np.abs(got - want).max(), tol)


@pytest.mark.parametrize("r,dims", [(2, (11, 20, 68)), (2, (9, 13, 70)), (3, (12, 18, 64)), (4, (13, 21, 72))])
def test_mfma_box_pure_shift(r, dims):
    """FP32 3D box outer products (n = 4 blocks, band vectors from the LDS
    table) with a single weight 1 at C^g[a][b][c]: the result is the grid
    shifted by (a - r, b - r, c - r), bit for bit.  r = 2 visits every offset,
    r = 3 and 4 a seeded sample; k extents 68 / 64 / 72 use direct-to-LDS
    planes, 70 the synchronous staging."""
    torch = torch_cuda()
    a0 = inputs.grid(dims, seed=820 + r)
    w = 2 * r + 1
    offs = [(a, b, c) for a in range(w) for b in range(w) for c in range(w)]
    if r > 2:
        rng = np.random.default_rng(830 + r)
        offs = [offs[i] for i in rng.choice(len(offs), size=40, replace=False)]
    x = torch.from_numpy(a0).cuda()
    for a, b, c in offs:
        cg = np.zeros((w, w, w))
        cg[a, b, c] = 1.0
        plan = st.Plan(dims, r, st.BOX, cg, boundary=st.BC_PERIODIC, dtype=st.F32, path=st.PATH_MFMA)
        assert plan.info["block_n"] == 4
        got = plan.run_steps(x, torch.empty_like(x), 1).cpu().numpy()
        assert np.array_equal(got, np.roll(a0, shift=(r - a, r - b, r - c), axis=(0, 1, 2))), (a, b, c)
        plan.close()


@pytest.mark.parametrize("r", [3, 4])
@pytest.mark.parametrize("density", [0.1, 0.5])
def test_general_3d_auto(r, density):
    """Irregular 3D stencils under AUTO (outer products on n = 4 blocks from
    r = 3, all (2r+1)^2 lines; the nonzero-tap gather for at most 88 / 128
    nonzero taps at r = 3 / 4) against the oracle's full (2r+1)^3 sum."""
    torch = torch_cuda()
    rng = np.random.default_rng(840 + r + int(10 * density))
    w = 2 * r + 1
    mask = rng.random((w, w, w)) < density
    cg = np.where(mask, rng.uniform(-1.0, 1.0, size=mask.shape), 0.0)
    cg /= max(1e-30, float(np.abs(cg).sum()))
    a0 = inputs.grid((14, 22, 76), seed=850 + r)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        plan = st.Plan(a0.shape, r, st.GENERAL, cg, boundary=bc, dtype=st.F32)
        want_path = st.PATH_GATHER if int(mask.sum()) <= {3: 88, 4: 128}[r] else st.PATH_MFMA
        assert plan.info["path"] == want_path
        x = torch.from_numpy(a0).cuda()
        got = plan.run_steps(x, torch.empty_like(x), 2).cpu().numpy().astype(np.float64)
        ce = eff_coeffs(cg, st.F32)
        want = oracle.run(a0, ce, r, st.BOX, bc, 2)
        tol = error_bound(ce, 3, r, st.BOX, st.F32, want_path, 2, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol, (bc, np.abs(got - want).max(), tol)
        plan.close()


def _sparse3d_patterns(r, seed):
    w = 2 * r + 1
    rng = np.random.default_rng(seed)
    z = np.zeros((w, w, w), dtype=bool)
    pats = {}
    m = z.copy(); m[np.arange(w), np.arange(w), np.arange(w)] = True; pats["space_diagonal"] = m
    m = z.copy(); m[0, 2 * r, 1] = True; pats["single"] = m
    m = z.copy(); m[r] = np.eye(w, dtype=bool); m[:, r, r] = True; pats["plane_diagonal_plus_i_arm"] = m
    pats["random"] = rng.random((w, w, w)) < min(0.5, 40.0 / w ** 3)
    pats["empty"] = z
    return pats


# The gather path of 3D GENERAL stencils walks the nonzero taps (at most
# 128): direct-to-LDS windows when the k extent allows 16-byte lines, the
# staged windows otherwise (k = 70 FP32, 75 FP64).
@pytest.mark.parametrize("dims", [(13, 40, 64), (9, 35, 70), (6, 33, 75)])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dtype", [st.F32, st.F64])
def test_general_3d_nonzero_tap_gather(dims, r, dtype):
    torch = torch_cuda()
    ndt = np.float32 if dtype == st.F32 else np.float64
    a0 = inputs.grid(dims, seed=860 + r, dtype=ndt)
    for name, mask in _sparse3d_patterns(r, 870 + r).items():
        rng = np.random.default_rng(880 + r)
        cg = np.where(mask, rng.uniform(-1.0, 1.0, size=mask.shape), 0.0)
        cg /= max(1e-30, float(np.abs(cg).sum()))
        for bc in (st.BC_ZERO, st.BC_PERIODIC):
            plan = st.Plan(dims, r, st.GENERAL, cg, boundary=bc, dtype=dtype, path=st.PATH_GATHER)
            assert plan.info["taps"] == int(mask.sum())
            x = torch.from_numpy(a0).cuda()
            got = plan.run_steps(x, torch.empty_like(x), 2).cpu().numpy().astype(np.float64)
            ce = eff_coeffs(cg, dtype)
            want = oracle.run(a0.astype(np.float64), ce, r, st.BOX, bc, 2)
            tol = error_bound(ce, 3, r, st.BOX, dtype, st.PATH_GATHER, 2, np.abs(a0).max())
            assert np.abs(got - want).max() <= tol, (name, bc, np.abs(got - want).max(), tol)
            plan.close()


@pytest.mark.parametrize("r", [1, 4])
def test_general_3d_nonzero_tap_gather_shift(r):
    """One weight 1 at C^g[a][b][c]: the 3D nonzero-tap gather shifts the grid
    by (a - r, b - r, c - r) exactly, for every plane a."""
    torch = torch_cuda()
    a0 = inputs.grid((11, 36, 64), seed=890 + r)
    w = 2 * r + 1
    for a in range(w):
        for b, c in ((0, 0), (w - 1, 1), (r, r), (1, w - 1)):
            cg = np.zeros((w, w, w))
            cg[a, b, c] = 1.0
            plan = st.Plan(a0.shape, r, st.GENERAL, cg, boundary=st.BC_PERIODIC, dtype=st.F32, path=st.PATH_GATHER)
            x = torch.from_numpy(a0).cuda()
            got = plan.run_steps(x, torch.empty_like(x), 1).cpu().numpy()
            assert np.array_equal(got, np.roll(a0, shift=(r - a, r - b, r - c), axis=(0, 1, 2))), (a, b, c)
            plan.close()


def _mask_with_taps(r, n, seed):
    w = 2 * r + 1
    rng = np.random.default_rng(seed)
    flat = np.zeros(w ** 3, dtype=bool)
    flat[rng.choice(w ** 3, size=n, replace=False)] = True
    return flat.reshape(w, w, w)


# The nonzero-tap gather holds taps 0..63 in one lane register and 64..127 in
# a second: exactly 64, 65 and the maximum 128 taps, direct-to-LDS (k = 64)
# and staged (k = 70 / 75) windows, both boundaries, FP32 and FP64 (whose
# order >= 3 form accumulates into the ring directly).
@pytest.mark.parametrize("r", [3, 4])
@pytest.mark.parametrize("ntaps", [64, 65, 128])
@pytest.mark.parametrize("dtype,dims", [(st.F32, (10, 40, 64)), (st.F32, (9, 35, 70)),
                                        (st.F64, (10, 40, 64)), (st.F64, (6, 33, 75))])
def test_general_3d_nonzero_tap_counts(r, ntaps, dtype, dims):
    torch = torch_cuda()
    ndt = np.float32 if dtype == st.F32 else np.float64
    a0 = inputs.grid(dims, seed=900 + r, dtype=ndt)
    mask = _mask_with_taps(r, ntaps, 910 + r + ntaps)
    rng = np.random.default_rng(920 + r)
    cg = np.where(mask, rng.uniform(-1.0, 1.0, size=mask.shape), 0.0)
    cg /= float(np.abs(cg).sum())
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        plan = st.Plan(dims, r, st.GENERAL, cg, boundary=bc, dtype=dtype, path=st.PATH_GATHER)
        assert plan.info["taps"] == ntaps and plan.info["executed_flops_per_point"] == 2.0 * ntaps
        x = torch.from_numpy(a0).cuda()
        got = plan.run_steps(x, torch.empty_like(x), 2).cpu().numpy().astype(np.float64)
        ce = eff_coeffs(cg, dtype)
        want = oracle.run(a0.astype(np.float64), ce, r, st.BOX, bc, 2)
        tol = error_bound(ce, 3, r, st.BOX, dtype, st.PATH_GATHER, 2, np.abs(a0).max())
        assert np.abs(got - want).max() <= tol, (bc, np.abs(got - want).max(), tol)
        plan.close()


@pytest.mark.parametrize("r", [3, 4])
@pytest.mark.parametrize("dtype", [st.F32, st.F64])
def test_general_3d_nonzero_tap_max_integer_bit_exact(r, dtype):
    """128 nonzero integer taps (the table's limit): bit-exact against the oracle."""
    torch = torch_cuda()
    ndt = np.float32 if dtype == st.F32 else np.float64
    a0 = inputs.int_grid((8, 36, 64), seed=930 + r).astype(ndt)
    mask = _mask_with_taps(r, 128, 940 + r)
    rng = np.random.default_rng(950 + r)
    v = rng.integers(-2, 3, size=mask.shape).astype(np.float64)
    v[v == 0] = 1.0
    cg = np.where(mask, v, 0.0)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        plan = st.Plan(a0.shape, r, st.GENERAL, cg, boundary=bc, dtype=dtype, path=st.PATH_GATHER)
        assert plan.info["executed_flops_per_point"] == 256.0
        x = torch.from_numpy(a0).cuda()
        got = plan.run_steps(x, torch.empty_like(x), 1).cpu().numpy().astype(np.float64)
        assert np.array_equal(got, oracle.run(a0.astype(np.float64), cg, r, st.BOX, bc, 1)), bc
        plan.close()


# Split-precision stars in both covers: PARALLEL (AUTO: the line along k on
# MFMA, the j and i arms on vector FMAs) and HYBRID (the lines along j and k
# on MFMA, the i arm on vector FMAs; Table 2), against the oracle with the
# split bound, bit-exact on integers, synchronous and direct-to-LDS planes.
@pytest.mark.parametrize("path", [BF, FH])
@pytest.mark.parametrize("lines", [st.LINES_PARALLEL, st.LINES_HYBRID])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_split_star_line_options(path, lines, r):
    c = inputs.coefficients(3, r, st.STAR, seed=960 + r, dtype=np.float64)
    ce = eff_coeffs(c, st.F32)
    info = st.describe((37, 45, 77), r, st.STAR, c, path=path, lines=lines)
    assert info["lines"] == lines and info["mfma_lines"] == (2 if lines == st.LINES_HYBRID else 1)
    for dims in [(37, 45, 77), (21, 45, 132), (9, 33, 64)]:
        a0 = inputs.grid(dims, seed=970 + r)
        for bc in (st.BC_ZERO, st.BC_PERIODIC):
            want = oracle.run(a0, ce, r, st.STAR, bc, 2)
            got = run_gpu(a0, c, r, st.STAR, bc, st.F32, path, 2, lines=lines)
            tol = error_bound(ce, 3, r, st.STAR, st.F32, path, 2, np.abs(a0).max())
            assert np.abs(got - want).max() <= tol, (dims, bc, np.abs(got - want).max(), tol)
    ci = inputs.int_coefficients(3, r, st.STAR, seed=980 + r)
    ai = inputs.int_grid((20, 37, 68), seed=990 + r)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        assert np.array_equal(run_gpu(ai, ci, r, st.STAR, bc, st.F32, path, 1, lines=lines),
                              oracle.run(ai, ci, r, st.STAR, bc, 1))


@pytest.mark.parametrize("dtype,shape,r,path", [
    (st.F64, st.STAR, 1, st.PATH_GATHER), (st.F64, st.BOX, 1, st.PATH_GATHER), (st.F64, st.STAR, 4, st.PATH_MFMA),
    (st.F32, st.STAR, 2, st.PATH_GATHER), (st.F32, st.STAR, 3, st.PATH_GATHER), (st.F32, st.BOX, 1, st.PATH_GATHER)])
@pytest.mark.parametrize("dims", [(96, 320, 320), (40, 384, 388)])
def test_whole_number_items_per_cu(dtype, shape, r, path, dims):
    """Planes of 50 / 84 (j, k) tiles, where the library's chunks leave a
    fraction of a work item per CU and the launch re-cuts the planes to a
    whole number per CU: against the oracle, and bit for bit against a
    requested chunk (never re-cut; a point's taps are summed in the same order
    whatever the chunking)."""
    c = inputs.coefficients(3, r, shape, seed=2600 + r, dtype=np.float64)
    ce = eff_coeffs(c, dtype)
    a0 = inputs.grid(dims, seed=2601, dtype=np.float32 if dtype == st.F32 else np.float64)
    steps = 3
    got = run_gpu(a0, c, r, shape, st.BC_ZERO, dtype, path, steps, time_block=1)
    fixed = run_gpu(a0, c, r, shape, st.BC_ZERO, dtype, path, steps, time_block=1, chunk=8)
    assert np.array_equal(got, fixed)
    want = oracle.run(a0, ce, r, shape, st.BC_ZERO, steps)
    tol = error_bound(ce, 3, r, shape, dtype, path, steps, np.abs(a0).max())
    err = np.abs(got - want).max()
    assert err <= tol, f"max err {err:.3e} > bound {tol:.3e}"


@pytest.mark.parametrize("dtype", [st.F32, st.F64])
@pytest.mark.parametrize("shape", [st.STAR, st.BOX])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("dims", [(8, 8, 8), (12, 16, 20), (5, 7, 3)])
def test_small_grid_whole_kernel_matches_tiled(dtype, shape, r, dims):
    """Grids that fit the LDS with their halo run the whole-grid gather (the
    library's chunk); a requested chunk keeps the tiled kernel.  Both sum a
    point's taps in the same order: bit for bit equal, and within the bound
    of the oracle, for both boundaries."""
    c = inputs.coefficients(3, r, shape, seed=2700 + r, dtype=np.float64)
    ce = eff_coeffs(c, dtype)
    a0 = inputs.grid(dims, seed=2701, dtype=np.float32 if dtype == st.F32 else np.float64)
    for bc in (st.BC_ZERO, st.BC_PERIODIC):
        whole = run_gpu(a0, c, r, shape, bc, dtype, st.PATH_GATHER, 3, time_block=1)
        tiled = run_gpu(a0, c, r, shape, bc, dtype, st.PATH_GATHER, 3, time_block=1, chunk=4)
        assert np.array_equal(whole, tiled), bc
        want = oracle.run(a0.astype(np.float64), ce, r, shape, bc, 3)
        assert np.abs(whole - want).max() <= error_bound(ce, 3, r, shape, dtype, st.PATH_GATHER, 3, np.abs(a0).max())
