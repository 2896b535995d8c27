"""Host-side tests of the C-ABI library (no GPU needed): symbol exports,
descriptor validation, the band builder against the paper's printed
coefficient-line examples, and the plan's operation counts against the
closed forms of Section 3.4 and Tables 1-2."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(st.LIB_PATH):
        from paper_2310_16298_amd import build
        build.build()
    return st.load_library()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "stencil.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(st.EXPORTS)


def test_status_strings(lib):
    for s in (st.OK, st.EINVAL, st.EUNSUPPORTED, st.ENOMEM, st.EHIP, st.EALIAS, st.EINTERNAL, st.ETOOBIG):
        assert st.status_string(s) not in ("", "unknown status")
    assert st.status_string(99) == "unknown status"
    assert "gfx950" in st.version()


def _box(nd, r):
    return inputs.coefficients(nd, r, inputs.BOX, seed=1, dtype=np.float64)


@pytest.mark.parametrize("bad", [
    dict(dims=(16,), radius=1),                     # 1D has no outer-product form
    dict(dims=(16, 16, 16, 16), radius=1),
    dict(dims=(16, 16), radius=0),
    dict(dims=(16, 16), radius=5),
    dict(dims=(0, 16), radius=1),
    dict(dims=(16, 16), radius=1, boundary=7),
    dict(dims=(16, 16), radius=1, dtype=5),
    dict(dims=(16, 16), radius=1, path=9),
])
def test_desc_check_rejects(lib, bad):
    dims, r = bad.pop("dims"), bad.pop("radius")
    nd = len(dims)
    rr = max(r, 1)
    c = np.ones((2 * rr + 1,) * max(nd, 1)) if nd in (2, 3) else np.ones(3)
    if r != rr or nd not in (2, 3):
        c = np.ones((3, 3))
    d, keep = st.make_desc(dims, r, inputs.BOX, c, **bad)
    if nd not in (2, 3):
        d.ndim = nd
    assert lib.stencil_desc_check(ctypes.byref(d)) == st.EINVAL


def test_desc_check_star_off_axis_and_nonfinite(lib):
    c = inputs.coefficients(2, 2, inputs.STAR, seed=2, dtype=np.float64)
    assert st.desc_check((32, 32), 2, inputs.STAR, c) == st.OK
    bad = c.copy()
    bad[0, 0] = 0.5
    assert st.desc_check((32, 32), 2, inputs.STAR, bad) == st.EINVAL
    bad = c.copy()
    bad[2, 2] = np.nan
    assert st.desc_check((32, 32), 2, inputs.STAR, bad) == st.EINVAL
    c3 = inputs.coefficients(3, 1, inputs.STAR, seed=3, dtype=np.float64)
    bad3 = c3.copy()
    bad3[0, 1, 0] = 1.0
    assert st.desc_check((8, 8, 8), 1, inputs.STAR, bad3) == st.EINVAL


def test_desc_check_unsupported(lib):
    c = _box(2, 1)
    assert st.desc_check((32, 32), 1, inputs.BOX, c, dtype=st.F64, path=st.PATH_MFMA_BF16X3) == st.EUNSUPPORTED
    assert st.desc_check((32, 32), 1, inputs.BOX, c, lines=st.LINES_ORTHOGONAL) == st.EUNSUPPORTED
    s = inputs.coefficients(2, 1, inputs.STAR, seed=4, dtype=np.float64)
    assert st.desc_check((32, 32), 1, inputs.STAR, s, lines=st.LINES_HYBRID) == st.EUNSUPPORTED


def test_null_arguments(lib):
    assert lib.stencil_desc_check(None) == st.EINVAL
    assert lib.stencil_plan(None, None) == st.EINVAL
    assert lib.stencil_plan_info(None, None) == st.EINVAL
    assert lib.stencil_apply(None, None, None, None) == st.EINVAL
    assert lib.stencil_run_steps(None, None, None, 1, None, None) == st.EINVAL
    assert lib.stencil_plan_destroy(None) == st.OK
    out = ctypes.c_void_p(1)
    assert lib.stencil_batch_create(None, None, None, 1, ctypes.byref(out)) == st.EINVAL
    assert out.value is None
    assert lib.stencil_batch_create(None, None, None, 0, None) == st.EINVAL
    assert lib.stencil_batch_run_steps(None, 1, None, None) == st.EINVAL
    assert lib.stencil_batch_info(None, None, None, None) == st.EINVAL
    assert lib.stencil_batch_destroy(None) == st.OK
    h = ctypes.c_void_p(1)
    assert lib.stencil_server_create(None, ctypes.byref(h)) == st.EINVAL
    assert h.value is None
    bad = st.ServerConfig(16, 0, 0)  # arena below 256 bytes
    assert lib.stencil_server_create(ctypes.byref(bad), ctypes.byref(h)) == st.EINVAL
    assert lib.stencil_server_stream(None, None) == st.EINVAL
    assert lib.stencil_server_submit(None, None, None, None, 1, None) == st.EINVAL
    assert lib.stencil_server_tick(None, None) == st.EINVAL
    cnt = ctypes.c_int32(0)
    assert lib.stencil_server_poll(None, None, 0, ctypes.byref(cnt)) == st.EINVAL
    assert lib.stencil_server_cancel(None, 1) == st.EINVAL
    assert lib.stencil_server_destroy(None) == st.OK


def test_tuning_fields(lib):
    c = _box(2, 2)
    assert st.desc_check((64, 64), 2, inputs.BOX, c, block_n=3) == st.EINVAL
    assert st.desc_check((64, 64), 2, inputs.BOX, c, chunk=-1) == st.EINVAL
    assert st.desc_check((64, 64), 2, inputs.BOX, c, time_block=-1) == st.EINVAL
    # n = 4 blocks exist only for the FP32 2D box / parallel-line star MFMA kernel
    assert st.desc_check((64, 64), 2, inputs.BOX, c, dtype=st.F64, path=st.PATH_MFMA, block_n=4) == st.EUNSUPPORTED
    assert st.desc_check((64, 64), 2, inputs.BOX, c, path=st.PATH_MFMA_BF16X3, block_n=4) == st.EUNSUPPORTED
    for bn, want in ((0, 4), (4, 4), (16, 16)):
        info = st.describe((64, 64), 2, inputs.BOX, c, path=st.PATH_MFMA, block_n=bn)
        assert info["block_n"] == want
    assert st.describe((64, 64), 2, inputs.BOX, c, path=st.PATH_GATHER, block_n=16)["block_n"] == 0
    assert st.desc_check((64, 64), 2, inputs.BOX, c, chunk=48) == st.OK


@pytest.mark.parametrize("r,f32max,f64max", [(1, 12, 8), (2, 6, 4), (3, 4, 2), (4, 3, 2)])
def test_time_block_limits(lib, r, f32max, f64max):
    """Time blocks: 2D gather form, the halo r*T rounded up to 4 within the
    kernel's LDS window (12 for FP32, 8 for FP64); 3D: order 1 star and box,
    FP32 stars up to order 4, two steps, last extent a multiple of 4."""
    c = _box(2, r)
    for dt, tmax in ((st.F32, f32max), (st.F64, f64max)):
        assert st.desc_check((100, 100), r, inputs.BOX, c, dtype=dt, time_block=tmax) == st.OK
        assert st.desc_check((100, 100), r, inputs.BOX, c, dtype=dt, time_block=tmax + 1) == st.EUNSUPPORTED
        info = st.describe((100, 100), r, inputs.BOX, c, dtype=dt, time_block=tmax)
        assert info["time_block"] == tmax and info["path"] == st.PATH_GATHER
    # outer products: FP32 2D boxes, two steps, column extent a multiple of 4, library tiles
    assert st.desc_check((100, 100), r, inputs.BOX, c, path=st.PATH_MFMA, time_block=2) == st.OK
    info = st.describe((100, 100), r, inputs.BOX, c, path=st.PATH_MFMA, time_block=2)
    assert info["time_block"] == 2 and info["path"] == st.PATH_MFMA
    for kw in ({"time_block": 3}, {"time_block": 2, "dtype": st.F64}, {"time_block": 2, "block_n": 16},
               {"time_block": 2, "reg_rows": 8}, {"time_block": 2, "tile_width": 128}):
        assert st.desc_check((100, 100), r, inputs.BOX, c, path=st.PATH_MFMA, **kw) == st.EUNSUPPORTED
    assert st.desc_check((100, 98), r, inputs.BOX, c, path=st.PATH_MFMA, time_block=2) == st.EUNSUPPORTED
    cs = inputs.coefficients(2, r, inputs.STAR, seed=1, dtype=np.float64)
    assert st.desc_check((100, 100), r, inputs.STAR, cs, path=st.PATH_MFMA, time_block=2) == st.EUNSUPPORTED
    for sp in (st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3):
        assert st.desc_check((100, 100), r, inputs.BOX, c, path=sp, time_block=2) == st.EUNSUPPORTED
    for dt in (st.F32, st.F64):
        for shape, c3 in ((inputs.BOX, _box(3, r)), (inputs.STAR, inputs.coefficients(3, r, inputs.STAR, seed=1))):
            built3 = r == 1 or (dt == st.F32 and shape == inputs.STAR)
            want3 = st.OK if built3 else st.EUNSUPPORTED
            assert st.desc_check((20, 20, 20), r, shape, c3, dtype=dt, time_block=2) == want3
            assert st.desc_check((20, 20, 20), r, shape, c3, dtype=dt, time_block=3) == st.EUNSUPPORTED
            assert st.desc_check((20, 20, 18), r, shape, c3, dtype=dt, time_block=2) == st.EUNSUPPORTED
            assert st.desc_check((20, 20, 20), r, shape, c3, dtype=dt, path=st.PATH_MFMA, time_block=2) == st.EUNSUPPORTED
            if built3:
                info3 = st.describe((20, 20, 20), r, shape, c3, dtype=dt, time_block=2)
                assert info3["time_block"] == 2 and info3["path"] == st.PATH_GATHER
            # AUTO: two steps per launch on small grids (order 1) and, FP32, on
            # planes of many (j, k) tiles (32 x 64 each)
            f32star1 = dt == st.F32 and shape == inputs.STAR and r == 1
            f32star2 = dt == st.F32 and shape == inputs.STAR and r == 2
            star1 = shape == inputs.STAR and r == 1
            stream96 = r == 1 or f32star2
            stream64 = star1 or f32star2 or (dt == st.F64 and r == 1)
            assert st.describe((64, 64, 64), r, shape, c3, dtype=dt)["time_block"] == (2 if r == 1 else 1)
            assert st.describe((64, 64, 62), r, shape, c3, dtype=dt)["time_block"] == 1
            assert st.describe((128, 128, 128), r, shape, c3, dtype=dt)["time_block"] == (2 if f32star1 else 1)
            assert st.describe((256, 256, 256), r, shape, c3, dtype=dt)["time_block"] == (2 if star1 else 1)
            assert st.describe((8, 512, 384), r, shape, c3, dtype=dt)["time_block"] == (2 if stream96 else 1)
            assert st.describe((8, 512, 320), r, shape, c3, dtype=dt)["time_block"] == (2 if stream64 else 1)
            assert st.describe((8, 384, 320), r, shape, c3, dtype=dt)["time_block"] == (2 if star1 or f32star2 else 1)
            assert st.describe((8, 320, 256), r, shape, c3, dtype=dt)["time_block"] == (2 if star1 else 1)
            assert st.describe((64, 64, 64), r, shape, c3, dtype=dt, chunk=8)["time_block"] == 1
        g3 = _box(3, r)
        g3[0, 0, 0] = 0.0
        assert st.desc_check((20, 20, 20), r, st.GENERAL, g3, dtype=dt, time_block=2) == st.EUNSUPPORTED
    assert st.describe((100, 100), r, inputs.BOX, c, time_block=1)["time_block"] == 1


# ------------------------------------------------------------ band builder

def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def _symbolic_cg():
    """Prime-valued C^g so that a misplaced entry is visible."""
    return np.array([[2., 3., 5.], [7., 11., 13.], [17., 19., 23.]])


def _name_value(cg, name):
    if name == "0":
        return 0.0
    assert name[0] == "C"
    return cg[int(name[1]), int(name[2])]


def test_band_reproduces_eq9(lib):
    """CLS(*,1) with n = 3 (Eq. (9)): column x of the band is the coefficient
    vector multiplying input row A[i-2+x][j]."""
    cg = _symbolic_cg()
    band = st.line_band(cg, 1, 3, 0, 1)
    assert band.shape == (3, 5)
    rows = _golden("eq9_cls_middle_column.txt")
    assert len(rows) == 5
    for x, row in enumerate(rows):
        assert int(row[0]) == x - 2
        want = [_name_value(cg, nm) for nm in row[1:]]
        assert list(band[:, x]) == want


def test_band_reproduces_eq14_row_line(lib):
    """Row line CLS(1,*) (Eq. (14)): input column j reaches outputs j-1, j, j+1
    with C12, C11, C10."""
    cg = _symbolic_cg()
    n = 4
    band = st.line_band(cg, 1, n, 1, 1)  # (n+2) x n
    rows = _golden("eq14_row_line.txt")
    # input column y = q + 1 + d_in ... take the centre input column y = 1 + q0
    for q0 in range(1, n - 1):
        y = q0 + 1  # window column of input column j = output column q0
        for dq, name in rows:
            assert band[y, q0 + int(dq)] == _name_value(cg, name)


def test_band_star_line_cover_eq13(lib):
    """Eq. (13): the 2D 5-point scatter matrix has full middle row/column and
    zero corners; the side column lines of a star therefore carry a single
    weight each (scalar x vector updates)."""
    rows = _golden("eq13_star5_scatter.txt")
    cg = _symbolic_cg() * np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    # C^s = J C^g J read back from the printed matrix
    for sr, row in enumerate(rows):
        for sc, name in enumerate(row):
            assert cg[2 - sr, 2 - sc] == _name_value(_symbolic_cg(), name)
    for b in (0, 2):
        band = st.line_band(cg, 1, 8, 0, b)
        assert np.count_nonzero(band) == 8  # one diagonal: n scalar-vector updates
    band = st.line_band(cg, 1, 8, 0, 1)
    assert np.count_nonzero(band) == 3 * 8


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_band_is_eq1_consistent(lib, r):
    """Summing band x shifted input over all lines reproduces Eq. (1) on an
    interior block (orientation check with an asymmetric C^g)."""
    rng = np.random.default_rng(r)
    cg = rng.integers(-9, 10, (2 * r + 1, 2 * r + 1)).astype(np.float64)
    n = 8
    h = rng.integers(-9, 10, (n + 2 * r, n + 2 * r)).astype(np.float64)  # halo'd input window
    got = np.zeros((n, n))
    for b in range(2 * r + 1):
        got += st.line_band(cg, r, n, 0, b) @ h[:, b:b + n]
    want = np.zeros((n, n))
    for p in range(n):
        for q in range(n):
            want[p, q] = sum(cg[a, b] * h[p + a, q + b] for a in range(2 * r + 1) for b in range(2 * r + 1))
    assert np.array_equal(got, want)
    got2 = np.zeros((n, n))
    for a in range(2 * r + 1):
        got2 += h[a:a + n, :] @ st.line_band(cg, r, n, 1, a)
    assert np.array_equal(got2, want)


def test_line_band_rejects(lib):
    cg = _symbolic_cg()
    with pytest.raises(st.StencilError):
        st.line_band(cg, 1, 3, 2, 0)
    with pytest.raises(st.StencilError):
        st.line_band(cg, 1, 3, 0, 3)


# -------------------------------------------------------- operation counts

@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_counts_2d(lib, r):
    for dt in (st.F32, st.F64):
        box = st.describe((64, 64), r, inputs.BOX, _box(2, r), path=st.PATH_MFMA, dtype=dt)
        n = box["block_n"]
        assert n == (4 if dt == st.F32 else 16)
        assert box["taps"] == (2 * r + 1) ** 2
        assert box["rank1_per_block"] == (2 * r + 1) * (2 * r + n)      # Section 3.4
        assert box["mfma_lines"] == 2 * r + 1
        assert box["k_rows"] >= box["rank1_per_block"]
    s = inputs.coefficients(2, r, inputs.STAR, seed=5, dtype=np.float64)
    par = st.describe((64, 64), r, inputs.STAR, s, path=st.PATH_MFMA, lines=st.LINES_PARALLEL)
    n = par["block_n"]
    assert par["rank1_per_block"] == (2 * r + n) + 2 * r * n        # Table 1, parallel
    assert par["mfma_lines"] == 1 and par["valu_lines"] == 2 * r
    orth = st.describe((64, 64), r, inputs.STAR, s, path=st.PATH_MFMA, lines=st.LINES_ORTHOGONAL)
    n = orth["block_n"]
    assert orth["rank1_per_block"] == 2 * (2 * r + n)               # Table 1, orthogonal
    assert orth["taps"] == 4 * r + 1
    auto = st.describe((64, 64), r, inputs.STAR, s, path=st.PATH_MFMA)
    assert auto["lines"] == (st.LINES_PARALLEL if r == 1 else st.LINES_ORTHOGONAL)
    g = st.describe((64, 64), r, inputs.BOX, _box(2, r), path=st.PATH_GATHER)
    assert g["executed_flops_per_point"] == 2 * (2 * r + 1) ** 2
    assert g["bytes_per_point"] == 8
    assert st.describe((64, 64), r, inputs.BOX, _box(2, r), dtype=st.F64, path=st.PATH_GATHER)["bytes_per_point"] == 16


# ------------------------------------------------------ minimum line cover

def _brute_cover(nz):
    w = nz.shape[0]
    best = 2 * w
    for mask in range(1 << (2 * w)):
        rows = [i for i in range(w) if mask >> i & 1]
        cols = [j for j in range(w) if mask >> (w + j) & 1]
        k = len(rows) + len(cols)
        if k >= best:
            continue
        if all(i in rows or j in cols for i, j in zip(*np.nonzero(nz))):
            best = k
    return best


def test_line_cover_closed_cases(lib):
    """Section 3.5: box -> 2r+1 parallel lines; star -> the two centre lines
    (the orthogonal option of Table 1); a diagonal pattern (Eq. (15)) needs
    2r+1 axis-parallel lines."""
    for r in (1, 2, 3, 4):
        w = 2 * r + 1
        rl, cl = st.line_cover(np.ones((w, w)), r)
        assert len(rl) + len(cl) == w
        star = inputs.coefficients(2, r, inputs.STAR, seed=r, dtype=np.float64)
        rl, cl = st.line_cover(star, r)
        assert (rl, cl) == ([r], [r])
        rl, cl = st.line_cover(np.eye(w), r)
        assert len(rl) + len(cl) == w


@pytest.mark.parametrize("seed", range(40))
def test_line_cover_is_minimum(lib, seed):
    rng = np.random.default_rng(seed)
    r = 1 + seed % 2
    w = 2 * r + 1
    nz = rng.random((w, w)) < rng.uniform(0.1, 0.6)
    c = np.where(nz, rng.uniform(0.5, 1.0, (w, w)), 0.0)
    rl, cl = st.line_cover(c, r)
    for i, j in zip(*np.nonzero(nz)):
        assert i in rl or j in cl
    assert len(rl) + len(cl) == _brute_cover(nz)


# ------------------------------------------------------------ autotuner (host part)

def test_autotune_rejects(lib):
    c = _box(2, 2)
    d, keep = st.make_desc((64, 64), 2, inputs.BOX, c)
    best = st.Desc()
    assert lib.stencil_autotune(None, None, 0, ctypes.byref(best), None, None, None, 0, None) == st.EINVAL
    assert lib.stencil_autotune(ctypes.byref(d), None, 0, None, None, None, None, 0, None) == st.EINVAL
    assert lib.stencil_autotune(ctypes.byref(d), None, 8, ctypes.byref(best), None, None, None, 0, None) == st.EINVAL
    assert lib.stencil_autotune(ctypes.byref(d), None, 0, ctypes.byref(best), None, None, None, 4, None) == st.EINVAL
    bad, keep2 = st.make_desc((64, 64), 5, inputs.BOX, _box(2, 4))
    assert lib.stencil_autotune(ctypes.byref(bad), None, 0, ctypes.byref(best), None, None, None, 0, None) == st.EINVAL


def test_autotune_cache_hit_needs_no_device(lib, tmp_path):
    """A cached entry is returned without measuring (the last entry of a key
    wins; other keys and malformed lines are skipped)."""
    cache = tmp_path / "tune.txt"
    key = "nd=2 shape=1 r=2 dtype=0 bc=1 dims=64,80,1 req=0,0,0,0,0,0,0,0"
    cache.write_text(
        "garbage line\n"
        f"{key} -> path=2 lines=1 block_n=16 chunk=0 time_block=0 reg_rows=0 tile_width=0 ms=0.250000\n"
        "nd=2 shape=1 r=2 dtype=0 bc=1 dims=64,81,1 req=0,0,0,0,0,0,0,0 -> path=1 lines=0 block_n=0 chunk=0 "
        "time_block=3 reg_rows=0 tile_width=0 ms=0.1\n"
        f"{key} -> path=2 lines=1 block_n=4 chunk=32 time_block=0 ms=0.2\n"  # an older format: skipped
        f"{key} -> path=2 lines=1 block_n=4 chunk=32 time_block=0 reg_rows=8 tile_width=128 ms=0.125000\n")
    knobs, ms, rows = st.autotune((64, 80), 2, inputs.BOX, _box(2, 2), boundary=st.BC_PERIODIC, cache=str(cache))
    assert knobs == {"path": st.PATH_MFMA, "lines": st.LINES_PARALLEL, "block_n": 4, "chunk": 32, "time_block": 0,
                     "reg_rows": 8, "tile_width": 128}
    assert ms == 0.125 and rows == []


# ------------------------------------------------------------ general shapes (Section 3.5)

def _pattern_cg(r, mask, seed):
    rng = np.random.default_rng(seed)
    return np.where(mask, rng.uniform(0.1, 1.0, size=mask.shape), 0.0)


@pytest.mark.parametrize("seed", range(12))
def test_general_plan_uses_minimum_cover(lib, seed):
    rng = np.random.default_rng(900 + seed)
    r = int(rng.integers(1, 5))
    w = 2 * r + 1
    mask = rng.random((w, w)) < rng.uniform(0.1, 0.6)
    c = _pattern_cg(r, mask, seed)
    rows, cols = st.line_cover(c, r)
    kl = -(-(16 + 2 * r) // 4) * 4
    nzc = int(mask.any(axis=0).sum())
    # n = 4 blocks: the nonzero columns alone when not dearer than the cover
    # with lines along j counted 1.5
    n4 = nzc if rows and 2 * nzc <= 2 * len(cols) + 3 * len(rows) else len(rows) + len(cols)
    for dt, bn, krows in ((st.F32, 0, 4 + 2 * r), (st.F32, 16, kl), (st.F64, 0, kl)):
        info = st.describe((64, 64), r, st.GENERAL, c, path=st.PATH_MFMA, dtype=dt, block_n=bn)
        assert info["mfma_lines"] == (n4 if krows == 4 + 2 * r else len(rows) + len(cols)) <= w
        assert info["taps"] == int(mask.sum())
        assert info["block_n"] == (4 if krows == 4 + 2 * r else 16) and info["valu_lines"] == 0
        assert info["k_rows"] == info["mfma_lines"] * krows
    assert st.desc_check((64, 64), r, st.GENERAL, c, lines=st.LINES_PARALLEL) == st.EUNSUPPORTED
    assert st.desc_check((64, 64), r, st.GENERAL, c, path=st.PATH_MFMA, dtype=st.F64, block_n=4) == st.EUNSUPPORTED
    # other paths take GENERAL as a box; so does AUTO in 3D (outer products from r = 3)
    assert st.describe((64, 64), r, st.GENERAL, c, path=st.PATH_GATHER)["path"] == st.PATH_GATHER
    want3 = st.PATH_MFMA if r >= 3 else st.PATH_GATHER
    assert st.describe((16, 16, 16), r, st.GENERAL, _box(3, r))["path"] == want3


@pytest.mark.parametrize("shape", [inputs.STAR, inputs.BOX])
def test_auto_path_choice(lib, shape):
    """AUTO: outer products on MFMA for FP32 boxes of radius >= 3 (2D and 3D),
    FP64 3D stars of radius 4 and 2D GENERAL covers, the gather kernel for the rest
    when the column extent allows direct-to-LDS windows (a multiple of 4; 2D),
    MFMA on other 2D extents; on FP32 2D direct-to-LDS grids wider than 64
    columns with no kernel knob set, the time-blocked gather."""
    for r in (1, 2, 3, 4):
        c = inputs.coefficients(2, r, shape, seed=3, dtype=np.float64)
        heavy = shape == inputs.BOX and r >= 3
        # FP32 direct-to-LDS grids wider than 64 columns: the time-blocked gather
        info = st.describe((96, 96), r, shape, c, dtype=st.F32)
        assert info["path"] == st.PATH_GATHER
        assert info["time_block"] == ({1: 8, 2: 4, 3: 4, 4: 3} if shape == inputs.STAR else {1: 8, 2: 4, 3: 4, 4: 2})[r]
        # any kernel knob set keeps one step per launch (and the one-step choice)
        one = st.describe((96, 96), r, shape, c, dtype=st.F32, chunk=64)
        assert one["time_block"] == 1 and one["path"] == (st.PATH_MFMA if heavy else st.PATH_GATHER)
        assert st.describe((96, 96), r, shape, c, dtype=st.F32, time_block=1)["time_block"] == 1
        assert st.describe((96, 96), r, shape, c, dtype=st.F32, path=st.PATH_GATHER)["time_block"] == 1
        info64 = st.describe((96, 96), r, shape, c, dtype=st.F64)
        assert info64["path"] == st.PATH_GATHER
        assert info64["time_block"] == ({1: 8, 2: 4, 3: 2, 4: 2} if shape == inputs.STAR else {1: 8, 2: 4, 3: 1, 4: 1})[r]
        # 64 columns: the time-blocked gather where the table has a step
        # count (the FP32 box of order 4 keeps the outer products)
        d32 = st.describe((64, 64), r, shape, c, dtype=st.F32)
        if shape == inputs.BOX and r == 4:
            assert d32["path"] == st.PATH_MFMA and d32["time_block"] == 1
        else:
            assert d32["path"] == st.PATH_GATHER
            assert d32["time_block"] == ({1: 8, 2: 4, 3: 4, 4: 3} if shape == inputs.STAR else {1: 8, 2: 4, 3: 4})[r]
        d64 = st.describe((64, 64), r, shape, c, dtype=st.F64)
        t64 = ({1: 8, 2: 4, 3: 2, 4: 2} if shape == inputs.STAR else {1: 8, 2: 4, 3: 1, 4: 1})[r]
        assert d64["time_block"] == t64 and d64["path"] == st.PATH_GATHER
        # narrower grids are time-blocked as well (the same table) ...
        assert st.describe((60, 60), r, shape, c, dtype=st.F32)["time_block"] == d32["time_block"]
        assert st.describe((60, 60), r, shape, c, dtype=st.F64)["time_block"] == t64
        # ... and one step per launch (a knob set): stars and the FP64 9-point
        # box take the outer products up to 64 columns
        narrow = shape == inputs.STAR or heavy
        one32 = st.describe((60, 60), r, shape, c, dtype=st.F32, chunk=16)
        assert one32["path"] == (st.PATH_MFMA if narrow else st.PATH_GATHER) and one32["time_block"] == 1
        narrow64 = shape == inputs.STAR or r == 1
        one64 = st.describe((60, 60), r, shape, c, dtype=st.F64, chunk=16)
        assert one64["path"] == (st.PATH_MFMA if narrow64 else st.PATH_GATHER) and one64["time_block"] == 1
        for dt in (st.F32, st.F64):
            assert st.describe((64, 66), r, shape, c, dtype=dt)["path"] == st.PATH_MFMA
        g = c.copy()
        g[0, 0] = 0.0  # not a full box: a GENERAL stencil
        assert st.describe((64, 64), r, st.GENERAL, g, dtype=st.F32)["path"] == st.PATH_MFMA
        c3 = inputs.coefficients(3, r, shape, seed=3, dtype=np.float64)
        assert st.describe((16, 16, 16), r, shape, c3, dtype=st.F32)["path"] == (st.PATH_MFMA if heavy else st.PATH_GATHER)
        assert st.describe((16, 16, 16), r, shape, c3, dtype=st.F64)["path"] == st.PATH_GATHER


def test_3d_mfma_block_edge(lib):
    """FP32 3D outer products default to n = 4 blocks for stars and boxes
    (executed flops 2 (2r+4) per line and point); FP64 uses 16x16 blocks, and
    the 16x16 form of a box exists up to r = 2."""
    for r in (1, 2, 3, 4):
        s = inputs.coefficients(3, r, inputs.STAR, seed=5, dtype=np.float64)
        info = st.describe((20, 20, 20), r, inputs.STAR, s, path=st.PATH_MFMA)
        assert info["block_n"] == 4 and info["k_rows"] == 2 * (2 * r + 4) and info["valu_lines"] == 2 * r
        assert st.describe((20, 20, 20), r, inputs.STAR, s, path=st.PATH_MFMA, block_n=16)["block_n"] == 16
        assert st.describe((20, 20, 20), r, inputs.STAR, s, path=st.PATH_MFMA, dtype=st.F64)["block_n"] == 16
    for r in (1, 2, 3, 4):
        w = 2 * r + 1
        b = st.describe((20, 20, 20), r, inputs.BOX, _box(3, r), path=st.PATH_MFMA)
        assert b["block_n"] == 4 and b["k_rows"] == w * w * (2 * r + 4) and b["mfma_lines"] == w * w
    assert st.describe((20, 20, 20), 2, inputs.BOX, _box(3, 2), path=st.PATH_MFMA, block_n=16)["block_n"] == 16
    assert st.desc_check((20, 20, 20), 3, inputs.BOX, _box(3, 3), path=st.PATH_MFMA, block_n=16) == st.EUNSUPPORTED
    assert st.describe((20, 20, 20), 2, inputs.BOX, _box(3, 2), path=st.PATH_MFMA, dtype=st.F64)["block_n"] == 16


def test_general_gather_choice(lib):
    """GENERAL 2D: the gather path walks the nonzero taps up to a measured count
    per order and dtype (every tap beyond it); AUTO on FP32 direct-to-LDS grids wider
    than 64 columns takes that gather when its fitted cost (12290 + 403 n per
    point, n nonzero taps capped at the measured count) is below the line
    cover's (12910 + 1530 L (2r+4)/12, L lines), and the cover otherwise."""
    limit = {st.F32: (0, 3, 10, 27, 43), st.F64: (0, 5, 10, 27, 31)}
    for r in (1, 2, 3, 4):
        w = 2 * r + 1
        for dt in (st.F32, st.F64):
            for n in range(1, w * w + 1):
                c = np.zeros(w * w); c[:n] = 0.1
                info = st.describe((256, 256), r, st.GENERAL, c.reshape(w, w), path=st.PATH_GATHER, dtype=dt)
                want = 2.0 * (n if n <= limit[dt][r] else w * w)
                assert info["taps"] == n and info["executed_flops_per_point"] == want, (r, dt, n)
        diag = np.eye(w)
        info = st.describe((256, 256), r, st.GENERAL, diag, path=st.PATH_GATHER, dtype=st.F32)
        assert info["taps"] == w and info["executed_flops_per_point"] == 2.0 * w
        full = np.ones((w, w))
        full[0, 0] = 0.0
        info = st.describe((256, 256), r, st.GENERAL, full, path=st.PATH_GATHER, dtype=st.F64)
        assert info["taps"] == w * w - 1 and info["executed_flops_per_point"] == 2.0 * w * w
        for mask in (np.eye(w, dtype=bool), np.eye(w, dtype=bool) | np.eye(w, dtype=bool)[::-1],
                     np.ones((w, w), dtype=bool), np.pad(np.ones((1, w), dtype=bool), ((w - 1, 0), (0, 0)))):
            c = np.where(mask, 0.5, 0.0)
            c[-1, 0] = 0.5  # plus one corner
            n = int((c != 0).sum())
            rows, cols = st.line_cover(c, r)
            nzc = int((c != 0).any(axis=0).sum())
            L = nzc if rows and 2 * nzc <= 2 * len(cols) + 3 * len(rows) else len(rows) + len(cols)
            n_eff = min(n, limit[st.F32][r])  # past the limit: the all-tap gather, priced at the crossover
            want = st.PATH_GATHER if 12 * 403 * n_eff < 12 * 620 + 1530 * L * (4 + 2 * r) else st.PATH_MFMA
            assert st.describe((256, 256), r, st.GENERAL, c, dtype=st.F32)["path"] == want, (r, n, L)
            # narrow or ragged grids keep the cover; FP64 the gather
            assert st.describe((64, 64), r, st.GENERAL, c, dtype=st.F32)["path"] == st.PATH_MFMA
            assert st.describe((256, 258), r, st.GENERAL, c, dtype=st.F32)["path"] == st.PATH_MFMA
            assert st.describe((256, 256), r, st.GENERAL, c, dtype=st.F64)["path"] == st.PATH_GATHER
    # extents without direct-to-LDS windows run (and report) every tap
    for dims, dt in (((256, 258), st.F64), ((64, 64), st.F32), ((80, 62), st.F64)):
        info = st.describe(dims, 2, st.GENERAL, np.eye(5), path=st.PATH_GATHER, dtype=dt)
        assert info["executed_flops_per_point"] == 2.0 * 25, dims
    assert st.describe((80, 64), 2, st.GENERAL, np.eye(5), path=st.PATH_GATHER, dtype=st.F64)["executed_flops_per_point"] == 10.0
    # past the tap limit AUTO prices the all-tap gather (which the plan then
    # runs) at the limit's cost: order 2, diagonal + 6 weights = 11 taps over
    # 5 lines -> gather, every one of the 25 taps executed
    c = np.eye(5)
    c[0, 1:4] = c[4, 1:4] = 0.5
    assert int((c != 0).sum()) == 11 and len(sum(st.line_cover(c, 2), [])) == 5
    info = st.describe((256, 256), 2, st.GENERAL, c, dtype=st.F32)
    assert info["path"] == st.PATH_GATHER and info["executed_flops_per_point"] == 50.0
    # a full order-2 GENERAL pattern: the all-tap gather (measured 617 vs 604 GSt/s for the box)
    assert st.describe((256, 256), 2, st.GENERAL, np.ones((5, 5)), dtype=st.F32)["path"] == st.PATH_GATHER
    # the measured order-4 cases: diagonals to the gather, short covers to MFMA
    w = 9
    assert st.describe((8192, 8192), 4, st.GENERAL, np.eye(w), dtype=st.F32)["path"] == st.PATH_GATHER
    ell = np.zeros((w, w)); ell[w - 1, :] = 1.0; ell[:, 0] = 1.0
    assert st.describe((8192, 8192), 4, st.GENERAL, ell, dtype=st.F32)["path"] == st.PATH_MFMA


def test_general_3d_gather_choice(lib):
    """GENERAL 3D: the gather path walks the nonzero taps up to 5 / 44 / 128 /
    128 of them (FP32, orders 1..4; FP64 3 / 40 / 128 / 128), every tap beyond;
    AUTO on FP32 takes that gather over the box outer products up to 88 (r = 3)
    and 128 (r = 4) nonzero taps."""
    limit = {st.F32: (0, 5, 44, 128, 128), st.F64: (0, 3, 40, 128, 128)}
    for r in (1, 2, 3, 4):
        w = 2 * r + 1
        for dt in (st.F32, st.F64):
            for n in sorted({1, 2, 3, 4, 5, 6, 16, 27, 40, 41, 44, 45, 64, 65, 88, 89, 124, 125, 128, 129, w ** 3}):
                if n > w ** 3:
                    continue
                c = np.zeros(w ** 3); c[:n] = 0.01
                c = c.reshape(w, w, w)
                info = st.describe((32, 32, 64), r, st.GENERAL, c, path=st.PATH_GATHER, dtype=dt)
                want = 2.0 * (n if n <= limit[dt][r] else w ** 3)
                assert info["taps"] == n and info["executed_flops_per_point"] == want, (r, dt, n)
                auto = st.describe((32, 32, 64), r, st.GENERAL, c, dtype=dt)["path"]
                mfma = dt == st.F32 and r >= 3 and n > {3: 88, 4: 128}[r]
                assert auto == (st.PATH_MFMA if mfma else st.PATH_GATHER), (r, dt, n)


# ---------------------------------------------------------------- no-allocation entry point

def _noalloc(lib, desc, b0=1 << 20, b1=1 << 30, steps=1):
    idx = ctypes.c_int32(-1)
    return lib.stencil_run_steps_noalloc(ctypes.byref(desc), b0, b1, steps, None, ctypes.byref(idx)), idx.value


def test_noalloc_rejects_operands_beyond_scratch_before_any_device_call(lib):
    # FP64 3D box of order 2 on 16x16 blocks: 25 lines x 5 K chunks x 64 lanes x 8 B = 64000 B of fragments
    c = inputs.coefficients(3, 2, inputs.BOX, seed=3, dtype=np.float64)
    d, keep = st.make_desc((40, 40, 64), 2, st.BOX, c, dtype=st.F64, path=st.PATH_MFMA)
    info = st.describe((40, 40, 64), 2, st.BOX, c, dtype=st.F64, path=st.PATH_MFMA)
    assert info["operand_bytes"] > st.NOALLOC_SCRATCH_BYTES
    assert _noalloc(lib, d)[0] == st.ETOOBIG  # no GPU here: the check precedes every device call


def test_noalloc_argument_errors(lib):
    c = _box(2, 1)
    d, keep = st.make_desc((64, 64), 1, st.BOX, c)
    assert lib.stencil_run_steps_noalloc(None, 1 << 20, 1 << 30, 1, None, None) == st.EINVAL
    assert lib.stencil_run_steps_noalloc(ctypes.byref(d), None, 1 << 30, 1, None, None) == st.EINVAL
    assert lib.stencil_run_steps_noalloc(ctypes.byref(d), 1 << 20, 1 << 30, -1, None, None) == st.EINVAL
    assert _noalloc(lib, d, b0=1 << 20, b1=(1 << 20) + 64)[0] == st.EALIAS
    # steps == 0 enqueues nothing and touches no device
    assert _noalloc(lib, d, steps=0) == (st.OK, 0)
    bad, keep2 = st.make_desc((64, 64), 5, st.BOX, np.ones(121))
    assert _noalloc(lib, bad)[0] == st.EINVAL


@pytest.mark.parametrize("nd", [2, 3])
@pytest.mark.parametrize("dtype", [st.F32, st.F64])
def test_operand_bytes_of_auto_plans_fit_the_noalloc_scratch(lib, nd, dtype):
    dims = (520, 384) if nd == 2 else (40, 48, 64)
    for r in range(1, 5):
        for shape in (st.STAR, st.BOX):
            c = inputs.coefficients(nd, r, shape, seed=r, dtype=np.float64)
            for path in (st.PATH_AUTO, st.PATH_GATHER, st.PATH_MFMA):
                if st.desc_check(dims, r, shape, c, dtype=dtype, path=path) != st.OK:
                    continue
                info = st.describe(dims, r, shape, c, dtype=dtype, path=path)
                if nd == 3 and dtype == st.F64 and shape == st.BOX and r == 2 and path == st.PATH_MFMA:
                    continue  # 64000 B of FP64 16x16 fragments: the one plan beyond the scratch
                assert 256 < info["operand_bytes"] <= st.NOALLOC_SCRATCH_BYTES, (r, shape, path, info)
                assert info["operand_bytes"] % 256 == 0


# ------------------------------------------------ register and workgroup tiles

def test_tile_knobs(lib):
    """reg_rows / tile_width select the register tile (rows per wave) and the
    workgroup tile (columns) of the 2D FP32 box outer products on n = 4 blocks;
    the plan reports them; other plans reject non-default values."""
    c = _box(2, 3)
    info = st.describe((256, 512), 3, inputs.BOX, c, path=st.PATH_MFMA)
    assert (info["reg_rows"], info["tile_width"]) == (16, 256)
    for rows in (8, 16, 32):
        for width in (128, 256):
            info = st.describe((256, 512), 3, inputs.BOX, c, path=st.PATH_MFMA, reg_rows=rows, tile_width=width)
            assert (info["reg_rows"], info["tile_width"], info["block_n"]) == (rows, width, 4)
    assert st.desc_check((256, 512), 3, inputs.BOX, c, reg_rows=12) == st.EINVAL
    assert st.desc_check((256, 512), 3, inputs.BOX, c, tile_width=64) == st.EINVAL
    s = inputs.coefficients(2, 3, inputs.STAR, seed=4, dtype=np.float64)
    for kw in (dict(path=st.PATH_GATHER), dict(path=st.PATH_MFMA, block_n=16), dict(path=st.PATH_MFMA_BF16X3)):
        assert st.desc_check((256, 512), 3, inputs.BOX, c, reg_rows=8, **kw) == st.EUNSUPPORTED, kw
    assert st.desc_check((256, 512), 3, inputs.STAR, s, path=st.PATH_MFMA, tile_width=128) == st.EUNSUPPORTED
    assert st.desc_check((16, 16, 16), 1, inputs.BOX, _box(3, 1), path=st.PATH_MFMA, reg_rows=32) == st.EUNSUPPORTED
    # the library's choice spelled out is accepted everywhere
    assert st.desc_check((256, 512), 3, inputs.BOX, c, path=st.PATH_GATHER, reg_rows=16, tile_width=256) == st.OK
    # gather and 3D plans report no tile
    assert st.describe((256, 512), 3, inputs.BOX, c, path=st.PATH_GATHER)["reg_rows"] == 0


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_split_3d_boxes_resolve(r):
    """FP32 3D boxes of every order take the split-precision products: all
    (2r+1)^2 lines along k on 16x16x32 MFMAs (K = 32 per line), three
    products (hi*hi, hi*lo, lo*hi) each; FP64 has no split path."""
    w = 2 * r + 1
    for path in (st.PATH_MFMA_BF16X3, st.PATH_MFMA_F16X3):
        info = st.describe((16, 16, 16), r, inputs.BOX, _box(3, r), path=path)
        assert info["path"] == path and info["mfma_lines"] == w * w and info["valu_lines"] == 0
        assert info["k_rows"] == 32 * w * w
        assert info["executed_flops_per_point"] == 3.0 * 2.0 * 32 * w * w
        assert st.desc_check((16, 16, 16), r, inputs.BOX, _box(3, r), dtype=st.F64, path=path) == st.EUNSUPPORTED
