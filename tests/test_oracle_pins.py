"""Pins of the CPU FP64 oracle against facts fixed by the paper and by
mathematics (no GPU).  Each pin is independent of the oracle's own code:
printed equations (golden fixtures), a library routine (scipy.ndimage),
a dense operator built from the fixture's term list, the scatter form of
Eq. (3)-(5), closed forms (FFT symbol, sine eigenmodes, constants,
polynomial moments).  A mistake such as a transposed or mirrored coefficient
tensor, a wrong boundary rule or a dropped tap fails at least one of them.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

from paper_2310_16298_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STAR, BOX = 0, 1
ZERO, PERIODIC = 0, 1


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _masked(c, radius, shape):
    return np.where(inputs.tap_mask(c.ndim, radius, shape), c, 0.0)


# ---------------------------------------------------------------- Eq. (1)

def test_eq1_printed_term_list(oracle_mod):
    """Interior points equal the nine printed terms of Eq. (1)."""
    terms = [tuple(int(v) for v in row) for row in _read_rows("eq1_gather_2d9p.txt")]
    assert len(terms) == 9
    primes = np.array([[2, 3, 5], [7, 11, 13], [17, 19, 23]], dtype=np.float64)
    a = inputs.int_grid((9, 11), seed=1).astype(np.float64)
    out = oracle_mod.run(a, primes, 1, BOX, ZERO, 1)
    for i in range(1, 8):
        for j in range(1, 10):
            want = sum(primes[cr, cc] * a[i + di, j + dj] for cr, cc, di, dj in terms)
            assert out[i, j] == want


def test_eq1_delta_response(oracle_mod):
    """A unit impulse at (i0, j0) lands C^g[a][b] at (i0-a+r, j0-b+r) (Eq. (1)
    read as a function of the output position)."""
    for r in (1, 2, 3):
        w = 2 * r + 1
        c = np.arange(1, w * w + 1, dtype=np.float64).reshape(w, w) * 3.0 + 1.0
        a = np.zeros((13, 14))
        a[6, 7] = 1.0
        out = oracle_mod.run(a, c, r, BOX, ZERO, 1)
        want = np.zeros_like(a)
        for aa in range(w):
            for bb in range(w):
                want[6 - aa + r, 7 - bb + r] = c[aa, bb]
        assert np.array_equal(out, want)


# ------------------------------------------------------- library routine

@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("bc", [ZERO, PERIODIC])
def test_matches_scipy_correlate(oracle_mod, ndim, radius, shape, bc):
    dims = (17, 23) if ndim == 2 else (9, 11, 13)
    a = inputs.grid(dims, seed=10 + radius, dtype=np.float64)
    c = np.random.default_rng(100 + radius).uniform(-1, 1, (2 * radius + 1,) * ndim)
    out = oracle_mod.run(a, c, radius, shape, bc, 1)   # star: oracle must ignore off-axis taps
    mode = "grid-wrap" if bc == PERIODIC else "constant"
    want = ndi.correlate(a, _masked(c, radius, shape), mode=mode, cval=0.0)
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-13 * np.abs(c).sum())


def test_periodic_small_grid_wraps_repeatedly(oracle_mod):
    """Extents smaller than the stencil width wrap more than once."""
    for dims in [(1, 5), (3, 2), (2, 2)]:
        a = inputs.grid(dims, seed=3, dtype=np.float64)
        c = np.random.default_rng(4).uniform(0, 1, (9, 9))
        out = oracle_mod.run(a, c, 4, BOX, PERIODIC, 1)
        want = np.zeros_like(a)
        for i, j in itertools.product(range(dims[0]), range(dims[1])):
            for p, q in itertools.product(range(9), range(9)):
                want[i, j] += c[p, q] * a[(i + p - 4) % dims[0], (j + q - 4) % dims[1]]
        np.testing.assert_allclose(out, want, rtol=0, atol=1e-13 * c.sum())


# --------------------------------------------------- dense operator, T steps

def _dense_operator(dims, radius, shape, bc, c):
    """Operator matrix built from the printed tap list pattern (input offset
    o carries C^g[o + r]) with Python loops."""
    n = int(np.prod(dims))
    m = np.zeros((n, n))
    pts = list(itertools.product(*[range(d) for d in dims]))
    offs = list(itertools.product(range(-radius, radius + 1), repeat=len(dims)))
    for row, x in enumerate(pts):
        for o in offs:
            if shape == STAR and sum(1 for v in o if v) > 1:
                continue
            y = [x[d] + o[d] for d in range(len(dims))]
            if bc == PERIODIC:
                y = [y[d] % dims[d] for d in range(len(dims))]
            elif any(y[d] < 0 or y[d] >= dims[d] for d in range(len(dims))):
                continue
            col = int(np.ravel_multi_index(tuple(y), dims))
            m[row, col] += c[tuple(v + radius for v in o)]
    return m


@pytest.mark.parametrize("dims,radius", [((6, 7), 1), ((5, 8), 2), ((4, 5, 6), 1), ((5, 4, 3), 2)])
@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("bc", [ZERO, PERIODIC])
def test_dense_operator_power(oracle_mod, dims, radius, shape, bc):
    a = inputs.grid(dims, seed=5, dtype=np.float64)
    c = inputs.coefficients(len(dims), radius, BOX, seed=6, dtype=np.float64)
    steps = 4
    m = _dense_operator(dims, radius, shape, bc, c)
    want = (np.linalg.matrix_power(m, steps) @ a.ravel()).reshape(dims)
    out = oracle_mod.run(a, c, radius, shape, bc, steps)
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-13)


# --------------------------------------------------------- scatter form

def _scatter_matrix_r1():
    """C^s layout for r = 1 as printed in Eq. (3)/(4)."""
    return [tuple(int(v) for v in row) for row in _read_rows("eq3_scatter_2d9p.txt")]


def test_eq4_is_row_and_column_reversal():
    """Eq. (5)-(6): C^s = J C^g J reproduces the printed C^s of Eq. (4)."""
    cg = np.arange(9).reshape(3, 3)
    j3 = np.fliplr(np.eye(3, dtype=int))
    cs = j3 @ cg @ j3
    for sr, sc, gr, gc in _scatter_matrix_r1():
        assert cs[sr, sc] == cg[gr, gc]


def _scatter_run(a, cg, radius, shape, bc, steps):
    """Independent scatter-form sweep (Eq. (3)): every input element adds
    C^s * A[i][j] to its (2r+1)^d output neighbourhood, C^s = J C^g J."""
    cs = _masked(cg, radius, shape)
    for axis in range(a.ndim):
        cs = np.flip(cs, axis=axis)
    dims = a.shape
    cur = a.copy()
    for _ in range(steps):
        out = np.zeros_like(cur)
        for x in itertools.product(*[range(d) for d in dims]):
            v = cur[x]
            for s in itertools.product(range(2 * radius + 1), repeat=a.ndim):
                w = cs[s]
                if w == 0.0:
                    continue
                y = [x[d] + s[d] - radius for d in range(a.ndim)]
                if bc == PERIODIC:
                    y = [y[d] % dims[d] for d in range(a.ndim)]
                elif any(y[d] < 0 or y[d] >= dims[d] for d in range(a.ndim)):
                    continue
                out[tuple(y)] += w * v
        cur = out
    return cur


def test_scatter_r1_printed_layout_matches_oracle(oracle_mod):
    """Scatter with the printed C^s layout (r = 1), integer data: bit-exact."""
    cg = inputs.int_coefficients(2, 1, BOX, seed=7, dtype=np.float64)
    a = inputs.int_grid((7, 9), seed=8, dtype=np.float64)
    out = np.zeros_like(a)
    for i, j in itertools.product(range(7), range(9)):
        for sr, sc, gr, gc in _scatter_matrix_r1():
            ii, jj = i - 1 + sr, j - 1 + sc
            if 0 <= ii < 7 and 0 <= jj < 9:
                out[ii, jj] += cg[gr, gc] * a[i, j]
    assert np.array_equal(out, oracle_mod.run(a, cg, 1, BOX, ZERO, 1))


@pytest.mark.parametrize("dims,radius", [((6, 9), 2), ((5, 7), 3), ((4, 5, 6), 1), ((5, 5, 5), 2)])
@pytest.mark.parametrize("shape", [STAR, BOX])
@pytest.mark.parametrize("bc", [ZERO, PERIODIC])
def test_scatter_equals_gather_integers(oracle_mod, dims, radius, shape, bc):
    cg = inputs.int_coefficients(len(dims), radius, BOX, seed=9, dtype=np.float64)
    a = inputs.int_grid(dims, seed=10, dtype=np.float64)
    want = _scatter_run(a, cg, radius, shape, bc, 2)
    assert np.array_equal(oracle_mod.run(a, cg, radius, shape, bc, 2), want)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("dims,radius,shape", [((32, 24), 2, BOX), ((16, 20), 4, STAR),
                                               ((12, 10, 14), 1, BOX), ((10, 12, 8), 3, STAR)])
def test_periodic_fft_symbol(oracle_mod, dims, radius, shape):
    """Periodic T-step result = inverse FFT of A_hat * lambda^T with
    lambda(k) = sum_o C^g[o] exp(+2 pi i k.o / N)."""
    nd = len(dims)
    a = inputs.grid(dims, seed=11, dtype=np.float64)
    c = inputs.coefficients(nd, radius, shape, seed=12, dtype=np.float64)
    steps = 5
    lam = np.zeros(dims, dtype=complex)
    freqs = np.meshgrid(*[np.arange(n) / n for n in dims], indexing="ij")
    for o in itertools.product(range(-radius, radius + 1), repeat=nd):
        w = c[tuple(v + radius for v in o)]
        if w == 0.0:
            continue
        phase = sum(2j * np.pi * freqs[d] * o[d] for d in range(nd))
        lam += w * np.exp(phase)
    want = np.fft.ifftn(np.fft.fftn(a) * lam ** steps).real
    out = oracle_mod.run(a, c, radius, shape, PERIODIC, steps)
    np.testing.assert_allclose(out, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("dims,p,q", [((512, 512), 1, 1), ((512, 512), 7, 300), ((37, 50), 3, 11)])
def test_sine_eigenmodes_zero_halo(oracle_mod, dims, p, q):
    """The 2D five-point diffusion operator (centre 1/2, neighbours 1/8) with a
    zero halo has eigenvectors sin(pi p (i+1)/(M+1)) sin(pi q (j+1)/(N+1))."""
    m, n = dims
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    # reduce the angle index exactly in integers so the mode is exact to ~1 ulp
    ki = (p * (i + 1)) % (2 * (m + 1))
    kj = (q * (j + 1)) % (2 * (n + 1))
    a = np.sin(np.pi * ki / (m + 1)) * np.sin(np.pi * kj / (n + 1))
    lam = 0.5 + 0.25 * np.cos(np.pi * p / (m + 1)) + 0.25 * np.cos(np.pi * q / (n + 1))
    steps = 10
    out = oracle_mod.run(a, inputs.diffusion_5pt(), 1, STAR, ZERO, steps)
    np.testing.assert_allclose(out, lam ** steps * a, rtol=0, atol=2e-14)


@pytest.mark.parametrize("ndim,radius,shape", [(2, 3, BOX), (2, 2, STAR), (3, 2, BOX), (3, 4, STAR)])
def test_constant_field(oracle_mod, ndim, radius, shape):
    """A constant c maps to c * sum(C^g) (exact with dyadic values);
    periodic everywhere, zero halo at distance >= r*T from every face."""
    w = 2 * radius + 1
    rng = np.random.default_rng(13)
    c = np.where(inputs.tap_mask(ndim, radius, shape), rng.integers(-16, 17, (w,) * ndim) / 64.0, 0.0)
    dims = (20, 21) if ndim == 2 else (12, 13, 14)
    a = np.full(dims, 0.75)
    steps = 2
    total = c.sum()
    out_p = oracle_mod.run(a, c, radius, shape, PERIODIC, steps)
    assert np.all(out_p == 0.75 * total ** steps)
    out_z = oracle_mod.run(a, c, radius, shape, ZERO, steps)
    h = radius * steps
    core = out_z[tuple(slice(h, d - h) for d in dims)]
    assert np.all(core == 0.75 * total ** steps)


def test_polynomial_moments(oracle_mod):
    """Quadratic p: one step gives sum over |alpha| <= 2 of
    d^alpha p(x) / alpha! * M_alpha with M_alpha = sum_o C^g[o] o^alpha
    (Taylor expansion, exact), at points >= r from the faces."""
    r = 3
    w = 2 * r + 1
    c = inputs.int_coefficients(2, r, BOX, seed=14, dtype=np.float64)
    k = [3, -2, 5, 1, -4, 2]  # p = k0 + k1 i + k2 j + k3 i^2 + k4 i j + k5 j^2
    m, n = 20, 23

    def p(i, j):
        return k[0] + k[1] * i + k[2] * j + k[3] * i * i + k[4] * i * j + k[5] * j * j

    a = np.array([[p(i, j) for j in range(n)] for i in range(m)], dtype=np.float64)
    out = oracle_mod.run(a, c, r, BOX, ZERO, 1)
    mom = {}
    for al in [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]:
        mom[al] = sum(Fraction(int(c[u, v])) * (u - r) ** al[0] * (v - r) ** al[1]
                      for u in range(w) for v in range(w))
    for i in range(r, m - r):
        for j in range(r, n - r):
            d = {(0, 0): p(i, j), (1, 0): k[1] + 2 * k[3] * i + k[4] * j,
                 (0, 1): k[2] + k[4] * i + 2 * k[5] * j,
                 (2, 0): Fraction(2 * k[3], 2), (1, 1): k[4], (0, 2): Fraction(2 * k[5], 2)}
            want = sum(Fraction(d[al]) * mom[al] for al in mom)
            assert out[i, j] == float(want)


def test_star_tap_counts(oracle_mod):
    """Section 3.4: a d-dimensional star of order r has 2rd+1 taps; a box
    has (2r+1)^d."""
    for ndim in (2, 3):
        for r in (1, 2, 3, 4):
            w = 2 * r + 1
            dims = (2 * w + 1,) * ndim
            a = np.zeros(dims)
            a[tuple(d // 2 for d in dims)] = 1.0
            ones = np.ones((w,) * ndim)
            assert np.count_nonzero(oracle_mod.run(a, ones, r, STAR, ZERO, 1)) == 2 * r * ndim + 1
            assert np.count_nonzero(oracle_mod.run(a, ones, r, BOX, ZERO, 1)) == w ** ndim


# ------------------------------------------------------ time loop, windows

def test_steps_compose_and_zero_steps(oracle_mod):
    a = inputs.grid((15, 16), seed=15, dtype=np.float64)
    c = inputs.coefficients(2, 2, BOX, seed=16, dtype=np.float64)
    cur = a
    for _ in range(5):
        cur = oracle_mod.run(cur, c, 2, BOX, PERIODIC, 1)
    assert np.array_equal(cur, oracle_mod.run(a, c, 2, BOX, PERIODIC, 5))
    assert np.array_equal(oracle_mod.run(a, c, 2, BOX, PERIODIC, 0), a)


@pytest.mark.parametrize("bc", [ZERO, PERIODIC])
@pytest.mark.parametrize("ndim", [2, 3])
def test_window_matches_full_run(oracle_mod, bc, ndim):
    dims = (40, 37) if ndim == 2 else (14, 15, 16)
    r, steps = 2, 3
    a = inputs.grid(dims, seed=17, dtype=np.float64)
    c = inputs.coefficients(ndim, r, BOX, seed=18, dtype=np.float64)
    full = oracle_mod.run(a, c, r, BOX, bc, steps)
    size = (5,) * ndim
    for lo in [(0,) * ndim, tuple(d - 5 for d in dims), tuple(d // 2 for d in dims)]:
        got = oracle_mod.window(a, c, r, BOX, bc, steps, lo, size)
        want = full[tuple(slice(lo[d], lo[d] + 5) for d in range(ndim))]
        assert np.array_equal(got, want)


# ------------------------------------------------- sensitivity of the pins

def test_pins_reject_planted_mistakes(oracle_mod):
    """Plausible oracle mistakes -- a transposed C^g, a mirrored C^g
    (convolution instead of correlation) -- are caught by the scipy pin."""
    a = inputs.grid((12, 13), seed=19, dtype=np.float64)
    c = np.random.default_rng(20).uniform(-1, 1, (5, 5))
    want = ndi.correlate(a, c, mode="constant")
    for bad in (c.T, c[::-1, ::-1], c[::-1, :]):
        got = oracle_mod.run(a, bad, 2, BOX, ZERO, 1)
        assert np.abs(got - want).max() > 1e-3
