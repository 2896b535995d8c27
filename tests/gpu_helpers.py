"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
bound the rounding error against the FP64 oracle.

Error bound (elementwise, absolute) for T steps of a stencil with m taps,
coefficient magnitudes summing to S and initial magnitude A = max|a0|:
each step's sum of m products has error <= gamma_m * S * max|a_t| (Higham),
the stored result adds u * max|a_{t+1}|, split operands add eps_p * S *
max|a_t| per step, and max|a_t| <= S^t A.  Summed over the steps:
    |gpu - oracle| <= T * (gamma_m + u + eps_p) * max(S, 1)^T * A.
u = 2^-24 (FP32 storage) or 2^-53 (FP64); gamma_m = m u / (1 - m u) with the
accumulation precision; eps_p = 3 * 2^-16 (BF16 hi/lo), 3 * 2^-22 (FP16
hi/lo), 0 otherwise.  A factor 2 of slack covers the bound's own rounding.
"""
import numpy as np

from paper_2310_16298_amd import stencil as st


def torch_cuda():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    st.load_library()  # fail loudly if the HIP library is missing
    return torch


def eff_coeffs(c, dtype):
    return c.astype(np.float32).astype(np.float64) if dtype == st.F32 else c.astype(np.float64)


def tap_count(ndim, r, shape):
    return (2 * r + 1) ** ndim if shape == st.BOX else 2 * r * ndim + 1


def error_bound(c_eff, ndim, r, shape, dtype, path, steps, amax):
    m = tap_count(ndim, r, shape)
    u = 2.0 ** -53 if dtype == st.F64 else 2.0 ** -24
    gamma = m * u / (1 - m * u)
    eps_p = {st.PATH_MFMA_BF16X3: 3 * 2.0 ** -16, st.PATH_MFMA_F16X3: 3 * 2.0 ** -22}.get(path, 0.0)
    if eps_p:
        gamma = 3 * m * u / (1 - 3 * m * u)
    s = max(float(np.abs(c_eff).sum()), 1.0)
    return 2.0 * steps * (gamma + u + eps_p) * s ** steps * amax + 1e-300


def run_gpu(a0, coeffs, radius, shape, bc, dtype, path, steps, lines=st.LINES_AUTO, check_info=True, **plan_kw):
    """Final state after `steps` Jacobi steps on the GPU (numpy FP64);
    plan_kw: further Plan knobs (block_n, chunk, ...)."""
    torch = torch_cuda()
    tdt = torch.float64 if dtype == st.F64 else torch.float32
    ndt = np.float64 if dtype == st.F64 else np.float32
    x = torch.from_numpy(np.ascontiguousarray(a0, dtype=ndt)).cuda()
    tmp = torch.empty_like(x)
    plan = st.Plan(a0.shape, radius, shape, coeffs, boundary=bc, dtype=dtype, path=path, lines=lines, **plan_kw)
    if check_info and path != st.PATH_AUTO:
        assert plan.info["path"] == path
    res = plan.run_steps(x, tmp, steps)
    torch.cuda.synchronize()
    out = res.cpu().numpy().astype(np.float64)
    plan.close()
    assert tdt == x.dtype
    return out
