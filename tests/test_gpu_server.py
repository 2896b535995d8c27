"""GPU tests of the serving loop: requests of mixed kinds and sizes, admitted
into a small arena as room frees up, advanced together tick by tick; each
result must equal (bitwise) the same descriptor run alone through a plan,
and match the CPU FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2310_16298_amd import inputs
from paper_2310_16298_amd import stencil as st

from gpu_helpers import eff_coeffs, error_bound, torch_cuda

pytestmark = pytest.mark.gpu

BF = st.PATH_MFMA_BF16X3

SPECS = [  # dims, r, shape, bc, dtype, path, steps
    ((64, 64), 1, st.BOX, st.BC_ZERO, st.F32, st.PATH_AUTO, 5),
    ((100, 77), 2, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_MFMA, 3),
    ((33, 45, 64), 1, st.STAR, st.BC_ZERO, st.F32, st.PATH_AUTO, 7),
    ((128, 96), 3, st.STAR, st.BC_ZERO, st.F64, st.PATH_MFMA, 1),
    ((20, 20, 20), 2, st.BOX, st.BC_PERIODIC, st.F64, st.PATH_GATHER, 4),
    ((300, 256), 4, st.BOX, st.BC_ZERO, st.F32, st.PATH_AUTO, 6),
    ((64, 200), 1, st.BOX, st.BC_PERIODIC, st.F32, BF, 2),
    ((17, 40, 70), 3, st.STAR, st.BC_PERIODIC, st.F32, st.PATH_MFMA, 5),
    ((48, 48), 2, st.STAR, st.BC_ZERO, st.F64, st.PATH_GATHER, 0),
    ((9, 9), 1, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_GATHER, 9),
    ((40, 24, 32), 4, st.STAR, st.BC_ZERO, st.F32, BF, 3),
    ((256, 64), 2, st.BOX, st.BC_ZERO, st.F32, st.PATH_MFMA, 8),
    ((64, 64), 2, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_AUTO, 137),  # many launches per tick
    ((24, 40, 48), 1, st.STAR, st.BC_ZERO, st.F64, st.PATH_GATHER, 70),
    ((512, 512), 1, st.STAR, st.BC_PERIODIC, st.F32, st.PATH_MFMA, 65),
    ((12, 26, 64), 4, st.BOX, st.BC_PERIODIC, st.F32, st.PATH_AUTO, 3),
    ((130, 264), 4, st.GENERAL, st.BC_PERIODIC, st.F32, st.PATH_GATHER, 4),  # nonzero-tap gather
    ((70, 132), 2, st.GENERAL, st.BC_ZERO, st.F64, st.PATH_AUTO, 3),
]


def _inputs(k, spec):
    dims, r, shape, bc, dt, path, steps = spec
    if shape == st.GENERAL:  # both diagonals with random weights
        w = 2 * r + 1
        m = np.eye(w, dtype=bool) | np.eye(w, dtype=bool)[::-1]
        c = np.where(m, np.random.default_rng(9700 + 10 * k).uniform(0.02, 0.1, (w, w)), 0.0)
    else:
        c = inputs.coefficients(len(dims), r, shape, seed=9700 + 10 * k, dtype=np.float64)
    a0 = inputs.grid(dims, seed=9701 + 10 * k, dtype=np.float64 if dt == st.F64 else np.float32)
    return c, a0


def _alone(torch, spec, c, a0):
    dims, r, shape, bc, dt, path, steps = spec
    plan = st.Plan(dims, r, shape, c, boundary=bc, dtype=dt, path=path)
    x = torch.from_numpy(a0).cuda()
    res = plan.run_steps(x, torch.empty_like(x), steps) if steps else x
    torch.cuda.synchronize()
    out = res.cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("arena_mib,max_active", [(4, 0), (64, 0), (64, 1), (64, 3)])
def test_server_results_equal_alone(arena_mib, max_active):
    torch = torch_cuda()
    srv = st.Server(arena_mib << 20, max_active=max_active, max_inflight_ticks=3)
    stream = srv.stream()
    data = [_inputs(k, spec) for k, spec in enumerate(SPECS)]
    outs, ids = {}, {}
    pending = list(range(len(SPECS)))
    done = set()
    ticks = 0
    while len(done) < len(SPECS):
        # submit two requests per tick while any remain: arrivals during the run
        for _ in range(2):
            if pending:
                k = pending.pop(0)
                dims, r, shape, bc, dt, path, steps = SPECS[k]
                c, a0 = data[k]
                with torch.cuda.stream(stream):
                    x = torch.from_numpy(a0).to("cuda", non_blocking=False)
                    out = torch.empty_like(x)
                torch.cuda.synchronize()
                rid = srv.submit(x, out, steps, r, shape, c, boundary=bc, path=path)
                ids[rid] = k
                outs[k] = out
        stats = srv.tick()
        ticks += 1
        if max_active:
            assert stats["active"] <= max_active
        assert stats["arena_in_use"] <= arena_mib << 20
        for rid in srv.poll():
            assert rid not in done
            done.add(rid)
        assert ticks < 10000
    torch.cuda.synchronize()
    assert sorted(done) == sorted(ids)
    for rid, k in ids.items():
        c, a0 = data[k]
        got = outs[k].cpu().numpy()
        assert np.array_equal(got, _alone(torch, SPECS[k], c, a0)), f"request {k} {SPECS[k]}"
    for k in (0, 2, 4, 9, 12, 13, 15, 16):
        dims, r, shape, bc, dt, path, steps = SPECS[k]
        c, a0 = data[k]
        ce = eff_coeffs(c, dt)
        shape = st.BOX if shape == st.GENERAL else shape  # the oracle sums every tap
        want = oracle.run(a0.astype(np.float64), ce, r, shape, bc, steps)
        tol = error_bound(ce, len(dims), r, shape, dt, path, steps, np.abs(a0).max())
        assert np.abs(outs[k].cpu().numpy().astype(np.float64) - want).max() <= tol
    srv.close()


def test_server_rejects():
    torch = torch_cuda()
    srv = st.Server(1 << 20)
    c = inputs.coefficients(2, 1, st.BOX, seed=1, dtype=np.float64)
    big = torch.zeros(1024, 1024, device="cuda")
    with pytest.raises(st.StencilError) as e:  # two 4 MiB grids never fit a 1 MiB arena
        srv.submit(big, torch.empty_like(big), 1, 1, st.BOX, c)
    assert e.value.status == st.ENOMEM
    x = torch.zeros(64, 64, device="cuda")
    with pytest.raises(st.StencilError) as e:
        srv.submit(x, x, 1, 1, st.BOX, c)
    assert e.value.status == st.EALIAS
    d, keep = st.make_desc((64, 64), 1, st.BOX, c, time_block=2)
    assert srv._lib.stencil_server_submit(srv._h, d, x.data_ptr(), big.data_ptr(), 1, None) == st.EUNSUPPORTED
    srv.close()


def test_server_cancel_isolates_the_rest():
    """Requests withdrawn while queued or resident are never reported and
    never write their outputs; every other request still equals its run
    alone bit for bit, and the arena empties."""
    torch = torch_cuda()
    picks = [0, 2, 5, 7, 11, 12, 13, 14]  # mixed 2D / 3D, FP32 / FP64, short and long runs
    data = {k: _inputs(k, SPECS[k]) for k in picks}
    srv = st.Server(96 << 20, max_active=3)
    ids, outs = {}, {}
    for k in picks:
        dims, r, shape, bc, dt, path, steps = SPECS[k]
        c, a0 = data[k]
        x = torch.from_numpy(a0).cuda()
        out = torch.full_like(x, 7.0)  # sentinel: a cancelled request's output stays untouched
        torch.cuda.synchronize()
        ids[srv.submit(x, out, steps, r, shape, c, boundary=bc, path=path)] = k
        outs[k] = out
    rids = list(ids)
    cancelled = {rids[7]}  # still queued behind max_active = 3
    srv.cancel(rids[7])
    srv.tick()
    st_ = srv.tick()
    assert st_["active"] >= 1
    srv.cancel(rids[5])  # the 64^2 request of 137 steps: resident or queued by now
    cancelled.add(rids[5])
    with pytest.raises(st.StencilError) as e:
        srv.cancel(rids[5])
    assert e.value.status == st.EINVAL
    with pytest.raises(st.StencilError) as e:
        srv.cancel(10_000)
    assert e.value.status == st.EINVAL
    done, ticks = set(), 0
    while len(done) < len(rids) - len(cancelled):
        stats = srv.tick()
        ticks += 1
        for rid in srv.poll():
            assert rid not in cancelled and rid not in done
            done.add(rid)
        assert ticks < 10000
    torch.cuda.synchronize()
    assert stats["arena_in_use"] == 0 and stats["active"] == 0 and stats["queued"] == 0
    for rid, k in ids.items():
        got = outs[k].cpu().numpy()
        if rid in cancelled:
            assert np.all(got == 7.0), f"cancelled request {k} wrote its output"
        else:
            c, a0 = data[k]
            assert np.array_equal(got, _alone(torch, SPECS[k], c, a0)), f"request {k} {SPECS[k]}"
    srv.close()
