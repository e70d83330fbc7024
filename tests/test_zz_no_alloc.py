"""gq_eval_noalloc (the evaluation whose workspace lives in the library's fixed device scratch)
against gq_eval through the C ABI: bitwise equal outputs on two calls in a row, the second with a
smaller input (fewer densities on a smaller geometry), for every kind; a request beyond the
scratch is refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import gq_inputs as gi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _ctx(g, **kw):
    from paper_1801_04070_amd import QBXFMM
    q = QBXFMM(device=0)
    q.set_geometry_from(g)
    q.build(**kw)
    return q


def _call(q, fn, kind, d1, d2, out):
    st = fn(q._h, kind, d1.shape[0], d1.data_ptr(), d1.stride(0),
            None if d2 is None else d2.data_ptr(), 0 if d2 is None else d2.stride(0),
            out.data_ptr(), out.stride(0))
    return st


@pytest.mark.parametrize("kind", [1, 2, 3, 4])
def test_noalloc_matches_eval_two_calls(kind):
    from paper_1801_04070_amd import library
    L = library()
    big = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    small = gi.starfish_c1()
    cases = []
    for g, nd, p in ((big, 3, dict(p_qbx=12, p_fmm=30)), (small, 1, dict(p_qbx=8, p_fmm=20))):
        q = _ctx(g, **p)
        d1 = _dev(np.stack([gi.fourier_density(g, seed=s) for s in range(nd)]))
        d2 = _dev(np.stack([gi.fourier_density(g, seed=50 + s) for s in range(nd)])) \
            if kind == 3 else None
        rows = nd * (2 if kind == 4 else 1)
        cases.append((q, d1, d2, rows, g.n_tgt))
    # no-alloc calls first (a fresh scratch), then the allocating ones
    got = []
    for q, d1, d2, rows, nt in cases:
        out = torch.full((rows, nt), float("nan"), dtype=torch.float64, device="cuda:0")
        assert _call(q, L.gq_eval_noalloc, kind, d1, d2, out) == 0, q._L.gq_last_error(q._h)
        torch.cuda.synchronize()
        got.append(out.cpu().numpy())
    for (q, d1, d2, rows, nt), g_out in zip(cases, got):
        out = torch.empty((rows, nt), dtype=torch.float64, device="cuda:0")
        assert _call(q, L.gq_eval, kind, d1, d2, out) == 0
        torch.cuda.synchronize()
        ref = out.cpu().numpy()
        assert np.isfinite(g_out).all()
        assert np.array_equal(g_out, ref)
    # and again after the allocating calls, still bitwise equal
    q, d1, d2, rows, nt = cases[1]
    out = torch.empty((rows, nt), dtype=torch.float64, device="cuda:0")
    assert _call(q, L.gq_eval_noalloc, kind, d1, d2, out) == 0
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), got[1])


def test_noalloc_refuses_beyond_scratch():
    from paper_1801_04070_amd import GQ_S_AND_D, _lib, library
    L = library()
    g = gi.config_geometry("c2")
    q = _ctx(g, p_qbx=12, p_fmm=30)
    d1 = _dev(np.stack([gi.fourier_density(g, seed=s) for s in range(8)]))
    out = torch.full((16, g.n_tgt), 7.0, dtype=torch.float64, device="cuda:0")
    st = _call(q, L.gq_eval_noalloc, GQ_S_AND_D, d1, None, out)
    assert st == _lib.GQ_EINVAL
    assert b"scratch" in q._L.gq_last_error(q._h)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 7.0).all()
    # one density of both kinds fits
    one = torch.empty((2, g.n_tgt), dtype=torch.float64, device="cuda:0")
    assert _call(q, L.gq_eval_noalloc, GQ_S_AND_D, d1[:1], None, one) == 0
    ref = q.eval(GQ_S_AND_D, d1[:1]).cpu().numpy()
    assert np.array_equal(one.cpu().numpy(), ref)
