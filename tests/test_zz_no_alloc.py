"""The allocation-free CFL time step (jfnk_cfl_dt_noalloc) through the C ABI against the
context's jfnk_cfl_dt: bit for bit, on two calls in a row (the second on a smaller grid, so
the static scratch holds the first call's partials when it starts), plus its host-side
refusals."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _call(J, N, pd, X, cfl, out, stream):
    ps = J._problem_struct(pd)
    return N.lib().jfnk_cfl_dt_noalloc(C.byref(ps), C.c_void_p(X.data_ptr()), float(cfl),
                                       C.c_void_p(out.data_ptr()), C.c_void_p(stream.cuda_stream))


def test_noalloc_cfl_dt_matches_the_context_call():
    import paper_1512_03662_amd as J
    from paper_1512_03662_amd import _native as N
    assert torch.cuda.is_available()
    cases = [
        (W.polytrope((48, 40, 36), 20.0, mach=1e-2, seed=3, chi_model="power", steps=1, cfl=500.0), 500.0),
        (W.acoustic_bump_2d(n=24), 10.0),
    ]
    stream = torch.cuda.current_stream()
    for w, cfl in cases:
        pd = w["problem"]
        X = torch.tensor(w["X0"], dtype=torch.float64, device="cuda:0")
        if len(pd["shape"]) == 2:   # give the 2D pulse a velocity field as well
            X[2:] = torch.tensor(W.random_vector(w["X0"][2:], 5, amp=0.1), dtype=torch.float64, device="cuda:0")
        print(f"# noalloc cfl_dt {w['name']}", flush=True)
        ctx = J.Context(pd)
        ref = ctx.cfl_dt(X, cfl)
        out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
        assert _call(J, N, pd, X, cfl, out, stream) == N.OK, N.lib().jfnk_last_error(None)
        torch.cuda.synchronize()
        got = float(out.cpu()[0])
        assert got == ref, (got, ref)
        ctx.close()


def test_noalloc_cfl_dt_refusals_on_the_host():
    import paper_1512_03662_amd as J
    from paper_1512_03662_amd import _native as N
    w = W.acoustic_bump_2d(n=16)
    X = torch.tensor(w["X0"], dtype=torch.float64, device="cuda:0")
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    L = N.lib()
    ps = J._problem_struct(w["problem"])
    assert L.jfnk_cfl_dt_noalloc(C.byref(ps), None, 1.0, C.c_void_p(out.data_ptr()), None) == N.E_INVALID
    assert L.jfnk_cfl_dt_noalloc(C.byref(ps), C.c_void_p(X.data_ptr()), 0.0, C.c_void_p(out.data_ptr()),
                                 None) == N.E_INVALID
    bad = dict(w["problem"])
    bad["shape"] = (3, 16)
    pb = J._problem_struct(bad)
    assert L.jfnk_cfl_dt_noalloc(C.byref(pb), C.c_void_p(X.data_ptr()), 1.0, C.c_void_p(out.data_ptr()),
                                 None) == N.E_INVALID
    assert b"4 cells" in L.jfnk_last_error(None)
