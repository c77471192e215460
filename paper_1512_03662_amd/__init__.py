"""MI355X-native JFNK implicit step with physics-based preconditioning.

Python face of the C ABI in include/jfnk.h.  PyTorch supplies device memory and the stream;
every step of the solver runs in the library's HIP kernels (libjfnk.so, built in-tree for
gfx950).  There is no CPU path: without the built library or a HIP device the calls raise.

    ctx = Context(problem, precond="sound", jv_mode="fd")
    X = torch.tensor(X0, device="cuda", dtype=torch.float64)
    dt = ctx.cfl_dt(X, cfl=100.0)
    stats = ctx.implicit_step(X, dt)          # X^n -> X^{n+1} in place

Problems are the plain dicts produced by ``workloads.make_problem``.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _native as N

__all__ = ["Context", "ImplicitSteps", "JfnkError", "library_path"]


class JfnkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"jfnk error {code}: {msg}")
        self.code = code


def library_path():
    return N.LIB_PATH


_PC = {"none": N.PC_NONE, "sound": N.PC_SOUND, "sound_thermal": N.PC_SOUND_THERMAL}
_JV = {"fd": N.JV_FD, "exact": N.JV_EXACT}
_PREC = {"fp64": N.FP64, "fp32": N.FP32}
_CHI = {"none": N.CHI_NONE, "const": N.CHI_CONST, "power": N.CHI_POWER}
_BC = {"periodic": N.BC_PERIODIC, "wall": N.BC_WALL}


def _problem_struct(p):
    s = N.Problem()
    nd = int(p["ndim"]) if "ndim" in p else len(p["shape"])
    s.ndim = nd
    for d in range(3):
        s.n[d] = int(p["shape"][d]) if d < nd else 1
        s.dx[d] = float(p["dx"][d]) if d < nd else 1.0
        s.bc[d] = _BC[p["bc"][d]] if d < nd else N.BC_PERIODIC
        g = p.get("g") or (0.0,) * nd
        s.g[d] = float(g[d]) if d < nd else 0.0
        qw = (p.get("qwall") or ((0.0, 0.0),) * nd)
        s.qwall[d][0] = float(qw[d][0]) if d < nd else 0.0
        s.qwall[d][1] = float(qw[d][1]) if d < nd else 0.0
    s.gamma = float(p["gamma"])
    s.chi_model = _CHI[p.get("chi_model", "none")]
    s.chi0 = float(p.get("chi0", 0.0))
    s.chi_tref = float(p.get("chi_tref", 1.0))
    s.chi_exp = float(p.get("chi_exp", 3.0))
    s.theta = float(p.get("theta", 1.0))
    s.a_rad = float(p.get("a_rad", 0.0))
    return s


def _opts_struct(base=None, **kw):
    o = N.Opts()
    N.lib().jfnk_default_opts(C.byref(o))
    if base is not None:
        C.memmove(C.byref(o), C.byref(base), C.sizeof(N.Opts))
    for k, v in kw.items():
        if v is None:
            continue
        if k == "precond":
            v = _PC[v] if isinstance(v, str) else v
        elif k == "jv_mode":
            v = _JV[v] if isinstance(v, str) else v
        elif k == "ell_precision":
            v = _PREC[v] if isinstance(v, str) else v
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Context:
    """One problem on one HIP stream (the current torch stream of ``device`` at creation)."""

    def __init__(self, problem, device="cuda:0", stream=None, **opts):
        self._lib = N.lib()
        self.problem = dict(problem)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the library runs on a HIP device only")
        nd = len(problem["shape"])
        self.nvar = 2 + nd
        self.field_shape = tuple(reversed(tuple(problem["shape"])))
        self.state_shape = (self.nvar,) + self.field_shape
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ps = _problem_struct(problem)
        self._os = _opts_struct(**opts)
        h = C.c_void_p()
        rc = self._lib.jfnk_create(C.byref(self._ps), C.byref(self._os),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != N.OK:
            raise JfnkError(rc, self._lib.jfnk_last_error(None).decode())
        self._h = h

    # ---- helpers ------------------------------------------------------------------------
    def _check(self, rc, allow=()):
        if rc != N.OK and rc not in allow:
            raise JfnkError(rc, self._lib.jfnk_last_error(self._h).decode())
        return rc

    def _vec(self, t, name):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 tensor on {self.device}")
        if tuple(t.shape) != self.state_shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.state_shape}")
        return t

    def _new(self):
        return torch.empty(self.state_shape, dtype=torch.float64, device=self.device)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.jfnk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_opts(self, **opts):
        o = _opts_struct(self._os, **opts)
        self._check(self._lib.jfnk_set_opts(self._h, C.byref(o)))
        self._os = o

    @property
    def opts(self):
        return {k: getattr(self._os, k) for k, _ in N.Opts._fields_}

    def workspace_bytes(self):
        return int(self._lib.jfnk_workspace_bytes(self._h))

    # ---- the ABI --------------------------------------------------------------------------
    def set_state_n(self, Xn, dt):
        self._check(self._lib.jfnk_set_state_n(self._h, _ptr(self._vec(Xn, "Xn")), float(dt)))

    def residual(self, X, out=None):
        out = self._new() if out is None else self._vec(out, "out")
        self._check(self._lib.jfnk_residual(self._h, _ptr(self._vec(X, "X")), _ptr(out)))
        return out

    def jvp(self, X, v, mode="exact", out=None):
        out = self._new() if out is None else self._vec(out, "out")
        m = _JV[mode] if isinstance(mode, str) else int(mode)
        self._check(self._lib.jfnk_jvp(self._h, _ptr(self._vec(X, "X")), _ptr(self._vec(v, "v")),
                                       _ptr(out), m))
        return out

    def vjp(self, X, w, out=None):
        out = self._new() if out is None else self._vec(out, "out")
        self._check(self._lib.jfnk_vjp(self._h, _ptr(self._vec(X, "X")), _ptr(self._vec(w, "w")),
                                       _ptr(out)))
        return out

    def vjp_prev(self, Xn, lam, out=None):
        out = self._new() if out is None else self._vec(out, "out")
        self._check(self._lib.jfnk_vjp_prev(self._h, _ptr(self._vec(Xn, "Xn")),
                                            _ptr(self._vec(lam, "lam")), _ptr(out)))
        return out

    def precond_apply(self, X, r, out=None):
        out = self._new() if out is None else self._vec(out, "out")
        self._check(self._lib.jfnk_precond_apply(self._h, _ptr(self._vec(X, "X")),
                                                 _ptr(self._vec(r, "r")), _ptr(out)))
        return out

    def precond_apply_transpose(self, X, w, out=None):
        out = self._new() if out is None else self._vec(out, "out")
        self._check(self._lib.jfnk_precond_apply_transpose(self._h, _ptr(self._vec(X, "X")),
                                                   _ptr(self._vec(w, "w")), _ptr(out)))
        return out

    def implicit_step(self, X, dt, raise_on_noconv=True):
        st = N.StepStats()
        rc = self._lib.jfnk_implicit_step(self._h, _ptr(self._vec(X, "X")), float(dt), C.byref(st))
        allow = () if raise_on_noconv else (N.E_NEWTON_NOCONV,)
        self._check(rc, allow)
        return st.as_dict()

    def si_step(self, X, dt):
        """One semi-implicit step in place (X^n -> X^{n+1}); returns the step statistics."""
        st = N.StepStats()
        self._check(self._lib.jfnk_si_step(self._h, _ptr(self._vec(X, "X")), float(dt), C.byref(st)))
        return st.as_dict()

    def adjoint_step(self, Xn1, Xn, dt, gbar_n1, out=None):
        out = self._new() if out is None else self._vec(out, "out")
        st = N.StepStats()
        self._check(self._lib.jfnk_adjoint_step(
            self._h, _ptr(self._vec(Xn1, "Xn1")), _ptr(self._vec(Xn, "Xn")), float(dt),
            _ptr(self._vec(gbar_n1, "gbar_n1")), _ptr(out), C.byref(st)))
        return out, st.as_dict()

    def cfl_dt(self, X, cfl):
        dt = self._lib.jfnk_cfl_dt(self._h, _ptr(self._vec(X, "X")), float(cfl))
        if not dt > 0:
            raise JfnkError(N.E_INVALID, self._lib.jfnk_last_error(self._h).decode())
        return dt


class ImplicitSteps(torch.autograd.Function):
    """X^0 -> X^n by n implicit steps with fixed time steps ``dts``.

    Forward keeps every X^k (per-step checkpoints); backward chains the adjoint of each step
    (transposed solve at the converged X^{k+1}).  The time steps are constants: they are
    not differentiated.
    """

    @staticmethod
    def forward(fctx, X0, ctx: Context, dts):
        X = X0.detach().clone()
        states = [X.clone()]
        for dt in dts:
            ctx.implicit_step(X, dt)
            states.append(X.clone())
        fctx.ctx = ctx
        fctx.dts = list(dts)
        fctx.save_for_backward(*states)
        return X.clone()

    @staticmethod
    def backward(fctx, gout):
        ctx = fctx.ctx
        states = fctx.saved_tensors
        g = gout.contiguous().to(torch.float64)
        for k in range(len(fctx.dts) - 1, -1, -1):
            g, _ = ctx.adjoint_step(states[k + 1], states[k], fctx.dts[k], g)
        return g, None, None
