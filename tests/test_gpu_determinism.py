"""Run-to-run reproducibility of the GPU path: the same inputs give bitwise the same outputs.

Nothing on the path uses atomics (J^T w is a gather, every reduction writes one partial per
block and sums them in a fixed order), and the host's decisions (Newton and GMRES stopping,
Givens rotations) follow from those sums alone.  The CG loop's batch size adapts to the
previous solve's iteration count, which changes how far ahead the host enqueues V-cycles
but not what the device computes: a second step in the same context, with different
batches, must give the same bits as the first and as a fresh context.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.residual import Problem, cfl_dt

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _lib():
    import paper_1512_03662_amd as J
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return J


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _same_bits(a, b):
    torch.cuda.synchronize()
    return torch.equal(a.view(torch.int64), b.view(torch.int64))


COUNTS = ("converged", "newton_its", "gmres_its", "cg_its")


@pytest.mark.parametrize("form", ["fd_fp64", "exact_fp32"])
def test_implicit_step_is_bitwise_reproducible(form):
    """64^3 convective box (chi ~ T^3, sound + thermal, CFL 50): the z-marching multigrid
    kernels, the 3D residual tiles, delayed CGS2 over 64^3 x 5 unknowns."""
    J = _lib()
    w = W.convective_box_3d(n=64, steps=1)
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], 50.0)
    jv, ell = form.split("_")
    print(f"# reproducible step {w['name']} {form}", flush=True)
    opts = dict(precond=w["precond"], jv_mode=jv, ell_precision=ell)
    ctx = J.Context(w["problem"], **opts)
    X0 = T(w["X0"])
    outs, stats = [], []
    for _ in range(2):                      # the same context twice (adapted CG batches)
        X = X0.clone()
        stats.append(ctx.implicit_step(X, dt))
        outs.append(X)
    ctx.close()
    ctx2 = J.Context(w["problem"], **opts)  # a fresh context
    X = X0.clone()
    stats.append(ctx2.implicit_step(X, dt))
    outs.append(X)
    ctx2.close()
    print(f"#   newton {stats[0]['newton_its']} gmres {stats[0]['gmres_its']} cg {stats[0]['cg_its']}",
          flush=True)
    assert stats[0]["converged"] == 1
    for s in stats[1:]:
        assert all(s[k] == stats[0][k] for k in COUNTS), (s, stats[0])
    assert not _same_bits(outs[0], X0)
    for o in outs[1:]:
        assert _same_bits(o, outs[0])


def test_products_and_adjoint_step_are_bitwise_reproducible():
    """F, both J.v forms, J^T w and a whole adjoint step on a 32^3 walled polytrope with
    chi ~ T^3, each evaluated twice."""
    J = _lib()
    w = W.polytrope((32, 32, 32), 20.0, mach=1e-4, seed=5, chi_model="power", cfl=20.0, steps=1)
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], 20.0)
    print("# reproducible products and adjoint step 32^3", flush=True)
    ctx = J.Context(w["problem"], precond="sound_thermal", jv_mode="fd")
    X0 = T(w["X0"])
    rng = np.random.default_rng(11)
    V = T(rng.standard_normal(X0.shape))
    ctx.set_state_n(X0, dt)
    X1 = X0.clone()
    assert ctx.implicit_step(X1, dt)["converged"] == 1
    calls = {
        "residual": lambda: ctx.residual(X1),
        "jvp_exact": lambda: ctx.jvp(X1, V, mode="exact"),
        "jvp_fd": lambda: ctx.jvp(X1, V, mode="fd"),
        "vjp": lambda: ctx.vjp(X1, V),
        "adjoint_step": lambda: ctx.adjoint_step(X1, X0, dt, V)[0],
    }
    for name, f in calls.items():
        a, b = f(), f()
        assert torch.isfinite(a).all(), name
        assert _same_bits(a, b), name
    ctx.close()
