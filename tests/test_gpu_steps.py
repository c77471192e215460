"""GPU parity of whole implicit steps at the configurations' shapes, through the C ABI.

* 3D steps (the z-marching multigrid kernels, 3D residual tiles and FGMRES together): the
  Taylor-Green box at Mach 1e-6 (32^3, periodic, CFL 1000, sound preconditioner) and a
  walled polytrope with chi ~ T^3 (16 x 16 x 32, sound + thermal, CFL 20), each in the plain
  form (FD J.v, FP64 elliptic) and the exact-J.v + FP32-elliptic form, against the root of
  the oracle's own JFNK step iterated far below the step's tolerance (Newton 1e-12, GMRES
  1e-8, CG 1e-8): ||R^-1 (X_gpu - X*)||_inf <= 1e-8 (Sect. 4.1, eq. nr_terminate).
* the first steps of the 2D 256^2 stratified box (constant chi, CFL 100) and of the 512^2
  box with chi ~ T^3 (CFL 50) against the oracle's JFNK step with the same options.
* iteration counts: the same algorithm on both sides, so Newton, GMRES and CG counts agree
  with the oracle's on small 2D cases.
* FP32 elliptic solves against the oracle's FP32 multigrid CG (np.float32 arithmetic) on
  grids whose large levels run the single-level kernels.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.mg import PCGSolver
from oracle.newton import jfnk_step, Opts, Stats
from oracle.pbp import PBP
from oracle.residual import Problem, cfl_dt
from oracle.scaling import scaling_LR

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _lib():
    import paper_1512_03662_amd as J
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return J


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def H(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


TIGHT = dict(newton_tol=1e-12, newton_max=30, gmres_eta=1e-8, gmres_maxit=600, cg_eta=1e-8, cg_maxit=200)

CASES_3D = {
    "taylor_green_32": (lambda: W.taylor_green_3d(n=32), 1000.0, "sound"),
    "polytrope_16x16x32": (lambda: W.polytrope((16, 16, 32), 20.0, mach=1e-4, seed=5, chi_model="power",
                                               cfl=20.0, steps=1), 20.0, "sound_thermal"),
}
_ROOTS = {}


def _tight_root(name):
    """The oracle's root of the first step (cached per case)."""
    if name not in _ROOTS:
        mk, cfl, pc = CASES_3D[name]
        w = mk()
        P = Problem.from_dict(w["problem"])
        dt = cfl_dt(P, w["X0"], cfl)
        st = Stats()
        Xr = jfnk_step(P, w["X0"], dt, Opts(precond=pc, jv_mode="fd", **TIGHT), st)
        assert st.converged and st.dx_norms[-1] < 1e-12, st.dx_norms
        _ROOTS[name] = (w, P, dt, Xr)
    return _ROOTS[name]


@pytest.mark.parametrize("form", ["fd_fp64", "exact_fp32"])
@pytest.mark.parametrize("name", sorted(CASES_3D))
def test_implicit_step_3d(name, form):
    J = _lib()
    w, P, dt, Xr = _tight_root(name)
    jv, ell = form.split("_")
    print(f"# 3D step {name} {form} shape {P.shape}", flush=True)
    ctx = J.Context(w["problem"], precond=CASES_3D[name][2], jv_mode=jv, ell_precision=ell)
    Xg = T(w["X0"])
    assert abs(ctx.cfl_dt(Xg, CASES_3D[name][1]) - dt) <= 1e-14 * dt
    st = ctx.implicit_step(Xg, dt)
    assert st["converged"] == 1, st
    _, R = scaling_LR(P, Xr)
    err = float(np.max(np.abs((H(Xg) - Xr) / R)))
    print(f"#   newton {st['newton_its']} gmres {st['gmres_its']} cg {st['cg_its']} "
          f"||R^-1 (X - X*)||_inf {err:.3e}", flush=True)
    assert err <= 1e-8, (err, st)
    ctx.close()


@pytest.mark.parametrize("cfg", ["stratified_2d", "stratified_2d_kappa"])
def test_first_step_of_the_2d_configs(cfg):
    """256^2 (constant chi, CFL 100) and 512^2 (chi ~ T^3, CFL 50): the first step against
    the oracle's JFNK step with the same options (FD J.v, FP64 MG-CG, Newton 1e-8)."""
    J = _lib()
    w = W.CONFIGS[cfg]()
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, w["cfl"])
    print(f"# first step {w['name']}", flush=True)
    st_o = Stats()
    Xo = jfnk_step(P, X0, dt, Opts(precond=w["precond"], jv_mode=w["jv_mode"]), st_o)
    assert st_o.converged
    ctx = J.Context(w["problem"], precond=w["precond"], jv_mode=w["jv_mode"])
    Xg = T(X0)
    st = ctx.implicit_step(Xg, dt)
    assert st["converged"] == 1
    _, R = scaling_LR(P, Xo)
    err = float(np.max(np.abs((H(Xg) - Xo) / R)))
    print(f"#   oracle newton {st_o.newton_its} gmres {sum(st_o.gmres_its)}; gpu newton "
          f"{st['newton_its']} gmres {st['gmres_its']}; ||R^-1 (X - X_or)||_inf {err:.3e}", flush=True)
    assert err <= 1e-8, err
    ctx.close()


COUNT_CASES = {
    "acoustic_bump_32": (lambda: W.acoustic_bump_2d(n=32), 10.0, "sound", "fd"),
    "polytrope_32_thermal": (lambda: W.polytrope((32, 32), 10.0, mach=1e-3, seed=5, chi_model="power",
                                                 steps=1, cfl=100.0), 100.0, "sound_thermal", "fd"),
    "polytrope_32_exact": (lambda: W.polytrope((32, 32), 10.0, mach=1e-3, seed=5, chi_model="const",
                                               steps=1, cfl=50.0), 50.0, "sound_thermal", "exact"),
    "polytrope_32_thermal_exact": (lambda: W.polytrope((32, 32), 10.0, mach=1e-3, seed=5, chi_model="power",
                                                       steps=1, cfl=100.0), 100.0, "sound_thermal", "exact"),
}


@pytest.mark.parametrize("name", sorted(COUNT_CASES))
def test_iteration_counts_match_the_oracle(name):
    """The GPU runs the oracle's algorithm (Newton, FGMRES(30), MG-CG to 1e-4; the Arnoldi
    vectors are orthogonalised twice on both sides, by CGS2 in the oracle and by its delayed
    form on the GPU, which is the same in exact arithmetic): Newton and GMRES iterations per
    step are the same.  The CG total is the same up to a few
    solves that stop one iteration apart: late Arnoldi vectors amplify rounding differences
    (summation order), and the stopping test ||r|| < eta' ||b|| of a solve that ends near
    the threshold can fall on the other side.  The oracle itself shows this: perturbing X^0
    by 1e-15 relative changes its CG total on the thermal 32^2 case by up to 2 of 1243
    (exact J.v) and 1281 (FD), with Newton and GMRES counts unchanged.  The bar is 0.5 %
    of the CG total."""
    J = _lib()
    mk, cfl, pc, jv = COUNT_CASES[name]
    w = mk()
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], cfl)
    st_o = Stats()
    jfnk_step(P, w["X0"], dt, Opts(precond=pc, jv_mode=jv), st_o)
    ctx = J.Context(w["problem"], precond=pc, jv_mode=jv)
    st = ctx.implicit_step(T(w["X0"]), dt)
    got = (st["newton_its"], st["gmres_its"], st["cg_its"])
    ref = (st_o.newton_its, sum(st_o.gmres_its), sum(st_o.cg_its))
    print(f"# counts {name}: gpu {got} oracle {ref} (per Newton: {st_o.gmres_its})", flush=True)
    assert got[:2] == ref[:2]
    assert abs(got[2] - ref[2]) <= 0.005 * ref[2]
    ctx.close()


@pytest.mark.parametrize("name,m", [("acoustic_bump_32", 1), ("acoustic_bump_32", 3),
                                    ("polytrope_32_thermal", 12), ("polytrope_32_thermal", 70)])
def test_restart_lengths_match_the_oracle(name, m):
    """FGMRES(m) from one Arnoldi step per cycle (no reorthogonalisation at all) to the longest
    restart the library accepts (70 basis vectors: the delayed reorthogonalisation's 140 sums
    per step): Newton and GMRES counts as the oracle's FGMRES(m) with CGS2, CG totals within
    0.5 %, and the step's state within the Newton tolerance of the oracle's."""
    J = _lib()
    mk, cfl, pc, jv = COUNT_CASES[name]
    w = mk()
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], cfl)
    st_o = Stats()
    Xo = jfnk_step(P, w["X0"], dt, Opts(precond=pc, jv_mode=jv, gmres_m=m, gmres_maxit=600), st_o)
    assert st_o.converged
    ctx = J.Context(w["problem"], precond=pc, jv_mode=jv, gmres_m=m, gmres_maxit=600)
    Xg = T(w["X0"])
    st = ctx.implicit_step(Xg, dt)
    got = (st["newton_its"], st["gmres_its"], st["cg_its"])
    ref = (st_o.newton_its, sum(st_o.gmres_its), sum(st_o.cg_its))
    _, R = scaling_LR(P, Xo)
    err = float(np.max(np.abs((H(Xg) - Xo) / R)))
    print(f"# FGMRES({m}) {name}: gpu {got} oracle {ref}; ||R^-1 (X - X_or)||_inf {err:.3e}", flush=True)
    assert got[:2] == ref[:2]
    assert abs(got[2] - ref[2]) <= 0.005 * ref[2]
    assert err <= 1e-8, err
    ctx.close()


@pytest.mark.parametrize("levels,degree", [(1, 2), (2, 2), (0, 1), (0, 3), (2, 3)])
def test_level_cap_step_matches_the_oracle(levels, degree):
    """A whole step with the multigrid hierarchy capped (opts.mg_levels; the oracle's
    max_levels): one level (the 32^2 operator solved densely) or two, and with the smoother's
    degree set (opts.mg_smooth; the oracle's degree).  Newton and GMRES counts as the
    oracle's, CG totals within 0.5 %, state within the Newton tolerance."""
    J = _lib()
    mk, cfl, pc, jv = COUNT_CASES["polytrope_32_thermal"]
    w = mk()
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], cfl)
    st_o = Stats()
    Xo = jfnk_step(P, w["X0"], dt, Opts(precond=pc, jv_mode=jv, mg_levels=levels, mg_smooth=degree), st_o)
    assert st_o.converged
    ctx = J.Context(w["problem"], precond=pc, jv_mode=jv, mg_levels=levels, mg_smooth=degree)
    Xg = T(w["X0"])
    st = ctx.implicit_step(Xg, dt)
    got = (st["newton_its"], st["gmres_its"], st["cg_its"])
    ref = (st_o.newton_its, sum(st_o.gmres_its), sum(st_o.cg_its))
    _, R = scaling_LR(P, Xo)
    err = float(np.max(np.abs((H(Xg) - Xo) / R)))
    print(f"# mg_levels {levels} degree {degree}: gpu {got} oracle {ref}; ||R^-1 (X - X_or)||_inf {err:.3e}",
          flush=True)
    assert got[:2] == ref[:2]
    assert abs(got[2] - ref[2]) <= 0.005 * ref[2]
    assert err <= 1e-8, err
    ctx.close()


@pytest.mark.parametrize("shape,bc", [((1024, 512), ("periodic", "wall")),
                                      ((128, 128, 48), ("periodic", "periodic", "wall"))])
def test_fp32_elliptic_against_the_oracle_fp32_mgcg(shape, bc):
    """FP32 coefficients, vectors and dot products on both sides (the oracle in np.float32,
    right-hand side normalised by its FP64 norm before the cast).  The two FP32 computations
    round differently (summation order), so they agree to FP32 rounding amplified by the CG
    iteration, not to FP64 rounding.  The oracle's FP32 and FP64 multigrid CG take the same
    iteration counts here and differ by at most 2.2e-7 of the largest entry per variable;
    the bar is 5e-6 against both (the solves' own tolerance is 1e-4)."""
    J = _lib()
    nd = len(shape)
    pd, X = W.random_state(shape, bc, seed=16, g=tuple([0.0] * (nd - 1) + [-1.0]), chi_model="power",
                           chi0=0.02, amp=0.2)
    P = Problem.from_dict(pd)
    dt = 0.05
    r = W.random_vector(X, 17)
    ref32 = PBP(P, X, dt, "sound_thermal", solver_factory=PCGSolver.factory(1e-4, 50, np.float32)).apply(r)
    ref64 = PBP(P, X, dt, "sound_thermal", solver_factory=PCGSolver.factory(1e-4, 50)).apply(r)
    ctx = J.Context(pd, precond="sound_thermal", ell_precision="fp32", cg_eta=1e-4, cg_maxit=50)
    ctx.set_state_n(T(X), dt)
    got = H(ctx.precond_apply(T(X), T(r)))
    e32 = [float(np.max(np.abs(got[k] - ref32[k])) / np.max(np.abs(ref32[k]))) for k in range(P.nvar)]
    e64 = [float(np.max(np.abs(got[k] - ref64[k])) / np.max(np.abs(ref64[k]))) for k in range(P.nvar)]
    print(f"# fp32 {shape}: vs oracle fp32 {max(e32):.2e}, vs oracle fp64 {max(e64):.2e}", flush=True)
    assert max(e32) <= 5e-6, e32
    assert max(e64) <= 5e-6, e64
    ctx.close()


@pytest.mark.parametrize("shape,bc,levels,degree", [((256, 128), ("periodic", "wall"), 0, 3),
                                                    ((64, 32, 32), ("periodic", "periodic", "wall"), 2, 1)])
def test_fp32_elliptic_with_multigrid_options(shape, bc, levels, degree):
    """The FP32 elliptic solves with the multigrid options set (smoother degree 3 or 1, which
    run the one-launch-per-step kernels, and a capped hierarchy) against the oracle's FP32
    multigrid CG with the same options, to the bar of the FP32 test above."""
    J = _lib()
    nd = len(shape)
    pd, X = W.random_state(shape, bc, seed=25, g=tuple([0.0] * (nd - 1) + [-1.0]), chi_model="power",
                           chi0=0.02, amp=0.2)
    P = Problem.from_dict(pd)
    dt = 0.05
    r = W.random_vector(X, 26)
    fac = PCGSolver.factory(1e-4, 50, np.float32, max_levels=levels, degree=degree)
    ref32 = PBP(P, X, dt, "sound_thermal", solver_factory=fac).apply(r)
    ctx = J.Context(pd, precond="sound_thermal", ell_precision="fp32", cg_eta=1e-4, cg_maxit=50,
                    mg_levels=levels, mg_smooth=degree)
    ctx.set_state_n(T(X), dt)
    got = H(ctx.precond_apply(T(X), T(r)))
    e32 = [float(np.max(np.abs(got[k] - ref32[k])) / np.max(np.abs(ref32[k]))) for k in range(P.nvar)]
    print(f"# fp32 {shape} levels {levels} degree {degree}: vs oracle fp32 {max(e32):.2e}", flush=True)
    assert max(e32) <= 5e-6, e32
    ctx.close()


def test_phase_timing_of_a_step():
    """opts.phase_timing = 1: the step's residual, J.v, preconditioner and orthogonalisation
    phases get positive GPU times that sum to less than the step's wall time; 0: all zero.
    The result of the step does not change."""
    import time
    J = _lib()
    w = W.polytrope((64, 64), 10.0, mach=1e-3, seed=5, chi_model="power", steps=1, cfl=100.0)
    ctx = J.Context(w["problem"], precond="sound_thermal")
    X0 = T(w["X0"])
    dt = ctx.cfl_dt(X0, 100.0)
    Xa = X0.clone()
    st0 = ctx.implicit_step(Xa, dt)
    assert (st0["t_resid"], st0["t_jv"], st0["t_prec"], st0["t_orth"]) == (0.0, 0.0, 0.0, 0.0)
    ctx.set_opts(phase_timing=1)
    Xb = X0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st1 = ctx.implicit_step(Xb, dt)
    wall_ms = 1e3 * (time.perf_counter() - t0)
    ph = [st1["t_resid"], st1["t_jv"], st1["t_prec"], st1["t_orth"]]
    print(f"# phases (ms) {ph}, wall {wall_ms:.2f}", flush=True)
    assert all(v > 0.0 for v in ph)
    assert sum(ph) <= wall_ms
    assert torch.equal(Xa, Xb)
    assert (st0["newton_its"], st0["gmres_its"], st0["cg_its"]) == (st1["newton_its"], st1["gmres_its"], st1["cg_its"])
    ctx.close()


VORTEX = [(1.0, 0.5), (1e6, 0.5), (1e10, 0.05)]


@pytest.mark.parametrize("t_inf,cfl_adv", VORTEX, ids=[f"Tinf{t:g}_cfladv{c:g}" for t, c in VORTEX])
def test_isentropic_vortex_step(t_inf, cfl_adv):
    """The isentropic vortex of the paper's low-Mach test (64^2, Mach 0.1, 1e-4, 1e-6 for
    T_inf = 1, 1e6, 1e10), one implicit step at the advective CFL number (dt = cfl_adv dx /
    u_inf) with the sound preconditioner and the FD J.v: the GPU against the oracle's JFNK step
    with the same options, state ||R^-1 (X_gpu - X_or)||_inf <= 1e-8 and the same Newton and
    GMRES counts (CG within 0.5 %)."""
    J = _lib()
    w = W.isentropic_vortex_2d(n=64, t_inf=t_inf)
    P = Problem.from_dict(w["problem"])
    dt = cfl_adv * w["problem"]["dx"][0] / 1.0
    print(f"# vortex T_inf {t_inf:g}, CFL_adv {cfl_adv:g}", flush=True)
    st_o = Stats()
    Xo = jfnk_step(P, w["X0"], dt, Opts(precond="sound", jv_mode="fd"), st_o)
    assert st_o.converged
    ctx = J.Context(w["problem"], precond="sound", jv_mode="fd")
    Xg = T(w["X0"])
    st = ctx.implicit_step(Xg, dt)
    assert st["converged"] == 1
    _, R = scaling_LR(P, Xo)
    err = float(np.max(np.abs((H(Xg) - Xo) / R)))
    got = (st["newton_its"], st["gmres_its"], st["cg_its"])
    ref = (st_o.newton_its, sum(st_o.gmres_its), sum(st_o.cg_its))
    print(f"#   gpu {got} oracle {ref}; ||R^-1 (X - X_or)||_inf {err:.3e}", flush=True)
    assert err <= 1e-8, err
    assert got[:2] == ref[:2]
    assert abs(got[2] - ref[2]) <= 0.005 * ref[2]
    ctx.close()


def test_taylor_green_hardest_row_exact_jv():
    """The hardest row of the paper's Taylor-Green timing table (Mach 1e-6, CFL_hydro 4.9e5,
    CFL_adv 0.49; the paper needed 291.5 GMRES iterations per Newton iteration) at 32^3 with
    the exact forward-mode J.v: one step against the oracle's JFNK step with the same options
    (complex-step J.v), ||R^-1 (X_gpu - X_or)||_inf <= 1e-8, the same Newton and GMRES counts
    (CG within 0.5 %), and pressure stays positive.  With the finite-difference product this
    row's first linear solve sits at the edge of convergence (see the study in the docs)."""
    J = _lib()
    w = W.taylor_green_3d(n=32, mach=1e-6, noise=0.0)
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], 4.9e5)
    st_o = Stats()
    Xo = jfnk_step(P, w["X0"], dt, Opts(precond="sound", jv_mode="exact"), st_o)
    assert st_o.converged
    ctx = J.Context(w["problem"], precond="sound", jv_mode="exact")
    Xg = T(w["X0"])
    st = ctx.implicit_step(Xg, dt)
    assert st["converged"] == 1
    _, R = scaling_LR(P, Xo)
    X1 = H(Xg)
    err = float(np.max(np.abs((X1 - Xo) / R)))
    got = (st["newton_its"], st["gmres_its"], st["cg_its"])
    ref = (st_o.newton_its, sum(st_o.gmres_its), sum(st_o.cg_its))
    print(f"# hardest TGV row 32^3 exact J.v: gpu {got} oracle {ref}; ||R^-1 (X - X_or)||_inf {err:.3e}", flush=True)
    assert err <= 1e-8, err
    assert got[:2] == ref[:2]
    assert abs(got[2] - ref[2]) <= 0.005 * ref[2]
    assert np.min((w["problem"]["gamma"] - 1.0) * X1[0] * X1[1]) > 0.0
    ctx.close()


ODD = [((65, 65), ("periodic", "wall")), ((130, 130), ("periodic", "wall")),
       ((17, 16, 17), ("periodic", "periodic", "wall"))]


@pytest.mark.parametrize("shape,bc", ODD, ids=["x".join(map(str, s)) for s, _ in ODD])
def test_precond_with_smoothed_bottom_level(shape, bc):
    """Grids whose coarsest multigrid level is too large for the dense inverse (an odd axis
    stops the coarsening: 65^2 and 17 x 16 x 17 have one level, 130^2 two): that level is
    smoothed instead of solved, on both sides; the preconditioner (MG-CG to 1e-4) and its
    transpose against the oracle's, 1e-9 of the largest entry per variable."""
    J = _lib()
    nd = len(shape)
    pd, X = W.random_state(shape, bc, seed=41, g=tuple([0.0] * (nd - 1) + [-1.0]), chi_model="power",
                           chi0=0.02, amp=0.2)
    P = Problem.from_dict(pd)
    dt = 0.05
    r = W.random_vector(X, 42)
    pbp = PBP(P, X, dt, "sound_thermal", solver_factory=PCGSolver.factory(1e-4))
    assert pbp.solve_p.mg.coarse_chol is None
    ctx = J.Context(pd, precond="sound_thermal")
    ctx.set_state_n(T(X), dt)
    ref, got = pbp.apply(r), H(ctx.precond_apply(T(X), T(r)))
    refT, gotT = pbp.apply_T(r), H(ctx.precond_apply_transpose(T(X), T(r)))
    for k in range(P.nvar):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-9 * np.max(np.abs(ref[k])), k
        assert np.max(np.abs(gotT[k] - refT[k])) <= 1e-9 * np.max(np.abs(refT[k])), k
    ctx.close()


def test_implicit_step_with_smoothed_bottom_level():
    """A 65^2 polytrope (one multigrid level, smoothed): the step against the oracle's JFNK
    step with the same options, and the same Newton and GMRES counts (CG within 0.5 %)."""
    J = _lib()
    w = W.polytrope((65, 65), 10.0, mach=1e-3, seed=5, chi_model="power", steps=1, cfl=100.0)
    P = Problem.from_dict(w["problem"])
    dt = cfl_dt(P, w["X0"], 100.0)
    st_o = Stats()
    Xo = jfnk_step(P, w["X0"], dt, Opts(precond="sound_thermal", jv_mode="fd"), st_o)
    ctx = J.Context(w["problem"], precond="sound_thermal")
    Xg = T(w["X0"])
    st = ctx.implicit_step(Xg, dt)
    _, R = scaling_LR(P, Xo)
    err = float(np.max(np.abs((H(Xg) - Xo) / R)))
    got = (st["newton_its"], st["gmres_its"], st["cg_its"])
    ref = (st_o.newton_its, sum(st_o.gmres_its), sum(st_o.cg_its))
    print(f"# 65^2 smoothed bottom: gpu {got} oracle {ref}; ||R^-1 (X - X_or)||_inf {err:.3e}", flush=True)
    assert st["converged"] == 1 and err <= 1e-8, err
    assert got[:2] == ref[:2]
    assert abs(got[2] - ref[2]) <= 0.005 * ref[2]
    ctx.close()


def test_red_giant_grid_shape_steps():
    """The grid shape of the paper's 3D red-giant run (72 x 65 x 65, Sect. 5.2) can be created
    (odd axes: one multigrid level, smoothed) and a step of a polytrope on it converges."""
    J = _lib()
    w = W.polytrope((72, 65, 65), 20.0, mach=1e-4, seed=5, chi_model="power", steps=1, cfl=50.0)
    ctx = J.Context(w["problem"], precond="sound_thermal")
    Xg = T(w["X0"])
    dt = ctx.cfl_dt(Xg, 50.0)
    st = ctx.implicit_step(Xg, dt)
    print(f"# 72x65x65: newton {st['newton_its']} gmres {st['gmres_its']} cg {st['cg_its']}", flush=True)
    assert st["converged"] == 1
    assert torch.isfinite(Xg).all() and float(Xg[0].min()) > 0.0
    ctx.close()
