"""GPU parity with the oracle at the stated step counts (needs an MI355X; slow).

- The accuracy workload: the density wave on the hybrid lattice at N = 8 and 16, to t = 0.1 (the
  paper's accuracy test, scaled to the unit cube).
- The benchmark's physics: the Taylor-Green vortex at Mach 0.1, mu = 1/1600, Pr = 0.72, on the
  hybrid lattice of [0, 2 pi]^3 at N = 16, 200 steps.
- The reconstruction at N = 32 (183,982 cells): the GPU's quadratics against the oracle's Eq. weno
  at sampled cells and points.

Both sides take the oracle's step sizes.  FP64 bar: relative L-infinity per component <= 1e-12 (the
three momentum components share the scale max |rho U|).  The FP32-mixed path's L1 (the integral of
|dQ| over the domain) and relative L-infinity against the same oracle runs are printed and bounded.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2203_09047_amd import inputs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-12


@pytest.fixture(scope="module")
def gks():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2203_09047_amd import gks as g

    g.load()
    return g


def _errors(got, ref, vol):
    scale = np.abs(ref).max(axis=1)
    scale[1:4] = scale[1:4].max()
    linf = np.abs(got - ref).max(axis=1) / scale
    l1 = (np.abs(got - ref) * vol).sum(axis=1)
    return linf, l1


def _march(gks, mesh, Q0, dts, kw, precision, report_every, min_big=0):
    """GPU steps of the given sizes: the states (mesh order) at the report steps and the last."""
    import torch

    host = gks.HostMesh(mesh, min_big=min_big)
    sol = gks.Solver(host, gks.params(precision=precision, **kw))
    Q = sol.upload(host.to_internal(Q0))
    snaps = {}
    for k, dt in enumerate(dts, 1):
        sol.step(Q, dt)
        if k % report_every == 0 or k == len(dts):
            sol.poll()
            torch.cuda.synchronize()
            snaps[k] = host.to_external(Q.cpu().numpy())
    return snaps


def _oracle_march(o, Q0, report_every, nsteps=0, t_end=0.0):
    """The oracle's run with its CFL step sizes (the last one shortened to land on t_end): the step
    sizes and the states at the report steps."""
    ref, snaps, dts, t = Q0.copy(), {}, [], 0.0
    while (t < t_end * (1 - 1e-14)) if t_end > 0 else (len(dts) < nsteps):
        dt = o.timestep(ref)
        if t_end > 0 and t + dt > t_end:
            dt = t_end - t
        ref = o.step(ref, dt)
        dts.append(dt)
        t += dt
        if len(dts) % report_every == 0:
            snaps[len(dts)] = ref.copy()
    snaps[len(dts)] = ref
    return dts, snaps


def _check(gks, mesh, Q0, kw, every, fp32_bound, nsteps=0, t_end=0.0, min_big=0):
    o = oracle.Oracle(mesh, oracle.params(**kw), min_big=min_big)
    vol = o.cell_geometry()[0]
    dts, ref = _oracle_march(o, Q0, every, nsteps, t_end)
    print(f"{len(dts)} steps", flush=True)
    got = _march(gks, mesh, Q0, dts, kw, 0, every, min_big)
    hist = {}
    for k in sorted(ref):
        hist[k], _ = _errors(got[k], ref[k], vol)
        print(f"FP64 step {k}: relative Linf {hist[k]}", flush=True)
    last = max(ref)
    g32 = _march(gks, mesh, Q0, dts, kw, 1, len(dts), min_big)
    linf32, l132 = _errors(g32[last], ref[last], vol)
    print(f"FP32-mixed after {last} steps: relative Linf {linf32}, L1 {l132}", flush=True)
    assert (linf32 <= fp32_bound).all(), linf32
    return hist, linf32, l132


@pytest.mark.parametrize("N", [8, 16])
def test_density_wave_hybrid_to_t_01(gks, N):
    print(f"case: density wave hybrid N={N} to t=0.1", flush=True)
    mesh = inputs.lattice(N, "hybrid")
    Q0 = inputs.cell_averages(mesh, inputs.wave())
    hist, _, _ = _check(gks, mesh, Q0, {}, 10, 1e-3, t_end=0.1)
    assert (hist[max(hist)] <= TOL).all()


@pytest.mark.parametrize("min_big", [16, 0])
def test_taylor_green_navier_stokes_hybrid_200_steps(gks, min_big):
    """CFL 0.3: at 0.5 the explicit step leaves the physical states on every lattice (pure hexahedra
    included) by step 100 of this acoustic flow.

    With 16-member big stencils the linearised scheme is stable and the FP64 difference stays within
    1e-12 over all 200 steps.  With the paper's stencils the linearised scheme has growing modes (on
    tetrahedra with 12-14 member stencils, see the tangent's power iteration in the CPU tests); the
    nonlinear weights keep the solution bounded, but rounding differences between two
    implementations are amplified: the bar holds over the first 40 steps, the difference peaks
    near it around steps 50-60 (1.2e-12 to 1.6e-12) and then grows by at most 3 % per step on
    average (measured: about 2 %)."""
    print(f"case: Taylor-Green NS hybrid N=16, 200 steps, CFL 0.3, min_big={min_big}", flush=True)
    kw = dict(viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=0.3)
    mesh = inputs.lattice(16, "hybrid", box=(2 * math.pi,) * 3)
    Q0 = inputs.cell_averages(mesh, inputs.tgv())
    hist, _, _ = _check(gks, mesh, Q0, kw, 10, 1e-2, nsteps=200, min_big=min_big)
    if min_big:
        assert all((h <= TOL).all() for h in hist.values())
    else:
        assert all((hist[k] <= TOL).all() for k in hist if k <= 40)
        assert hist[200].max() <= hist[40].max() * 1.03 ** 160, (hist[40], hist[200])


def _poly_eval(c, X):
    """Value [5] and gradient [5, 3] of the per-cell quadratics c [5, 10] at the offset X."""
    x, y, z = X
    mono = np.array([1, x, y, z, x * x, x * y, x * z, y * y, y * z, z * z])
    dmono = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [2 * x, 0, 0], [y, x, 0], [z, 0, x],
                      [0, 2 * y, 0], [0, z, y], [0, 0, 2 * z]])
    return c @ mono, c @ dmono


def test_reconstruction_at_n32_sampled_cells(gks):
    """K1 at 183,982 cells (Taylor-Green Mach 0.1, the benchmark's field): 2000 sampled cells, the
    GPU's quadratic against the oracle's Eq. weno at a random point of each, value to 1e-12 of the
    component's scale and gradient to 1e-10."""
    import torch

    print("case: reconstruction hybrid N=32, 2000 sampled cells", flush=True)
    mesh = inputs.lattice(32, "hybrid", box=(2 * math.pi,) * 3)
    Q0 = inputs.cell_averages(mesh, inputs.tgv())
    host = gks.HostMesh(mesh)
    sol = gks.Solver(host)
    coeff = sol.reconstruct(sol.upload(host.to_internal(Q0)))
    torch.cuda.synchronize()
    coeff = coeff.cpu().numpy()
    o = oracle.Oracle(mesh)
    vol, xc, _, _ = o.cell_geometry()
    rng = np.random.default_rng(32)
    V, RV, G, RG = [], [], [], []
    for i in rng.choice(host.n, 2000, replace=False):
        ext = host.perm[i]
        X = 0.4 * vol[ext] ** (1 / 3) * rng.standard_normal(3)
        v, g = _poly_eval(coeff[i], X)
        rv, rg = o.weno_eval(Q0, ext, xc[ext] + X)
        V.append(v), RV.append(rv), G.append(g), RG.append(rg)
    V, RV, G, RG = map(np.array, (V, RV, G, RG))
    # per component scales, the three momentum components sharing one (rho W starts at zero)
    vs = np.abs(RV).max(axis=0)
    gs = np.abs(RG).max(axis=(0, 2))
    vs[1:4], gs[1:4] = vs[1:4].max(), gs[1:4].max()
    ev = (np.abs(V - RV) / vs).max(axis=0)
    eg = (np.abs(G - RG).max(axis=2) / gs).max(axis=0)
    print("relative value error per component", ev, "gradient", eg, flush=True)
    assert (ev <= TOL).all() and (eg <= 1e-10).all()
