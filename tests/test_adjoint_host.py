"""The hand-written reverse (adjoint) pieces, executed on the host, against finite differences.

The library exposes host executions of the same templated Gauss-point flux and
WENO combination that its kernels run, and of their reverse-mode products.
Central differences with one Richardson step pin every input cotangent.
"""
import ctypes

import numpy as np
import pytest

from paper_2203_09047_amd import gks


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def prim_to_cons(rho, U, p):
    U = np.asarray(U, float)
    return np.r_[rho, rho * U, p / 0.4 + 0.5 * rho * U @ U]


def richardson(fun, h):
    return (4 * fun(h / 2) - fun(h)) / 3


@pytest.mark.parametrize("viscous", [False, True])
def test_gauss_point_flux_vjp_matches_finite_differences(viscous):
    lib = gks.load()
    prm = gks.params(viscous=viscous, mu=2e-3, Pr=0.72 if viscous else 1.0)
    rng = np.random.default_rng(11 + viscous)
    for _ in range(3):
        x = [prim_to_cons(1 + 0.3 * rng.random(), 0.5 * rng.standard_normal(3), 1 + 0.3 * rng.random()),
             0.3 * rng.standard_normal((3, 5)),
             prim_to_cons(0.6 + 0.3 * rng.random(), 0.5 * rng.standard_normal(3), 0.7 + 0.3 * rng.random()),
             0.3 * rng.standard_normal((3, 5))]
        dt = 0.02

        def f(x):
            out = np.zeros(10)
            assert lib.gks_gp_flux_host(*(_p(np.ascontiguousarray(a)) for a in x), dt, ctypes.byref(prm), _p(out)) == 0
            return out

        ob = rng.standard_normal(10)
        g = [np.zeros(5), np.zeros((3, 5)), np.zeros(5), np.zeros((3, 5))]
        assert lib.gks_gp_flux_vjp_host(*(_p(np.ascontiguousarray(a)) for a in x), dt, ctypes.byref(prm), _p(ob),
                                        *(_p(a) for a in g)) == 0
        scale = max(np.abs(a).max() for a in g)
        for vi in range(4):
            for idx in np.ndindex(x[vi].shape):
                def d(h):
                    xp = [a.copy() for a in x]
                    xm = [a.copy() for a in x]
                    xp[vi][idx] += h
                    xm[vi][idx] -= h
                    return ob @ (f(xp) - f(xm)) / (2 * h)

                assert abs(richardson(d, 1e-4) - g[vi][idx]) < 1e-8 * scale, (vi, idx)


@pytest.mark.parametrize("force_linear", [False, True])
@pytest.mark.parametrize("M", [4, 6, 8])
def test_weno_combination_vjp_matches_finite_differences(force_linear, M):
    lib = gks.load()
    prm = gks.params(force_linear=force_linear)
    rng = np.random.default_rng(M + 10 * force_linear)
    a = rng.standard_normal(9)
    r = rng.standard_normal((8, 3))
    gi = np.zeros((8, 6))
    for s in range(8):
        A = rng.standard_normal((3, 3))
        Gi = np.linalg.inv(A @ A.T + np.eye(3))
        gi[s] = [Gi[0, 0], Gi[0, 1], Gi[0, 2], Gi[1, 1], Gi[1, 2], Gi[2, 2]]
    S = np.array([0.1, 0.01, -0.02, 0.12, 0.015, 0.09])
    v23, q0 = 0.7, 1.3

    def f(a, r, q0):
        c = np.zeros(10)
        lib.gks_weno_combine_host(_p(a), _p(np.ascontiguousarray(r)), _p(gi), M, v23, _p(S), q0, ctypes.byref(prm),
                                  _p(c))
        return c

    cb = rng.standard_normal(10)
    ab, rb, qb = np.zeros(9), np.zeros((8, 3)), np.zeros(1)
    lib.gks_weno_combine_vjp_host(_p(a), _p(r), _p(gi), M, v23, _p(S), ctypes.byref(prm), _p(cb), _p(ab), _p(rb),
                                  _p(qb))
    for j in range(9):
        def d(h):
            ap, am = a.copy(), a.copy()
            ap[j] += h
            am[j] -= h
            return cb @ (f(ap, r, q0) - f(am, r, q0)) / (2 * h)

        assert abs(richardson(d, 1e-4) - ab[j]) < 1e-8
    for s in range(8):
        for q in range(3):
            def d(h):
                rp, rm = r.copy(), r.copy()
                rp[s, q] += h
                rm[s, q] -= h
                return cb @ (f(a, rp, q0) - f(a, rm, q0)) / (2 * h)

            want = richardson(d, 1e-4) if s < M else 0.0
            assert abs(want - rb[s, q]) < 1e-8, (s, q)
    assert abs(richardson(lambda h: cb @ (f(a, r, q0 + h) - f(a, r, q0 - h)) / (2 * h), 1e-4) - qb[0]) < 1e-8


@pytest.mark.parametrize("case", ["euler", "ns_pr072"])
def test_gauss_point_flux_vjp_against_the_oracle_tangent(case):
    """The library's hand-written reverse of the Gauss-point flux against the oracle's forward-mode
    derivative (its complex-step build), with the paper's collision time (tau_C = 1): for random input
    directions v and output cotangents w, w . (J v) from the oracle equals (J^T w) . v from the
    library, to rounding."""
    import oracle

    lib = gks.load()
    kw = dict(euler={}, ns_pr072=dict(viscous=True, mu=2e-3, Pr=0.72))[case]
    prm = gks.params(tau_C=1.0, **kw)
    oprm = oracle.params(tau_C=1.0, **kw)
    rng = np.random.default_rng(21)
    for _ in range(5):
        x = [prim_to_cons(1 + 0.3 * rng.random(), 0.5 * rng.standard_normal(3), 1 + 0.3 * rng.random()),
             0.3 * rng.standard_normal((3, 5)),
             prim_to_cons(0.6 + 0.3 * rng.random(), 0.5 * rng.standard_normal(3), 0.7 + 0.3 * rng.random()),
             0.3 * rng.standard_normal((3, 5))]
        v = [rng.standard_normal(a.shape) for a in x]
        dt = 0.02
        ob = rng.standard_normal(10)
        g = [np.zeros(5), np.zeros((3, 5)), np.zeros(5), np.zeros((3, 5))]
        assert lib.gks_gp_flux_vjp_host(*(_p(np.ascontiguousarray(a)) for a in x), dt, ctypes.byref(prm), _p(ob),
                                        *(_p(a) for a in g)) == 0
        _, jv = oracle.gp_flux_tangent(oprm, *x, dt, *v)
        lhs = float(ob @ jv)
        rhs = float(sum((a * b).sum() for a, b in zip(g, v)))
        scale = np.abs(ob).sum() * np.abs(jv).max()
        assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)
