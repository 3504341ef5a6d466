"""Write config4_tangent_N16.json: directional derivatives of the kinetic energy after 100 steps.

Workload (the gradient case): the hybrid lattice at N = 16 on the periodic unit cube (mesh seed 2203,
23,031 cells), Euler (gamma = 1.4), the density wave plus the seeded low-pass velocity perturbation
(amplitude 0.05, wavenumbers <= 4, seed 9047), CFL 0.5, the paper's collision time (tau_eps = 0.01,
C = 1; the opening of Section 5), 100 S2O4 steps.  J = sum_i |Omega_i| |rho U_i|^2 / (2 rho_i) at step
100.  Directions k = 1..32: the seeded Gaussian field inputs.gaussian(k, 5 n) in the mesh's cell
order, [5][n], scaled to unit 2-norm and then per component by max_i |Q0_c,i|.

Only the oracle computes: its FP64 run fixes the step sizes (frozen), and its complex-step build gives
dJ/dQ0 . v_k exactly to rounding along each direction.  Usage (writes next to this file; each
direction is saved as soon as it is done, so an interrupted run resumes):

    python tests/golden/make_config4_tangent.py [--threads T]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_09047_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "config4_tangent_N16.json")
N, STEPS, NDIR = 16, 100, 32


def direction(k, Q0):
    v = inputs.gaussian(k, Q0.size).reshape(Q0.shape)
    v /= np.linalg.norm(v)
    return v * np.abs(Q0).max(axis=1, keepdims=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.threads:
        oracle.set_threads(a.threads)
    mesh = inputs.lattice(N, "hybrid")
    Q0 = inputs.cell_averages(mesh, inputs.perturbed_wave())
    prm = oracle.params()
    o = oracle.Oracle(mesh, prm)
    vol = o.cell_geometry()[0]
    if os.path.exists(OUT):
        rec = json.load(open(OUT))
    else:
        t0 = time.time()
        QT, dts = o.run(Q0, nsteps=STEPS)
        rec = dict(
            source="written by tests/golden/make_config4_tangent.py from the oracle only",
            workload=f"hybrid lattice N={N} periodic unit cube, perturbed density wave, Euler, CFL 0.5, "
                     f"tau_eps 0.01, tau_C 1, {STEPS} S2O4 steps",
            n_cells=int(mesh.n_cells), steps=STEPS, J=oracle.kinetic_energy(vol, QT),
            dts=[float(x) for x in dts], directions=[],
            forward_seconds=time.time() - t0)
    T = oracle.Tangent(mesh, prm)
    done = {d["seed"] for d in rec["directions"]}
    for k in range(1, NDIR + 1):
        if k in done:
            continue
        t0 = time.time()
        QT, VT = T.run(Q0, direction(k, Q0), rec["dts"])
        J, dJ = oracle.kinetic_energy(vol, QT, VT)
        assert J == rec["J"], (J, rec["J"])  # the complex build's real parts are the FP64 run's
        rec["directions"].append(dict(seed=k, dJ=dJ, seconds=time.time() - t0))
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(rec, f, indent=1)
        os.replace(tmp, OUT)
        print(f"direction {k}: dJ = {dJ!r} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
