"""Throughput of the explicit WENO gas-kinetic S2O4 step on one MI355X.

Workload: hybrid tetrahedron/pyramid/prism/hexahedron lattice mesh of the
periodic box [0, 2 pi]^3 with N = 64 lattice cells per side (about 1.47 M
cells), compressible Navier-Stokes Taylor-Green vortex at Mach 0.1,
Re = 1600, Pr = 0.72.  A step is one full two-stage fourth-order step: CFL
time step, then twice WENO reconstruction -> face GKS flux -> stage update.
Inputs are resident in HBM before the timed region.

Prints one JSON line: FP64 cell-updates/s as ``value``, with the FP32-mixed
throughput, the per-kernel breakdown, the roofline of the dominant kernel and
the oracle's CPU rate on a bounded sample beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
# FP64 operations the flux kernel executes per Gauss point (Navier-Stokes, Pr != 1): the hardware
# counters SQ_INSTS_VALU_FMA_F64 (x 2), _MUL_F64 and _ADD_F64 over one launch at N = 64, divided by
# the launch's 4 F Gauss points (2250 FMA + 901 MUL + 194 ADD per point).  The source-level count
# (flux_ops_per_gauss_point) is larger: the compiler folds constant factors and shares products.
FLUX_FP64_FLOPS_PER_GP = 2 * 2250 + 901 + 194
# committed HBM counter summary (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated), valid only for the
# kernel sources it was measured on and for the workload it was measured on (N = 64)
COUNTERS_JSON = os.path.join(ROOT, "profiles", "hbm_counters_hybrid-N64-tgv.json")
COUNTERS_N = 64
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2203_09047_amd", "csrc", f)
                  for f in ("gks_device.hip", "gks_flux.h", "gks_flux_adj.h", "gks_weno.h", "gks_internal.h")]
# rocprofv3 kernel names -> the library's kernel keys
KERNEL_NAMES = {"k_reconstruct<double>(": "reconstruct", "k_flux_chunked<true, false>(": "flux", "k_stage1<double>(": "stage1",
                "k_stage2<double>(": "stage2", "k_dt_partial(": "timestep", "k_flux_adj_a<true>(": "flux_adj_a",
                "k_flux_adj_b<true>(": "flux_adj_b", "k_reconstruct_adj(": "reconstruct_adj",
                "k_cbar_gather(": "cbar_gather", "k_transpose_gather(": "transpose_gather"}



def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes (read + written) per launch from the committed counter summary; empty once the
    kernel sources differ from the ones the counters were taken on."""
    try:
        with open(COUNTERS_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return {}
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return {k: v["read_bytes"] + v["write_bytes"] for k, v in d["kernels"].items()}


def counters_from(fetch_db, write_db):
    """Counter summary from two rocprofv3 databases (one FETCH_SIZE run, one WRITE_SIZE run, both with
    --copy-calibration): per-kernel mean KiB per dispatch scaled by what the counter reads for the
    calibration copies of 1 GiB."""
    import sqlite3

    def per_kernel(db):
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                           "order by dispatch_id").fetchall()
        copies = [r[3] for r in rows if r[1] == "__amd_rocclr_copyBuffer" and r[2] == 131072][:3]
        factor = (1 << 30) / (sum(copies) / len(copies) * 1024.0)
        acc = {}
        for _, name, _, v in rows:
            for frag, key in KERNEL_NAMES.items():
                if frag in name:
                    acc.setdefault(key, []).append(v)
        return factor, {k: sum(v) / len(v) * 1024.0 * factor for k, v in acc.items()}

    ff, rd = per_kernel(fetch_db)
    wf, wr = per_kernel(write_db)
    return dict(kernel_source_sha256=kernel_source_hash(), fetch_factor=ff, write_factor=wf,
                kernels={k: dict(read_bytes=rd[k], write_bytes=wr.get(k, 0.0)) for k in rd})


def algorithmic_bytes(host, es):
    """Compulsory HBM bytes per launch of each kernel (es = bytes of the reduced-precision type)."""
    n, nf, ns = host.n, host.n_faces, host.n_stencil
    nsc = host.n_subcoef  # sub-stencil entries
    ncf = host.n_cellfaces
    # own cell averages (the gathered ones are the same array, read once), stencil pointers and member
    # cells, pseudo-inverse rows, sub-stencil list pointers / positions / 3-vectors, M, |Omega|^(2/3),
    # second moments, coefficients written
    recon = (40 * n + 4 * n + 4 * ns + 9 * es * ns + 32 * n + nsc + 3 * es * nsc + n + 8 * n + 48 * n
             + 50 * es * n)
    flux = 8 * nf + 9 * 4 * 8 * nf + 50 * es * n + 10 * es * nf + (40 * n if es == 4 else 0)
    stage1 = 4 * n + 4 * ncf + 10 * es * nf + 8 * n + 40 * n + 40 * n + 40 * n
    stage2 = 4 * n + 4 * ncf + 10 * es * nf + 8 * n + 40 * n + 40 * n
    timestep = 48 * n
    return dict(reconstruct=recon, flux=flux, stage1=stage1, stage2=stage2, timestep=timestep)


def run_gpu(args, mesh, Q0, precision, smooth=False, law=None):
    import torch

    from paper_2203_09047_amd import gks

    host = gks.HostMesh(mesh) if not hasattr(run_gpu, "host") else run_gpu.host
    run_gpu.host = host
    prm = gks.params(precision=precision, viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=0.5, smooth=smooth,
                     **(law or {}))
    sol = gks.Solver(host, prm)
    Q = sol.upload(host.to_internal(Q0))
    for _ in range(args.warmup):
        sol.step(Q)
    torch.cuda.synchronize()
    sol.poll()
    sol.profile(True)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        sol.step(Q)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    prof = sol.profile_read()
    sol.profile(False)
    sol.poll()
    q = Q.cpu().numpy()
    assert np.isfinite(q).all()
    run_gpu.last_q = q
    return host, sol, ms, prof


def run_adjoint(args, host, mesh, Q0):
    """Adjoint/forward time ratio of a checkpointed rollout (FP64): forward = nsteps S2O4 steps with
    checkpoint stores, backward = segment recomputation + the discrete adjoint of every step."""
    import torch

    from paper_2203_09047_amd import gks
    from paper_2203_09047_amd.adjoint import Rollout

    prm = gks.params(precision=gks.FP64, viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=0.5)
    sol = gks.Solver(host, prm)
    Q = sol.upload(host.to_internal(Q0)).requires_grad_(True)
    # warm-up of every kernel involved
    out = Rollout.apply(Q, sol, 2, 2)
    J, g = sol.kinetic_energy(out.detach(), grad=True)
    out.backward(g)
    torch.cuda.synchronize()
    Q.grad = None
    sol.profile(True)
    t0 = time.perf_counter()
    out = Rollout.apply(Q, sol, args.adj_steps, 10)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_f = sol.profile_read()
    J, g = sol.kinetic_energy(out.detach(), grad=True)
    out.backward(g)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    prof_b = sol.profile_read()
    sol.profile(False)
    sol.poll()
    assert torch.isfinite(Q.grad).all()
    kern = {k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1]) for k, v in prof_b.items() if v[1]}
    return dict(steps=args.adj_steps, checkpoint_every=10, forward_s=t1 - t0, backward_s=t2 - t1,
                ratio=(t2 - t1) / (t1 - t0), kernels_backward=kern)


def copy_bandwidth():
    """Device-to-device copy of 1 GiB (FP64), 10 times between HIP events: bytes read + written / time."""
    import torch

    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 10 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def cpu_baseline(N_sample=16, threads=1):
    import oracle
    from paper_2203_09047_amd import inputs

    oracle.set_threads(threads)  # the oracle's two parallel loops (results do not depend on the count)
    mesh = inputs.lattice(N_sample, "hybrid", box=(2 * math.pi,) * 3)
    Q0 = inputs.cell_averages(mesh, inputs.tgv())
    prm = oracle.params(viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=0.5)
    o = oracle.Oracle(mesh, prm)
    dt = o.timestep(Q0)
    t = time.perf_counter()
    o.step(Q0, dt)
    el = time.perf_counter() - t
    used = oracle.threads()
    return dict(value=mesh.n_cells / el, unit="cell-updates/s", cores=used, kind="oracle",
                sample=f"hybrid lattice N={N_sample} ({mesh.n_cells} cells), Taylor-Green Mach 0.1 NS, "
                       f"1 S2O4 step, FP64 C oracle on {used} thread(s), {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-smooth", action="store_true", help="skip the smooth-flow flux (Eq. flux-2) comparison")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit Jacobi step timing")
    ap.add_argument("--no-power-law", action="store_true", help="skip the power-law viscosity timing")
    ap.add_argument("--adj-steps", type=int, default=20, help="steps of the adjoint/forward ratio (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--counters-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="print the HBM counter summary of two rocprofv3 databases as JSON and exit")
    args = ap.parse_args()
    if args.counters_from:
        print(json.dumps(counters_from(*args.counters_from), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2203_09047_amd import gks, inputs

    gks.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU")
    if args.copy_calibration:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 1 GiB (read 1 GiB + write 1 GiB each)")
        del x, y
    t = time.perf_counter()
    mesh = inputs.lattice(args.N, "hybrid", box=(2 * math.pi,) * 3)
    Q0 = inputs.cell_averages(mesh, inputs.tgv())
    log(f"mesh N={args.N}: {mesh.n_cells} cells {mesh.hist} ({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    host, sol, ms64, prof64 = run_gpu(args, mesh, Q0, gks.FP64)
    log(f"fp64: {args.steps} steps {ms64:.2f} ms (setup+run {time.perf_counter() - t:.1f} s) {prof64}")
    n = host.n
    value = n * args.steps / (ms64 * 1e-3)
    res = {
        "metric": "cell-updates/s per S2O4 step (FP64 vs FP32-mixed) + adjoint/forward time ratio",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"hybrid-lattice N={args.N} periodic [0,2pi]^3 Taylor-Green Ma0.1 Re1600 Pr0.72 NS",
                   "cells": n, "faces": host.n_faces, "hist": mesh.hist},
    }
    kern = {k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1]) for k, v in prof64.items() if v[1]}
    res["kernels_fp64"] = kern
    bytes64 = algorithmic_bytes(host, 8)
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    # source-level FP64 operation count of one Gauss point (informational)
    res["flux_ops_per_gauss_point"] = gks.gp_op_count(viscous=True, Pr=0.72)
    traffic = measured_traffic() if args.N == COUNTERS_N else {}

    def roofline(k):
        avg_s = kern[k]["avg_ms"] * 1e-3
        tr = traffic.get(k)
        if k == "flux":
            achieved = FLUX_FP64_FLOPS_PER_GP * 4 * host.n_faces / avg_s / 1e12
            return dict(kernel=k, bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                        frac=achieved / FP64_VECTOR_PEAK_TFLOPS, traffic=tr)
        achieved = bytes64[k] / avg_s / 1e9
        return dict(kernel=k, bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=achieved / HBM_PEAK_GBS, traffic=tr)

    res["roofline"] = roofline(dom)
    res["roofline_kernels"] = {k: roofline(k) for k in ("reconstruct", "flux", "stage1", "stage2") if k in kern}
    q64 = run_gpu.last_q
    res["hbm_fraction_of_step_fp64"] = sum(bytes64[k] * kern[k]["launches"] for k in kern) / args.steps / (
        ms64 / args.steps * 1e-3) / 1e9 / HBM_PEAK_GBS

    # attainable-roofline fraction of the step: each kernel's lower bound max(bytes / HBM peak,
    # flops / FP64 peak) summed over the step's launches, over the measured step time
    def bound_s(k):
        t_mem = bytes64[k] / (HBM_PEAK_GBS * 1e9)
        t_alu = FLUX_FP64_FLOPS_PER_GP * 4 * host.n_faces / (FP64_VECTOR_PEAK_TFLOPS * 1e12) if k == "flux" else 0.0
        return max(t_mem, t_alu)

    res["roofline_fraction_of_step_fp64"] = sum(bound_s(k) * kern[k]["launches"] for k in kern if k in bytes64) / (
        ms64 * 1e-3)
    if args.adj_steps > 0:
        del sol
        torch.cuda.empty_cache()
        adj = run_adjoint(args, host, mesh, Q0)
        log(f"adjoint: {adj}")
        res["adjoint"] = adj
        res["adjoint_forward_ratio"] = adj["ratio"]
        sol = None
    if not args.no_fp32:
        del sol
        torch.cuda.empty_cache()
        _, sol32, ms32, prof32 = run_gpu(args, mesh, Q0, gks.FP32_MIXED)
        log(f"fp32-mixed: {ms32:.2f} ms {prof32}")
        q32 = run_gpu.last_q
        err = (np.abs(q32 - q64).max(axis=1) / np.abs(q64).max(axis=1)).tolist()
        res["fp32_mixed"] = dict(value=n * args.steps / (ms32 * 1e-3), ms_per_step=ms32 / args.steps,
                                 speedup_vs_fp64=ms64 / ms32,
                                 rel_linf_error_vs_fp64_per_component=err,
                                 error_after_steps=args.warmup + args.steps,
                                 kernels={k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1])
                                          for k, v in prof32.items() if v[1]})
    if not args.no_smooth:
        # the same workload with the smooth-flow flux (Eq. flux-2) at the Gauss points
        _, solsm, mssm, profsm = run_gpu(args, mesh, Q0, gks.FP64, smooth=True)
        log(f"fp64 smooth flux: {mssm:.2f} ms {profsm}")
        qsm = run_gpu.last_q
        del solsm
        ksm = {k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1]) for k, v in profsm.items() if v[1]}
        res["smooth_flux_fp64"] = dict(
            value=n * args.steps / (mssm * 1e-3), ms_per_step=mssm / args.steps, speedup_vs_full_flux=ms64 / mssm,
            flux_kernel_speedup=kern["flux"]["avg_ms"] / ksm["flux"]["avg_ms"],
            rel_linf_difference_vs_full_flux_per_component=(np.abs(qsm - q64).max(axis=1)
                                                            / np.abs(q64).max(axis=1)).tolist(),
            after_steps=args.warmup + args.steps, kernels=ksm)
    if not args.no_power_law:
        # the same workload with the viscosity law mu (T / T_ref)^0.7 (T_ref the initial mean temperature)
        T = float((0.4 * (Q0[4] - 0.5 * (Q0[1:4] ** 2).sum(axis=0) / Q0[0]) / Q0[0]).mean())
        _, solpl, mspl, profpl = run_gpu(args, mesh, Q0, gks.FP64, law=dict(mu_power=0.7, T_ref=T))
        log(f"fp64 power-law viscosity: {mspl:.2f} ms {profpl}")
        qpl = run_gpu.last_q
        del solpl
        kpl = {k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1]) for k, v in profpl.items() if v[1]}
        res["power_law_viscosity_fp64"] = dict(
            value=n * args.steps / (mspl * 1e-3), ms_per_step=mspl / args.steps, mu_power=0.7, T_ref=T,
            flux_kernel_slowdown=kpl["flux"]["avg_ms"] / kern["flux"]["avg_ms"],
            rel_linf_difference_vs_constant_mu_per_component=(np.abs(qpl - q64).max(axis=1)
                                                              / np.abs(q64).max(axis=1)).tolist(),
            after_steps=args.warmup + args.steps, kernels=kpl)
    if not args.no_implicit:
        # the paper's steady-solver path: one implicit step = reconstruction + flux over the CFL step,
        # the flux-split implicit operator with a pseudo-time step 10 times that, 3 Jacobi sweeps
        from paper_2203_09047_amd import gks as _g
        soli = _g.Solver(run_gpu.host, _g.params(viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=0.5))
        Qi = soli.upload(run_gpu.host.to_internal(Q0))
        for _ in range(args.warmup):
            soli.implicit_step(Qi, dt_factor=10.0, kmax=3)
        soli.poll()
        soli.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            soli.implicit_step(Qi, dt_factor=10.0, kmax=3)
        e1.record()
        torch.cuda.synchronize()
        msi = e0.elapsed_time(e1)
        profi = soli.profile_read()
        soli.profile(False)
        soli.poll()
        del soli
        res["implicit_jacobi_fp64"] = dict(
            value=n * args.steps / (msi * 1e-3), unit="cell-steps/s", ms_per_step=msi / args.steps, kmax=3,
            dt_factor=10.0, kernels={k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1]) for k, v in profi.items() if v[1]})
    res["hbm_copy_gbs_measured"] = copy_bandwidth()
    if not args.no_cpu:
        t = time.perf_counter()
        res["cpu_baseline"] = cpu_baseline()
        res["cpu_all_cores"] = cpu_baseline(threads=os.cpu_count() if os.environ.get("OMP_NUM_THREADS") is None
                                            else int(os.environ["OMP_NUM_THREADS"]))
        log(f"cpu baseline {time.perf_counter() - t:.1f} s")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
