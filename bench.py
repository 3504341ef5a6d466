"""Throughput of the explicit WENO gas-kinetic S2O4 step on one MI355X.

Workload: hybrid tetrahedron/pyramid/prism/hexahedron lattice mesh of the
periodic box [0, 2 pi]^3 with N = 64 lattice cells per side (about 1.47 M
cells), compressible Navier-Stokes Taylor-Green vortex at Mach 0.1,
Re = 1600, Pr = 0.72, CFL 0.3, 200 steps.  A step is one full two-stage
fourth-order step: CFL time step, then twice WENO reconstruction -> face GKS
flux -> stage update.  Inputs are resident in HBM before the timed region.

The timed steps run with the library's per-launch events off; a further
short pass with them on gives the per-kernel durations of the rooflines.
Prints one JSON line: FP64 cell-updates/s as ``value``, with the FP32-mixed
throughput and its difference from FP64, the N = 96 lattice, the per-kernel
breakdown, the roofline of the dominant kernel and the oracle's CPU rate on a
bounded sample beside it.
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
# committed VALU counter summary (rocprofv3 SQ_INSTS_VALU and the FP64/FP32 FMA, MUL, ADD counts per
# dispatch): the flux's flops per Gauss point and each kernel's VALU issue utilisation, valid only for
# the kernel sources it was measured on
VALU_JSON = os.path.join(ROOT, "profiles", "valu_counters_hybrid-N64-tgv.json")
CLOCK_GHZ = 2.4
SIMDS = 1024  # 256 compute units x 4 SIMDs
# committed HBM counter summary (rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated), valid only for the
# kernel sources it was measured on and for the workload it was measured on (N = 64)
COUNTERS_JSON = os.path.join(ROOT, "profiles", "hbm_counters_hybrid-N64-tgv.json")
COUNTERS_N = 64
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2203_09047_amd", "csrc", f)
                  for f in ("gks_device.hip", "gks_flux.h", "gks_flux_adj.h", "gks_weno.h", "gks_internal.h", "gks_bc.h")]
# rocprofv3 kernel names -> the library's kernel keys
KERNEL_NAMES = {"k_reconstruct<double, false, 0>(": "reconstruct", "k_flux_chunked<true, false>(": "flux", "k_stage1<double>(": "stage1",
                "k_stage2<double>(": "stage2", "k_dt_partial(": "timestep", "k_flux_adj_a<true>(": "flux_adj_a",
                "k_flux_adj_b<true>(": "flux_adj_b", "k_reconstruct_adj(": "reconstruct_adj",
                "k_cbar_gather(": "cbar_gather", "k_transpose_gather(": "transpose_gather",
                "k_reconstruct<float, false, 0>(": "reconstruct_fp32", "k_flux<float, true, false, false>(": "flux_fp32",
                "k_stage1<float>(": "stage1_fp32", "k_stage2<float>(": "stage2_fp32"}
VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_ADD_F64",
                 "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_ADD_F32")



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


def measured_valu():
    """Per-kernel mean VALU counts per dispatch from the committed summary; empty once the kernel sources
    differ from the ones the counters were taken on."""
    try:
        with open(VALU_JSON) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return {}
    if d.get("kernel_source_sha256") != kernel_source_hash():
        return {}
    return d["kernels"]


def flops(counts, prec):
    """Floating-point operations of one dispatch from its VALU counts: the counters count wave
    instructions (64 lanes each, every lane active in these kernels), an FMA counts two."""
    t = "F64" if prec == 64 else "F32"
    return 64 * (2 * counts.get(f"SQ_INSTS_VALU_FMA_{t}", 0.0) + counts.get(f"SQ_INSTS_VALU_MUL_{t}", 0.0)
                 + counts.get(f"SQ_INSTS_VALU_ADD_{t}", 0.0))


def valu_from(dbs):
    """VALU counter summary from rocprofv3 databases of --pmc runs (any split of VALU_COUNTERS over the
    runs): per kernel and counter, the mean value per dispatch, summed over the device's dies."""
    import sqlite3

    acc = {}
    for db in dbs:
        con = sqlite3.connect(db)
        rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
        per = {}
        for disp, name, ctr, v in rows:
            for frag, key in KERNEL_NAMES.items():
                if frag in name and ctr in VALU_COUNTERS:
                    per.setdefault((key, ctr, disp), 0.0)
                    per[(key, ctr, disp)] += v
        for (key, ctr, _), v in per.items():
            acc.setdefault(key, {}).setdefault(ctr, []).append(v)
    return dict(kernel_source_sha256=kernel_source_hash(),
                kernels={k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in acc.items()})


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


def run_gpu(host, Q0, precision, steps, warmup, prof_steps, cfl, smooth=False, law=None):
    """Warm-up steps, then `steps` timed steps with HIP events on the solver's stream and the library's
    per-launch events off, a status poll (positivity), then `prof_steps` further steps with per-launch
    events on for the per-kernel durations.  Returns (solver, timed ms, kernel profile, state after the
    timed steps)."""
    import torch

    from paper_2203_09047_amd import gks

    prm = gks.params(precision=precision, viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=cfl, smooth=smooth,
                     **(law or {}))
    sol = gks.Solver(host, prm)
    Q = sol.upload(host.to_internal(Q0))
    for _ in range(warmup):
        sol.step(Q)
    sol.poll()
    stream = sol.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        sol.step(Q)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sol.poll()  # GKS_ENONPHYS raises: every timed state stayed physical
    q = Q.cpu().numpy()
    assert np.isfinite(q).all()
    prof = {}
    if prof_steps:
        sol.profile(True)
        for _ in range(prof_steps):
            sol.step(Q)
        prof = sol.profile_read()
        sol.profile(False)
        sol.poll()
    return sol, ms, prof, q


def state_summary(q, gamma=1.4):
    rho = q[0]
    p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho)
    return dict(min_rho=float(rho.min()), min_p=float(p.min()))


def differences(q, ref, vol):
    """Relative L-infinity per component (the momentum components share the scale max |rho U|) and L1
    (the integral of |dQ| over the domain)."""
    scale = np.abs(ref).max(axis=1)
    scale[1:4] = scale[1:4].max()
    return dict(rel_linf=(np.abs(q - ref).max(axis=1) / scale).tolist(),
                l1=(np.abs(q - ref) * vol).sum(axis=1).tolist())


def kernel_table(prof):
    return {k: dict(avg_ms=v[0] / max(v[1], 1), launches=v[1]) for k, v in prof.items() if v[1]}


def run_adjoint(args, host, Q0):
    """Adjoint/forward time ratio of a checkpointed rollout (FP64): forward = nsteps S2O4 steps with
    checkpoint stores, backward = segment recomputation + the discrete adjoint of every step."""
    import torch

    from paper_2203_09047_amd import gks
    from paper_2203_09047_amd.adjoint import Rollout

    prm = gks.params(precision=gks.FP64, viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=args.cfl)
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
    g_ckpt = Q.grad.clone()
    # store-all: the forward keeps every step's states and coefficient tape, the backward only runs adjoints
    Q.grad = None
    t3 = time.perf_counter()
    out = Rollout.apply(Q, sol, args.adj_steps, 10, True, True)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    J, g = sol.kinetic_energy(out.detach(), grad=True)
    out.backward(g)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    sol.profile(False)
    sol.poll()
    assert torch.isfinite(Q.grad).all()
    same = float((Q.grad - g_ckpt).abs().max() / g_ckpt.abs().max())
    return dict(steps=args.adj_steps, checkpoint_every=10, forward_s=t1 - t0, backward_s=t2 - t1,
                ratio=(t2 - t1) / (t1 - t0), kernels_backward=kernel_table(prof_b),
                store_all=dict(forward_s=t4 - t3, backward_s=t5 - t4, ratio=(t5 - t4) / (t1 - t0),
                               stored_gb=args.adj_steps * (sol.tape_bytes + 2 * Q.numel() * 8) / 1e9,
                               gradient_vs_checkpointed=same))


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


def cpu_baseline(N_sample=24, threads=1, cfl=0.3):
    import oracle
    from paper_2203_09047_amd import inputs

    oracle.set_threads(threads)  # the oracle's two parallel loops (results do not depend on the count)
    mesh = inputs.lattice(N_sample, "hybrid", box=(2 * math.pi,) * 3)
    Q0 = inputs.cell_averages(mesh, inputs.tgv())
    prm = oracle.params(viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=cfl)
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
    ap.add_argument("--steps", type=int, default=200, help="timed S2O4 steps (the workload's 200)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prof-steps", type=int, default=20, help="steps with per-launch events, after the timed ones")
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--cfl", type=float, default=0.3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-n96", action="store_true", help="skip the N = 96 lattice (4.96 M cells)")
    ap.add_argument("--n96-steps", type=int, default=20, help="timed steps of the N = 96 and cavity legs")
    ap.add_argument("--no-cavity", action="store_true", help="skip the lid-driven cavity (walls) timing")
    ap.add_argument("--no-paper-cavity", action="store_true",
                    help="skip the paper's implicit cavity timing (102,400 cells, 1000 steps)")
    ap.add_argument("--no-smooth", action="store_true", help="skip the smooth-flow flux (Eq. flux-2) comparison")
    ap.add_argument("--no-implicit", action="store_true", help="skip the implicit Jacobi step timing")
    ap.add_argument("--no-power-law", action="store_true", help="skip the power-law viscosity timing")
    ap.add_argument("--adj-steps", type=int, default=20, help="steps of the adjoint/forward ratio (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--counters-from", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="print the HBM counter summary of two rocprofv3 databases as JSON and exit")
    ap.add_argument("--valu-from", nargs="+", metavar="DB",
                    help="print the VALU counter summary of rocprofv3 --pmc databases as JSON and exit")
    args = ap.parse_args()
    if args.counters_from:
        print(json.dumps(counters_from(*args.counters_from), indent=1))
        return
    if args.valu_from:
        print(json.dumps(valu_from(args.valu_from), indent=1))
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
    host = gks.HostMesh(mesh)
    vol, _ = host.geometry()
    log(f"mesh N={args.N}: {mesh.n_cells} cells {mesh.hist} ({time.perf_counter() - t:.1f} s)")
    sol, ms64, prof64, q64 = run_gpu(host, Q0, gks.FP64, args.steps, args.warmup, args.prof_steps, args.cfl)
    del sol
    log(f"fp64: {args.steps} steps {ms64:.2f} ms {prof64}")
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
        "config": {"workload": f"hybrid-lattice N={args.N} periodic [0,2pi]^3 Taylor-Green Ma0.1 Re1600 Pr0.72 NS "
                               f"CFL{args.cfl}",
                   "cells": n, "faces": host.n_faces, "hist": mesh.hist},
        "state_after_timed_steps": dict(steps=args.warmup + args.steps, **state_summary(q64)),
    }
    kern = kernel_table(prof64)
    res["kernels_fp64"] = kern
    bytes64 = algorithmic_bytes(host, 8)
    dom = max(kern, key=lambda k: kern[k]["avg_ms"] * kern[k]["launches"])
    ops = gks.gp_op_count(viscous=True, Pr=0.72)
    res["flux_ops_per_gauss_point"] = ops
    traffic = measured_traffic() if args.N == COUNTERS_N else {}
    valu = measured_valu() if args.N == COUNTERS_N else {}
    ngp = 4 * host.n_faces
    # flops of one flux launch: the hardware count taken on these kernel sources; without one the flux's
    # rate is not reported (the source-level count of the Gauss-point body overstates it: it misses the
    # compiler's folding, 9.9k against 5.6k flops)
    if "flux" in valu:
        flux_flops, flops_source = flops(valu["flux"], 64), "rocprofv3 SQ_INSTS_VALU_{FMA,MUL,ADD}_F64"
    else:
        flux_flops, flops_source = None, "none: no VALU counts taken on these kernel sources"
    res["flux_fp64_flops_per_gauss_point"] = dict(value=flux_flops / ngp if flux_flops else None,
                                                  source=flops_source,
                                                  source_level_count=ops["add"] + ops["mul"] + ops["div"])

    def valu_util(key, avg_ms):
        """Share of the SIMDs' issue cycles taken by the kernel's VALU instructions, each wave64
        instruction 4 cycles (the FP64 rate: 16 lanes a cycle); not defined for the FP32 kernels, whose
        arithmetic issues at 32 lanes a cycle beside 4-cycle moves and integer work."""
        c = valu.get(key)
        if not c or "SQ_INSTS_VALU" not in c or key.endswith("_fp32"):
            return None
        return c["SQ_INSTS_VALU"] * 4 / (SIMDS * CLOCK_GHZ * 1e9 * avg_ms * 1e-3)

    def roofline(k, table, nbytes, key):
        avg_s = table[k]["avg_ms"] * 1e-3
        out = dict(kernel=k, traffic=traffic.get(key), valu_issue_util=valu_util(key, table[k]["avg_ms"]))
        if k == "flux" and key == "flux":
            achieved = flux_flops / avg_s / 1e12 if flux_flops else None
            out.update(bound="alu", achieved=achieved, peak=FP64_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                       frac=achieved / FP64_VECTOR_PEAK_TFLOPS if achieved else None,
                       hbm_gbs=nbytes[k] / avg_s / 1e9)
        else:
            achieved = nbytes[k] / avg_s / 1e9
            out.update(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS)
        return out

    res["roofline"] = roofline(dom, kern, bytes64, dom)
    res["roofline_kernels"] = {k: roofline(k, kern, bytes64, k) for k in ("reconstruct", "flux", "stage1", "stage2")
                               if k in kern}
    prof_steps = max(args.prof_steps, 1)
    step_s_prof = sum(kern[k]["avg_ms"] * kern[k]["launches"] for k in kern) / prof_steps * 1e-3
    step_s = ms64 / args.steps * 1e-3
    step_bytes64 = sum(bytes64[k] * kern[k]["launches"] for k in kern if k in bytes64) / prof_steps
    res["hbm_fraction_of_step_fp64"] = step_bytes64 / step_s / 1e9 / HBM_PEAK_GBS

    # attainable-roofline fraction of the step: each kernel's lower bound max(bytes / HBM peak,
    # flops / FP64 peak) summed over the step's launches, over the measured step time
    def bound_s(k, nbytes):
        t_mem = nbytes[k] / (HBM_PEAK_GBS * 1e9)
        t_alu = flux_flops / (FP64_VECTOR_PEAK_TFLOPS * 1e12) if k == "flux" else 0.0
        return max(t_mem, t_alu)

    res["roofline_fraction_of_step_fp64"] = sum(bound_s(k, bytes64) * kern[k]["launches"] for k in kern
                                                if k in bytes64) / prof_steps / step_s if flux_flops else None
    res["per_launch_event_overhead"] = dict(
        timed_ms_per_step=step_s * 1e3, sum_of_kernel_ms_per_step_with_events=step_s_prof * 1e3)
    if args.adj_steps > 0:
        torch.cuda.empty_cache()
        adj = run_adjoint(args, host, Q0)
        log(f"adjoint: {adj}")
        res["adjoint"] = adj
        res["adjoint_forward_ratio"] = adj["ratio"]
        res["adjoint_forward_ratio_store_all"] = adj["store_all"]["ratio"]
    if not args.no_fp32:
        torch.cuda.empty_cache()
        sol32, ms32, prof32, q32 = run_gpu(host, Q0, gks.FP32_MIXED, args.steps, args.warmup, args.prof_steps,
                                           args.cfl)
        del sol32
        log(f"fp32-mixed: {ms32:.2f} ms {prof32}")
        k32 = kernel_table(prof32)
        bytes32 = algorithmic_bytes(host, 4)
        step32 = ms32 / args.steps * 1e-3
        fp32 = dict(value=n * args.steps / (ms32 * 1e-3), ms_per_step=ms32 / args.steps, speedup_vs_fp64=ms64 / ms32,
                    difference_vs_fp64=dict(after_steps=args.warmup + args.steps, **differences(q32, q64, vol)),
                    state_after_timed_steps=state_summary(q32), kernels=k32)
        fp32["hbm_fraction_of_step"] = sum(bytes32[k] * k32[k]["launches"] for k in k32 if k in bytes32) / prof_steps \
            / step32 / 1e9 / HBM_PEAK_GBS
        if "flux" in k32:
            c = valu.get("flux_fp32")
            fl = flops(c, 32) if c else None
            avg_s = k32["flux"]["avg_ms"] * 1e-3
            fp32["flux_roofline"] = dict(
                bound="alu", unit="TFLOP/s", peak=FP32_VECTOR_PEAK_TFLOPS,
                achieved=fl / avg_s / 1e12 if fl else None,
                frac=fl / avg_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS if fl else None,
                hbm_gbs=bytes32["flux"] / avg_s / 1e9)
        res["fp32_mixed"] = fp32
    if not args.no_smooth:
        # the same workload with the smooth-flow flux (Eq. flux-2) at the Gauss points
        solsm, mssm, profsm, qsm = run_gpu(host, Q0, gks.FP64, args.steps, args.warmup, args.prof_steps, args.cfl,
                                           smooth=True)
        del solsm
        log(f"fp64 smooth flux: {mssm:.2f} ms {profsm}")
        ksm = kernel_table(profsm)
        res["smooth_flux_fp64"] = dict(
            value=n * args.steps / (mssm * 1e-3), ms_per_step=mssm / args.steps, speedup_vs_full_flux=ms64 / mssm,
            flux_kernel_speedup=kern["flux"]["avg_ms"] / ksm["flux"]["avg_ms"],
            difference_vs_full_flux=dict(after_steps=args.warmup + args.steps, **differences(qsm, q64, vol)),
            kernels=ksm)
    if not args.no_power_law:
        # the same workload with the viscosity law mu (T / T_ref)^0.7 (T_ref the initial mean temperature)
        T = float((0.4 * (Q0[4] - 0.5 * (Q0[1:4] ** 2).sum(axis=0) / Q0[0]) / Q0[0]).mean())
        solpl, mspl, profpl, qpl = run_gpu(host, Q0, gks.FP64, args.steps, args.warmup, args.prof_steps, args.cfl,
                                           law=dict(mu_power=0.7, T_ref=T))
        del solpl
        log(f"fp64 power-law viscosity: {mspl:.2f} ms {profpl}")
        kpl = kernel_table(profpl)
        res["power_law_viscosity_fp64"] = dict(
            value=n * args.steps / (mspl * 1e-3), ms_per_step=mspl / args.steps, mu_power=0.7, T_ref=T,
            flux_kernel_slowdown=kpl["flux"]["avg_ms"] / kern["flux"]["avg_ms"],
            difference_vs_constant_mu=dict(after_steps=args.warmup + args.steps, **differences(qpl, q64, vol)),
            kernels=kpl)
    if not args.no_implicit:
        # the paper's steady-solver path: one implicit step = reconstruction + flux over the CFL step,
        # the flux-split implicit operator with a pseudo-time step 10 times that, 3 Jacobi sweeps
        soli = gks.Solver(host, gks.params(viscous=True, mu=1.0 / 1600.0, Pr=0.72, cfl=args.cfl))
        Qi = soli.upload(host.to_internal(Q0))
        nimp = 20
        for _ in range(args.warmup):
            soli.implicit_step(Qi, dt_factor=10.0, kmax=3)
        soli.poll()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(soli.stream)
        for _ in range(nimp):
            soli.implicit_step(Qi, dt_factor=10.0, kmax=3)
        e1.record(soli.stream)
        torch.cuda.synchronize()
        msi = e0.elapsed_time(e1)
        soli.profile(True)
        for _ in range(args.prof_steps):
            soli.implicit_step(Qi, dt_factor=10.0, kmax=3)
        profi = soli.profile_read()
        soli.profile(False)
        soli.poll()
        del soli
        res["implicit_jacobi_fp64"] = dict(
            value=n * nimp / (msi * 1e-3), unit="cell-steps/s", steps=nimp, ms_per_step=msi / nimp, kmax=3,
            dt_factor=10.0, kernels=kernel_table(profi))
    if not args.no_cavity:
        # the paper's lid-driven cavity (Mach 0.15, Re = 1000, isothermal no-slip walls, the lid y = 1) on the
        # walled hybrid lattice of the unit box at the same N, FP64, events off
        t = time.perf_counter()
        meshc = inputs.lattice(args.N, "hybrid", periodic=False)
        p0 = 1.0 / 1.4
        Qc = inputs.cell_averages(meshc, inputs.uniform(1.0, 0.0, 0.0, 0.0, p0))
        hostc = gks.HostMesh(meshc)
        bc = [gks.boundary(gks.BC_ISOTHERMAL, Tw=p0) for _ in range(6)]
        bc[3] = gks.boundary(gks.BC_ISOTHERMAL, uw=(0.15, 0.0, 0.0), Tw=p0)
        prm = gks.params(viscous=True, mu=0.15 / 1000.0, Pr=0.72, cfl=args.cfl, bc=bc)
        solc = gks.Solver(hostc, prm)
        Qd = solc.upload(hostc.to_internal(Qc))
        for _ in range(args.warmup):
            solc.step(Qd)
        solc.poll()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(solc.stream)
        for _ in range(args.n96_steps):
            solc.step(Qd)
        e1.record(solc.stream)
        torch.cuda.synchronize()
        msc = e0.elapsed_time(e1)
        solc.profile(True)
        for _ in range(args.prof_steps):
            solc.step(Qd)
        profc = solc.profile_read()
        solc.profile(False)
        solc.poll()
        qc = Qd.cpu().numpy()
        res["lid_driven_cavity_fp64"] = dict(
            value=hostc.n * args.n96_steps / (msc * 1e-3), ms_per_step=msc / args.n96_steps, cells=hostc.n,
            steps=args.n96_steps, state_after_timed_steps=state_summary(qc),
            max_speed=float(np.sqrt((qc[1:4] ** 2).sum(axis=0)).max() / qc[0].min()), kernels=kernel_table(profc))
        log(f"cavity: {msc:.2f} ms ({time.perf_counter() - t:.1f} s)")
        del solc, hostc, Qd
        torch.cuda.empty_cache()
    if not args.no_n96:
        # the workload's larger lattice: FP64 and FP32-mixed, events off
        t = time.perf_counter()
        del host
        torch.cuda.empty_cache()
        mesh96 = inputs.lattice(96, "hybrid", box=(2 * math.pi,) * 3)
        Q96 = inputs.cell_averages(mesh96, inputs.tgv())
        host96 = gks.HostMesh(mesh96)
        log(f"mesh N=96: {mesh96.n_cells} cells ({time.perf_counter() - t:.1f} s)")
        n96 = {}
        for name, prec in (("fp64", gks.FP64), ("fp32_mixed", gks.FP32_MIXED)):
            if prec == gks.FP32_MIXED and args.no_fp32:
                continue
            s96, ms96, _, q96 = run_gpu(host96, Q96, prec, args.n96_steps, args.warmup, 0, args.cfl)
            del s96
            torch.cuda.empty_cache()
            n96[name] = dict(value=host96.n * args.n96_steps / (ms96 * 1e-3), ms_per_step=ms96 / args.n96_steps,
                             state_after_timed_steps=state_summary(q96))
        res["n96"] = dict(cells=host96.n, faces=host96.n_faces, steps=args.n96_steps, warmup=args.warmup, **n96)
        del host96
    if not args.no_paper_cavity:
        # the paper's own GPU timing case: its lid-driven cavity (Mach 0.15, Re = 1000, isothermal no-slip
        # walls) with the smooth-flow flux and the implicit Jacobi steady solver at k_max = 3, on a mesh
        # of the paper's size and cell mix (102,400 cells: 25,600 hexahedra and 76,800 prisms, here the
        # unrefined 40^3 lattice of the unit box in columns of either); 1000 steps timed, FP64, events off
        t = time.perf_counter()
        meshp = inputs.lattice(40, "hexprism", periodic=False)
        p0 = 1.0 / 1.4
        hostp = gks.HostMesh(meshp)
        bc = [gks.boundary(gks.BC_ISOTHERMAL, Tw=p0) for _ in range(6)]
        bc[3] = gks.boundary(gks.BC_ISOTHERMAL, uw=(0.15, 0.0, 0.0), Tw=p0)
        solp = gks.Solver(hostp, gks.params(viscous=True, mu=0.15 / 1000.0, Pr=0.72, cfl=args.cfl, smooth=True,
                                            bc=bc))
        Qp = solp.upload(hostp.to_internal(inputs.cell_averages(meshp, inputs.uniform(1.0, 0.0, 0.0, 0.0, p0))))
        for _ in range(10):
            solp.implicit_step(Qp, dt_factor=10.0, kmax=3)
        solp.poll()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(solp.stream)
        for _ in range(1000):
            solp.implicit_step(Qp, dt_factor=10.0, kmax=3)
        e1.record(solp.stream)
        torch.cuda.synchronize()
        msp = e0.elapsed_time(e1)
        solp.profile(True)
        for _ in range(args.prof_steps):
            solp.implicit_step(Qp, dt_factor=10.0, kmax=3)
        profp = solp.profile_read()
        solp.profile(False)
        solp.poll()
        qp = Qp.cpu().numpy()
        res["paper_cavity_implicit_fp64"] = dict(
            s_per_1000_steps=msp * 1e-3, value=hostp.n * 1000 / (msp * 1e-3), unit="cell-steps/s", cells=hostp.n,
            faces=hostp.n_faces, hist=meshp.hist, steps=1000, kmax=3, dt_factor=10.0, flux="smooth (Eq. flux-2)",
            state_after_timed_steps=state_summary(qp),
            max_speed=float(np.sqrt((qp[1:4] ** 2).sum(axis=0)).max() / qp[0].min()), kernels=kernel_table(profp),
            paper=dict(s_per_1000_steps=97.0, cells=102400, faces=274560,
                       hardware="Nvidia TITAN RTX, CUDA Fortran, FP64 (Jacobi k_max = 3, smooth-flow flux)"),
            speedup_vs_paper=97.0 / (msp * 1e-3))
        log(f"paper cavity (implicit): {msp:.1f} ms per 1000 steps ({time.perf_counter() - t:.1f} s)")
        del solp, hostp, Qp
        torch.cuda.empty_cache()
    res["hbm_copy_gbs_measured"] = copy_bandwidth()
    if not args.no_cpu:
        t = time.perf_counter()
        res["cpu_baseline"] = cpu_baseline(cfl=args.cfl)
        res["cpu_all_cores"] = cpu_baseline(threads=os.cpu_count() if os.environ.get("OMP_NUM_THREADS") is None
                                            else int(os.environ["OMP_NUM_THREADS"]), cfl=args.cfl)
        log(f"cpu baseline {time.perf_counter() - t:.1f} s")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
