"""Benchmark: one Newton step of a DIRK stage of the macro-element HDG method
on one MI355X (linearise -> second-layer condensation -> FGMRES to 1e-8 ->
local recovery -> update), on the Taylor-Green workload: 24^3 periodic hexes
on [-pi, pi]^3, macros of 3^3 elements (512 macros), p = 2, Mach 0.1,
Re 1600, seeded 1e-4 noise, first stage of Alexander's DIRK(3,3) with
dt = CFL h / (V0 (p+1)), CFL = 1.

Prints one JSON line.  Per-phase times come from HIP events recorded on the
library's stream around each C-ABI call; the global apply is also timed on
its own over repeated calls (HBM roofline).  The CPU baseline runs the
oracle (test infrastructure) on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DIRK-stage solve time to FGMRES tol 1e-8 + condense TFLOP/s, plain vs mixed/learned"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def workload_arrays(ctx, cfg, seed=0):
    from paper_2402_11361_amd import inputs
    mx, fx = ctx.node_coords()
    N = ctx.n_u_macro // (cfg["dim"] + 2)
    nf_nodes = None
    macro_coords = [mx[i * N:(i + 1) * N] for i in range(ctx.n_macros)]
    # faces: uniform size on this workload
    nfn = (ctx.n_glob // (cfg["dim"] + 2))
    n_faces = 3 * ctx.n_macros
    per = nfn // n_faces
    face_coords = [fx[f * per:(f + 1) * per] for f in range(n_faces)]
    u, q, uh = inputs.make_state(cfg, macro_coords, face_coords, seed=seed)
    return u, q, uh


def condense_flops(n_u, n_b):
    """Algorithmic flops of the elimination of one augmented macro matrix:
    LU of S (2/3 n_u^3) + S^{-1} C (2 n_u^2 n_b) + D Y (2 n_b^2 n_u)."""
    return (2.0 / 3.0) * n_u ** 3 + 2.0 * n_u ** 2 * n_b + 2.0 * n_b ** 2 * n_u


def cpu_baseline(cfg, n_sample=2):
    """Oracle leg: complex-step linearisation and route-B condensation of
    n_sample macros of the same workload, extrapolated to all macros (the
    global direct solve is not included)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from oracle import dirk
    from paper_2402_11361_amd import inputs
    M = box_mesh(3, cfg["n_elem"], cfg["m"], cfg["p"], lo=cfg["lo"], hi=cfg["hi"], periodic=True)
    S = System(M, Phys(Re=cfg["Re"], Mach=cfg["mach"]))
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, uh = inputs.make_state(cfg, mc, fc, seed=0)
    A, b, c = dirk.dirk33()
    dii = 1.0 / A[0, 0]
    dt = inputs.cfl_dt(cfg)
    w = -dii * u
    t0 = time.perf_counter()
    lin = S.linearize(q, u, uh, w=w, dt=dt, dii=dii, macros=list(range(n_sample)))
    t1 = time.perf_counter()
    S.condense(lin, "B")
    t2 = time.perf_counter()
    per_macro_ms = 1e3 * (t2 - t0) / n_sample
    return dict(value=per_macro_ms * M.n_macros, unit="ms/Newton-step (linearise+condense, extrapolated)",
                cores=len(os.sched_getaffinity(0)), kind="oracle",
                sample=f"{n_sample} of {M.n_macros} macros: complex-step linearisation "
                       f"{1e3 * (t1 - t0) / n_sample:.0f} ms/macro + LAPACK route-B condensation "
                       f"{1e3 * (t2 - t1) / n_sample:.0f} ms/macro, x{M.n_macros // n_sample}; global solve excluded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--applies", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import Context, mesh_spec_box

    cfg = dict(inputs.CONFIGS[args.config])
    spec = mesh_spec_box(cfg["dim"], cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], cfg["periodic"])
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    u_n = dev(u0)
    q_init, u_init, uh_init = dev(q0), dev(u0), dev(uh0)
    alpha = 0.435866521508459
    dii = 1.0 / alpha
    dt = inputs.cfl_dt(cfg)
    w = -dii * u_n
    q, u, uh = q_init.clone(), u_init.clone(), uh_init.clone()
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(bhat)
    dq = torch.zeros_like(q)
    du = torch.zeros_like(u)
    rtol = cfg["rtol"]

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def newton_step(record):
        q.copy_(q_init); u.copy_(u_init); uh.copy_(uh_init)
        e0 = ev()
        nrm = ctx.linearize_stage(q, u, uh, w, dt, dii)
        e1 = ev()
        ctx.condense(bhat)
        e2 = ev()
        x.zero_()
        info = ctx.fgmres_solve(bhat, x, rtol=rtol, restart=30, max_outer=300, inner_its=5)
        e3 = ev()
        ctx.local_backsolve(x, dq, du)
        ctx.axpy(1.0, dq, q); ctx.axpy(1.0, du, u); ctx.axpy(1.0, x, uh)
        e4 = ev()
        if record is not None:
            record.append((e0, e1, e2, e3, e4, info, nrm))

    for _ in range(args.warmup):
        newton_step(None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        newton_step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = np.array([[a.elapsed_time(b) for a, b in ((r[0], r[1]), (r[1], r[2]), (r[2], r[3]), (r[3], r[4]))]
                       for r in rec])
    ms_step = 1e3 * wall / args.steps
    lin_ms, cond_ms, kry_ms, bs_ms = phases.mean(axis=0)
    its = [r[5]["outer_its"] for r in rec]
    inner = [r[5]["inner_its"] for r in rec]
    # global apply on its own (HBM-bound GEMV over the condensed blocks)
    xa = torch.randn(ctx.n_glob, dtype=torch.float64, device="cuda")
    ya = torch.zeros_like(xa)
    for _ in range(3):
        ctx.apply_global(xa, ya)
    torch.cuda.synchronize()
    ea = ev()
    for _ in range(args.applies):
        ctx.apply_global(xa, ya)
    eb = ev()
    torch.cuda.synchronize()
    apply_ms = ea.elapsed_time(eb) / args.applies
    nb, nu, nm = ctx.n_b_macro, ctx.n_u_macro, ctx.n_macros
    apply_bytes = 8.0 * nm * nb * nb + 8.0 * nm * nb + 8.0 * nm * nb + 8.0 * ctx.n_glob
    apply_gbs = apply_bytes / (apply_ms * 1e-3) / 1e9
    flops = condense_flops(nu, nb) * nm
    cond_tflops = flops / (cond_ms * 1e-3) / 1e12
    # dominant kernel: the batched elimination inside hdg_condense (MFMA-bound)
    roofline = dict(bound="mfma", achieved=round(cond_tflops, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                    frac=round(cond_tflops / PEAK_FP64_TFLOPS, 4), traffic=None,
                    kernel="hdg_condense (form + batched FP64 LU/TRSM/GEMM elimination)",
                    flops_per_launch=flops, ms_per_launch=round(float(cond_ms), 3))
    out = dict(metric=METRIC, value=round(ms_step, 3), unit="ms/Newton-step", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=False, scaling="weak",
               vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=f"{args.config}: TGV 24^3 periodic hex, 3^3-element macros (512), p=2, "
                                    f"Mach 0.1, Re 1600, DIRK(3,3) stage 1, FGMRES rtol {rtol}",
                           n_macros=nm, n_u_macro=nu, n_b_macro=nb, n_glob=ctx.n_glob),
               phases_ms=dict(linearize=round(float(lin_ms), 3), condense=round(float(cond_ms), 3),
                              fgmres=round(float(kry_ms), 3), backsolve_update=round(float(bs_ms), 3)),
               fgmres=dict(outer_its=its, inner_its=inner, rel_res=[r[5]["res"] / r[5]["res0"] for r in rec]),
               condense_tflops=round(cond_tflops, 3), apply_ms=round(apply_ms, 4), apply_gbs=round(apply_gbs, 1),
               apply_frac_hbm=round(apply_gbs / PEAK_HBM_GBS, 4), residual_norms=[float(v) for v in rec[0][6]],
               roofline=roofline)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
