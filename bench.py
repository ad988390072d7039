"""Benchmark: one DIRK stage of the macro-element HDG method solved by Newton's
method on one MI355X (each Newton step: linearise -> second-layer condensation
-> FGMRES to 1e-8 -> local recovery -> update), on the Taylor-Green workload: 24^3 periodic hexes
on [-pi, pi]^3, macros of 3^3 elements (512 macros), p = 2, Mach 0.1,
Re 1600, seeded 1e-4 noise, first stage of Alexander's DIRK(3,3) with
dt = CFL h / (V0 (p+1)), CFL = 1.

Prints one JSON line.  Per-phase times come from HIP events recorded on the
library's stream around each C-ABI call; the global apply is also timed on
its own over repeated calls (HBM roofline).  The CPU baseline runs the
oracle (test infrastructure) on a bounded sample of the same workload.
"""
import argparse
import gc
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
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# HBM bytes per hdg_condense call of the FP64 path on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by what the counters
# read for a 1 GiB device copy in the same run (profiles/stage_solve_tgv24_m3_p2_fp64.md),
# valid only while the kernel sources hash to `sha`.
CONDENSE_TRAFFIC = {"sha": "e0ebc3daaf95b564", "bytes": 1161.2e9}
CONDENSE_SOURCES = ("k_form.hip", "k_lu.hip")


def sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in CONDENSE_SOURCES:
        with open(os.path.join(ROOT, "paper_2402_11361_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def workload_arrays(ctx, cfg, seed=0):
    from paper_2402_11361_amd import inputs
    macro_coords, face_coords = ctx.node_coords_split()
    u, q, uh = inputs.make_state(cfg, macro_coords, face_coords, seed=seed)
    return u, q, uh


def condense_flops(cfg, n_u, n_b, elems=None):
    """Algorithmic flops of the condensation of one macro: LU of S (2/3 n_u^3),
    S^{-1} C (2 n_u^2 n_b), D Y (2 n_b^2 n_u), plus the formation of S
    (F_S = 2 d n_s^2 (p+1)^{2d} N E) and of the coupling blocks
    (F_C = 4 d n_s^2 (p+1)^{2d} (n_b / n_s) E) from element-blocked products,
    E = m^d elements per macro."""
    d, p = cfg["dim"], cfg["p"]
    E = elems if elems is not None else cfg["m"] ** d
    ns = d + 2
    N = n_u // ns
    F_S = 2.0 * d * ns ** 2 * (p + 1) ** (2 * d) * N * E
    F_C = 4.0 * d * ns ** 2 * (p + 1) ** (2 * d) * (n_b / ns) * E
    return (2.0 / 3.0) * n_u ** 3 + 2.0 * n_u ** 2 * n_b + 2.0 * n_b ** 2 * n_u + F_S + F_C


def uneven_variant(args, dev_fn, variants):
    """Stage solves on the 32^3 mesh cut into seeded segments of 2, 3 and 4
    elements per axis (27 macro shapes in one mesh), plain FP64 and FP32
    condensation."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.driver import StageDriver, alexander_dirk33
    from paper_2402_11361_amd.hdg import HDG_FP32, HDG_FP64, Context
    cfg = dict(inputs.CONFIGS["tgv32_uneven_p2"])
    seg = inputs.segments(cfg)
    spec = dict(dim=3, n_elem=[cfg["n_elem"]] * 3, lo=[cfg["lo"]] * 3, hi=[cfg["hi"]] * 3, periodic=[True] * 3,
                seg_len=seg, p=cfg["p"])
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    q_i, u_i, uh_i = dev_fn(q0), dev_fn(u0), dev_fn(uh0)
    A, _, _ = alexander_dirk33()
    dii = 1.0 / A[0, 0]
    dt = inputs.cfl_dt(cfg)
    w = -dii * u_i
    q, u, uh = q_i.clone(), u_i.clone(), uh_i.clone()
    flops = 0.0
    # per-macro element counts in macro order (axis 0 fastest)
    elems = [a * b * c for c in seg[2] for b in seg[1] for a in seg[0]]
    for i in range(ctx.n_macros):
        nu = int(ctx.u_off[i + 1] - ctx.u_off[i])
        nb = int(ctx.b_off[i + 1] - ctx.b_off[i])
        flops += condense_flops(cfg, nu, nb, elems[i])
    out = dict(workload="32^3 periodic Taylor-Green, segments of 2/3/4 elements per axis (seed 3), p=2, "
                        f"{ctx.n_macros} macros of 27 shapes, n_glob {ctx.n_glob}",
               n_macros=ctx.n_macros, n_glob=ctx.n_glob, condense_flops=flops)

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    if args.set_tuning:
        shape = [int(v) for v in args.set_tuning.split(",")]
        for prec in (HDG_FP64, HDG_FP32):
            for k in range(ctx.class_count()):
                ctx.set_tuning(k, prec, *shape)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        ctx.linearize_stage(q_i, u_i, uh_i, w, dt, dii, norms=False)
        for prec in (HDG_FP64, HDG_FP32):
            ctx.autotune(prec, args.tune_cache)
        out["autotune_seconds"] = round(time.perf_counter() - t0, 2)
    for name, prec in (("plain_fp64", HDG_FP64), ("mixed_fp32", HDG_FP32)):
        marks = []
        drv = StageDriver(ctx, rtol=cfg["rtol"], condense_prec=prec, mark=lambda ph: marks.append((ph, ev())))
        for rep in range(2):  # warm-up, then timed
            q.copy_(q_i); u.copy_(u_i); uh.copy_(uh_i)
            marks.clear()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = drv.solve_stage(q, u, uh, w, dt, dii)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
        cond = [e.elapsed_time(e2) for (ph, e), (_, e2) in zip(marks[:-1], marks[1:]) if ph == "condense"]
        cm = float(np.mean(cond))
        peak = PEAK_FP64_TFLOPS if prec == HDG_FP64 else PEAK_FP32_TFLOPS
        out[name] = dict(ms_per_stage=round(1e3 * wall, 3), newton_its=info["newton_its"],
                         fgmres_outer=[k["outer_its"] for k in info["krylov"]], condense_ms=round(cm, 3),
                         condense_tflops=round(flops / (cm * 1e-3) / 1e12, 3),
                         condense_frac_peak=round(flops / (cm * 1e-3) / 1e12 / peak, 4))
    variants["uneven_macros_32cubed"] = out
    ctx.close()


def big_variant(args, dev_fn, variants):
    """The 48^3 workload (1728 macros of 4^3 elements, p = 2): chunked FP32
    condensation, FP32 inner operator, graph-captured FGMRES steps; whole
    DIRK(3,3) time steps from the seeded state."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.driver import StageDriver
    from paper_2402_11361_amd.hdg import HDG_FP32, Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv48_m4_p2"])
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    free, _ = torch.cuda.mem_get_info()
    per = ctx.fit_chunking(free - (8 << 30))
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    q, u, uh = dev_fn(q0), dev_fn(u0), dev_fn(uh0)
    dt = inputs.cfl_dt(cfg)
    drv = StageDriver(ctx, rtol=cfg["rtol"], condense_prec=HDG_FP32, inner_prec=HDG_FP32,
                      graph_steps=args.graph_steps)
    steps = []
    for n in range(args.big_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = drv.step(q, u, uh, dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        steps.append(dict(ms=round(1e3 * wall, 1), ms_per_stage=round(1e3 * wall / len(infos), 1),
                          newton_its=[i["newton_its"] for i in infos],
                          fgmres_outer=[[k["outer_its"] for k in i["krylov"]] for i in infos]))
        print(f"[bench] 48^3 time step {n + 1}: {steps[-1]['ms']} ms", file=sys.stderr, flush=True)
    variants["tgv48_chunked_fp32_graph_steps"] = dict(
        workload="48^3 periodic Taylor-Green, 4^3-element macros (1728), p=2, "
                 f"n_glob {ctx.n_glob}; {per} macros per condensation chunk",
        macros_per_chunk=per, workspace_gb=round(ctx.workspace_bytes / 1e9, 1), time_steps=steps)
    ctx.close()


def first_layer_variant(args, dev_fn, variants):
    """Standard (first-layer) condensation of (q, u) together against the
    second layer, both FP64 on the 24^3 workload in two chunks, from the
    same linearisation: time per condensation and the largest difference of
    the condensed blocks of a few macros."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import HDG_FP64, Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv24_m3_p2"])
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    ctx.set_chunking((ctx.n_macros + 1) // 2)
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    dii = 1.0 / 0.435866521508459
    dt = inputs.cfl_dt(cfg)
    u = dev_fn(u0)
    ctx.linearize_stage(dev_fn(q0), u, dev_fn(uh0), -dii * u, dt, dii, norms=False)
    if args.set_tuning:
        ctx.set_tuning(0, HDG_FP64, *[int(v) for v in args.set_tuning.split(",")])
    else:
        ctx.autotune(HDG_FP64, args.tune_cache)
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    sample = [0, ctx.n_macros // 2, ctx.n_macros - 1]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    ms2 = timed(lambda: ctx.condense(bhat, HDG_FP64), 2)
    second = [ctx.get_condensed(i)[0] for i in sample]
    print(f"[bench] second-layer condensation {ms2:.1f} ms", file=sys.stderr, flush=True)
    ms1 = timed(lambda: ctx.condense_first_layer(bhat), 1)
    print(f"[bench] first-layer condensation {ms1:.1f} ms", file=sys.stderr, flush=True)
    diff = max(float(np.abs(ctx.get_condensed(i)[0] - a).max() / np.abs(a).max()) for i, a in zip(sample, second))
    nu, nb = ctx.n_u_macro, ctx.n_b_macro
    variants["first_vs_second_layer_fp64"] = dict(
        workload="24^3 periodic Taylor-Green, 3^3-element macros (512), p=2, two condensation chunks",
        ms_second_layer=round(ms2, 1), ms_first_layer=round(ms1, 1), ratio=round(ms1 / ms2, 2),
        pivot_order=dict(second=nu, first=4 * nu), ahat_rel_diff=diff, tuning=list(ctx.tuning(0, HDG_FP64)),
        nb=nb)
    ctx.close()


def tgv_dissipation_variant(args, dev_fn, variants):
    """Re = 100 Taylor-Green time integration from the clean initial field on
    two discretisations of equal effective resolution, (m, p) = (3, 2) and
    (2, 3) (6 macros per axis, N_eff = 42^3): kinetic energy and the
    dissipation rate of eq. C5321 after every DIRK(3,3) step, with
    -dE_k/dt by central differences as a check (Sec. 5.3).  FP32
    condensation with the BF16 inner operator and graph-captured FGMRES
    steps; Newton refines every stage to the FP64 tolerance."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.driver import StageDriver
    from paper_2402_11361_amd.hdg import HDG_BF16, HDG_FP32, Context, mesh_spec_box
    out = {}
    for name in ("tgv_re100_m3_p2", "tgv_re100_m2_p3"):
        cfg = dict(inputs.CONFIGS[name])
        spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
        stream = torch.cuda.current_stream()
        ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
        ctx.bind_workspace()
        u0, q0, uh0 = workload_arrays(ctx, cfg)
        q, u, uh = dev_fn(q0), dev_fn(u0), dev_fn(uh0)
        V0 = cfg["mach"]           # L = 1: t_c = L / V0, E_k in V0^2, eps in V0^3 / L
        dt = inputs.cfl_dt(cfg)
        n_steps = int(math.ceil(args.tgv_eps * (1.0 / V0) / dt - 1e-9))
        drv = StageDriver(ctx, rtol=cfg["rtol"], condense_prec=HDG_FP32, inner_prec=HDG_BF16,
                          graph_steps=args.graph_steps)
        ek, eps, _ = ctx.flow_diagnostics(q, u)
        t_s, ek_s, eps_s, newton, outer = [0.0], [ek / V0 ** 2], [eps / V0 ** 3], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(n_steps):
            infos = drv.step(q, u, uh, dt)
            ek, eps, _ = ctx.flow_diagnostics(q, u)
            t_s.append((n + 1) * dt * V0)
            ek_s.append(ek / V0 ** 2)
            eps_s.append(eps / V0 ** 3)
            newton += [i["newton_its"] for i in infos]
            outer += [k["outer_its"] for i in infos for k in i["krylov"]]
            if (n + 1) % 10 == 0 or n + 1 == n_steps:
                print(f"[bench] {name} step {n + 1}/{n_steps} t/t_c {t_s[-1]:.2f} E_k {ek_s[-1]:.5f} "
                      f"eps {eps_s[-1]:.5f}", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        t_a, e_a, d_a = np.array(t_s), np.array(ek_s), np.array(eps_s)
        dedt = -(e_a[2:] - e_a[:-2]) / (t_a[2:] - t_a[:-2])   # at t_a[1:-1]
        mismatch = float(np.max(np.abs(dedt - d_a[1:-1])) / np.max(d_a))
        ipk = int(np.argmax(d_a))
        out[name] = dict(
            workload=f"Taylor-Green Re 100, Mach 0.1, {cfg['n_elem']}^3 elements in 6^3 macros of "
                     f"{cfg['m']}^3, p={cfg['p']}, N_eff 42^3, n_glob {ctx.n_glob}",
            dt_over_tc=round(dt * V0, 5), steps=n_steps, wall_s=round(wall, 1),
            s_per_step=round(wall / max(n_steps, 1), 3),
            newton_its=[min(newton), max(newton)] if newton else [], fgmres_outer=[min(outer), max(outer)] if outer else [],
            eps_peak=round(float(d_a[ipk]), 6), t_eps_peak=round(float(t_a[ipk]), 3),
            max_rel_diff_minus_dEdt_vs_eps=round(mismatch, 4),
            t=[round(v, 4) for v in t_s], E_k=[round(v, 7) for v in ek_s], eps=[round(v, 7) for v in eps_s])
        ctx.close()
        del q, u, uh, drv
        gc.collect()
        torch.cuda.empty_cache()
    a, b = out["tgv_re100_m3_p2"], out["tgv_re100_m2_p3"]
    variants["tgv_re100_dissipation_m3p2_vs_m2p3"] = dict(
        t_end_over_tc=args.tgv_eps, runs=out,
        eps_peak_rel_diff=round(abs(a["eps_peak"] - b["eps_peak"]) / max(a["eps_peak"], b["eps_peak"]), 4))


def learned_p3_variant(args, dev_fn, variants):
    """The learned coarse correction on the 32^3 mesh with 4^3-element macros
    at p = 3 (512 macros, chunked FP32 condensation): pairs harvested from a
    plain solve on the seed-100 state, evaluated on the held-out seed-200
    state (first Newton step), plain and learned preconditioner."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import HDG_FP32, Context, mesh_spec_box
    from paper_2402_11361_amd.learned import CoarseCorrection
    cfg = dict(inputs.CONFIGS["tgv32_m4_p3"])
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    free, _ = torch.cuda.mem_get_info()
    per = ctx.fit_chunking(free - (12 << 30))
    ctx.bind_workspace()
    dt = inputs.cfl_dt(cfg)
    dii = 1.0 / 0.435866521508459
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")

    def condense_state(seed):
        u0, q0, uh0 = workload_arrays(ctx, cfg, seed=seed)
        q, u, uh = dev_fn(q0), dev_fn(u0), dev_fn(uh0)
        ctx.linearize_stage(q, u, uh, -dii * u, dt, dii)
        ctx.condense(bhat, HDG_FP32)

    t0 = time.perf_counter()
    cc = CoarseCorrection(ctx, hidden=256, max_batch=1024, seed=0)
    condense_state(100)
    cc.harvest(bhat, n_vectors=args.train_vectors, inner_prec=HDG_FP32)
    X, T = torch.cat(cc.X), torch.cat(cc.T)
    loss0 = cc.eval_loss(X, T)
    cc.train(epochs=args.train_epochs, lr=1e-3, batch=1024)
    loss1 = cc.eval_loss(X, T)
    cc.bind()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] p=3 learned: {cc.n_pairs()} pairs, loss {loss0:.3e} -> {loss1:.3e}", file=sys.stderr, flush=True)
    condense_state(200)
    evals = {}
    for name, lrn in (("plain", False), ("learned", True)):
        x = torch.zeros_like(bhat)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        info = ctx.fgmres_solve(bhat, x, rtol=cfg["rtol"], restart=30, max_outer=300, inner_its=5,
                                inner_prec=HDG_FP32, use_learned=lrn)
        torch.cuda.synchronize()
        evals[name] = dict(outer_its=info["outer_its"], inner_its=info["inner_its"], ms=round(1e3 * (time.perf_counter() - ts), 1),
                           fallbacks=info["fallbacks"], converged=info["converged"])
    variants["tgv32_m4_p3_learned"] = dict(
        workload=f"32^3 periodic Taylor-Green, 4^3-element macros (512), p=3, n_glob {ctx.n_glob}; chunked FP32 "
                 f"condensation ({per} macros per chunk); train on seed 100, evaluate on seed 200",
        pairs=cc.n_pairs(), loss_initial=loss0, loss_final=loss1, train_s=round(t1 - t0, 1), solve=evals)
    ctx.close()


def train_learned(ctx, cfg, dev, dii, dt, args):
    """Train the learned coarse correction on pairs harvested from plain FGMRES
    solves of the first Newton step on states with other noise seeds (1, 2, ...);
    the timed stage (seed 0) is held out.  Returns a summary."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import HDG_FP32
    from paper_2402_11361_amd.learned import CoarseCorrection
    t0 = time.perf_counter()
    cc = CoarseCorrection(ctx, hidden=256, max_batch=1024, seed=0)
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    for s in range(1, args.train_seeds + 1):
        u0, q0, uh0 = workload_arrays(ctx, cfg, seed=s)
        q, u, uh = dev(q0), dev(u0), dev(uh0)
        ctx.linearize_stage(q, u, uh, -dii * u, dt, dii)
        ctx.condense(bhat, HDG_FP32)
        cc.harvest(bhat, n_vectors=args.train_vectors)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X, T = torch.cat(cc.X), torch.cat(cc.T)
    loss0 = cc.eval_loss(X, T)
    hist = cc.train(epochs=args.train_epochs, lr=1e-3, batch=1024)
    loss1 = cc.eval_loss(X, T)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    cc.bind()
    return dict(pairs=cc.n_pairs(), seeds=list(range(1, args.train_seeds + 1)), harvest_s=round(t1 - t0, 2),
                train_s=round(t2 - t1, 2), epochs=args.train_epochs, loss_initial=loss0, loss_final=loss1,
                hidden=256, inference="BF16 weights, FP32 accumulation")


def blas_threads():
    """Threads the oracle's LAPACK/BLAS calls use (NumPy's BLAS pool)."""
    try:
        from threadpoolctl import threadpool_info
        n = [i["num_threads"] for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return len(os.sched_getaffinity(0))


def cpu_baseline(cfg, newton_its, n_sample=2):
    """Oracle leg: complex-step linearisation, route-B condensation and local
    recovery of n_sample macros of the same workload, scaled to all macros and
    to the Newton iterations the GPU took for one stage (the oracle's global
    solve is not included, so this under-counts the CPU time)."""
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from oracle import dirk
    from paper_2402_11361_amd import inputs
    M = box_mesh(cfg["dim"], cfg["n_elem"], cfg["m"], cfg["p"], lo=cfg["lo"], hi=cfg["hi"], periodic=cfg["periodic"])
    S = System(M, Phys(Re=cfg["Re"], Mach=cfg["mach"]))
    mc = [M.macro_node_coords(i) for i in range(M.n_macros)]
    fc = [M.face_node_coords(f) for f in range(M.n_faces)]
    u, q, uh = inputs.make_state(cfg, mc, fc, seed=0)
    A, b, c = dirk.dirk33()
    dii = 1.0 / A[0, 0]
    dt = inputs.cfl_dt(cfg)
    w = -dii * u
    sample = list(range(n_sample))
    t0 = time.perf_counter()
    lin = S.linearize(q, u, uh, w=w, dt=dt, dii=dii, macros=sample)
    t1 = time.perf_counter()
    con = S.condense(lin, "B")
    t2 = time.perf_counter()
    x = np.random.default_rng(5).uniform(-1, 1, M.n_glob)
    S.backsolve(lin, con, x)
    t3 = time.perf_counter()
    per_macro = (t3 - t0) / n_sample
    scale = M.n_macros * max(newton_its, 1)
    return dict(value=round(1e3 * per_macro * scale, 1),
                unit="ms/DIRK-stage (local work only, extrapolated)",
                cores=blas_threads(), kind="oracle",
                sample=f"{n_sample} of {M.n_macros} macros, one Newton step: complex-step linearisation "
                       f"{1e3 * (t1 - t0) / n_sample:.0f} ms/macro + LAPACK route-B condensation "
                       f"{1e3 * (t2 - t1) / n_sample:.0f} ms/macro + recovery "
                       f"{1e3 * (t3 - t2) / n_sample:.0f} ms/macro, scaled x{M.n_macros} macros "
                       f"x{max(newton_its, 1)} Newton steps; oracle global solve excluded")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="tgv24_m3_p2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--plain-only", action="store_true", help="time only the plain FP64 variant")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction variant")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-macro 32^3 variant")
    ap.add_argument("--graph-steps", type=int, default=10, help="FGMRES steps per captured HIP graph")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default elimination launch shapes")
    ap.add_argument("--learned-p3", action="store_true",
                    help="also train and evaluate the learned correction on the 32^3 p=3 workload")
    ap.add_argument("--big-steps", type=int, default=0,
                    help="also time this many DIRK(3,3) steps of the 48^3 workload (chunked condensation)")
    ap.add_argument("--tune-cache", default=None, help="text file of earlier autotuner choices (read and appended)")
    ap.add_argument("--plain-prec", choices=("fp64", "fp32"), default="fp64",
                    help="condensation precision of the main timed variant (profiling of the FP32 path)")
    ap.add_argument("--uneven-only", action="store_true",
                    help="time only the uneven-macro 32^3 variant (profiling); prints its JSON")
    ap.add_argument("--set-tuning", default=None, metavar="TPW,WIDE,LOOK",
                    help="fixed elimination launch shape for every class instead of the autotuner (profiling)")
    ap.add_argument("--first-layer", action="store_true",
                    help="also time the standard (first-layer) condensation against the second layer at 24^3")
    ap.add_argument("--tgv-eps", type=float, default=0.0, metavar="T_END",
                    help="also integrate the Re = 100 Taylor-Green flow to t/t_c = T_END on (m,p) = (3,2) and (2,3) "
                         "and report the dissipation rate")
    ap.add_argument("--train-seeds", type=int, default=2)
    ap.add_argument("--train-vectors", type=int, default=40)
    ap.add_argument("--train-epochs", type=int, default=60)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.driver import StageDriver, alexander_dirk33
    from paper_2402_11361_amd.hdg import HDG_BF16, HDG_FP32, HDG_FP64, Context, mesh_spec_box

    if args.uneven_only:
        dev0 = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
        variants = {}
        uneven_variant(args, dev0, variants)
        print(json.dumps(dict(metric=METRIC, unit="ms/DIRK-stage", n_gpus=1, data="synthetic", variants=variants)),
              flush=True)
        return
    cfg = dict(inputs.CONFIGS[args.config])
    spec = mesh_spec_box(cfg["dim"], cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], cfg["periodic"])
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    q_init, u_init, uh_init = dev(q0), dev(u0), dev(uh0)
    A, _, _ = alexander_dirk33()
    dii = 1.0 / A[0, 0]
    dt = inputs.cfl_dt(cfg)
    w = -dii * u_init
    q, u, uh = q_init.clone(), u_init.clone(), uh_init.clone()
    rtol = cfg["rtol"]

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    # elimination launch shapes per macro class from the autotuner, timed on
    # the linearisation at the initial state (outside the timed region)
    tuning = {}
    if args.set_tuning:
        shape = [int(v) for v in args.set_tuning.split(",")]
        for prec in (HDG_FP64, HDG_FP32):
            for k in range(ctx.class_count()):
                ctx.set_tuning(k, prec, *shape)
        tuning = dict(fixed=shape)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        ctx.linearize_stage(q_init, u_init, uh_init, w, dt, dii, norms=False)
        for name, prec in (("fp64", HDG_FP64), ("fp32", HDG_FP32)):
            ctx.autotune(prec, args.tune_cache)
            tuning[name] = [list(ctx.tuning(k, prec)) for k in range(ctx.class_count())]
        tuning["seconds"] = round(time.perf_counter() - t0, 2)

    # plain copy of 1 GiB: the reference for scaling HBM byte counters
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0 = ev(); dst.copy_(src); c1 = ev()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * src.numel() * 8 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    def run_variant(cond_prec, inner_prec, steps, warmup, use_learned=False, graph_steps=0, inner_its=5,
                    max_outer=300):
        """Warm-up stages, then `steps` timed stage solves from the same state."""
        marks = []
        drv = StageDriver(ctx, rtol=rtol, restart=30, inner_its=inner_its, max_outer=max_outer, condense_prec=cond_prec,
                          inner_prec=inner_prec, mark=lambda phase: marks.append((phase, ev())),
                          use_learned=use_learned, graph_steps=graph_steps)

        def stage():
            q.copy_(q_init); u.copy_(u_init); uh.copy_(uh_init)
            return drv.solve_stage(q, u, uh, w, dt, dii)

        for _ in range(warmup):
            stage()
        torch.cuda.synchronize()
        marks.clear()
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(stage())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phase_ms, cond_calls = {}, []
        for (ph, e), (_, e2) in zip(marks[:-1], marks[1:]):
            if ph == "end":
                continue
            t = e.elapsed_time(e2)
            phase_ms[ph] = phase_ms.get(ph, 0.0) + t / steps
            if ph == "condense":
                cond_calls.append(t)
        return dict(ms_per_stage=1e3 * wall / steps, phase_ms=phase_ms, cond_calls=cond_calls,
                    newton_its=infos[-1]["newton_its"], newton_res=infos[-1]["res_hist"],
                    outer=[[k["outer_its"] for k in inf["krylov"]] for inf in infos],
                    inner=[[k["inner_its"] for k in inf["krylov"]] for inf in infos],
                    fallbacks=[[k.get("fallbacks", 0) for k in inf["krylov"]] for inf in infos],
                    u=u.clone(), uh=uh.clone())

    def time_apply():
        """Global apply on its own (HBM-bound GEMV over the condensed blocks)."""
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
        return ea.elapsed_time(eb) / args.applies

    nb, nu, nm = ctx.n_b_macro, ctx.n_u_macro, ctx.n_macros
    flops = condense_flops(cfg, nu, nb) * nm
    main_prec = HDG_FP32 if args.plain_prec == "fp32" else HDG_FP64
    plain = run_variant(main_prec, main_prec, args.steps, args.warmup)
    apply_ms = time_apply()
    ms_step = plain["ms_per_stage"]
    phase_ms, cond_calls = plain["phase_ms"], plain["cond_calls"]
    newton_its, outer, inner = plain["newton_its"], plain["outer"], plain["inner"]
    variants = {}
    if not args.plain_only:
        mixed = run_variant(HDG_FP32, HDG_FP64, args.steps, args.warmup)
        cm = float(np.mean(mixed["cond_calls"]))
        apply32_ms = time_apply()
        du = float((mixed["u"] - plain["u"]).abs().max() / plain["u"].abs().max())
        duh = float((mixed["uh"] - plain["uh"]).abs().max() / plain["uh"].abs().max())
        variants["mixed_fp32_condense"] = dict(
            ms_per_stage=round(mixed["ms_per_stage"], 3),
            speedup_vs_plain=round(ms_step / mixed["ms_per_stage"], 3),
            phases_ms={k: round(v, 3) for k, v in mixed["phase_ms"].items()},
            newton_its=mixed["newton_its"], newton_res=mixed["newton_res"],
            fgmres=dict(outer_its=mixed["outer"], inner_its=mixed["inner"]),
            condense_ms=round(cm, 3), condense_tflops=round(flops / (cm * 1e-3) / 1e12, 3),
            condense_frac_fp32_peak=round(flops / (cm * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            stage_solution_rel_diff_vs_plain=dict(u=du, uhat=duh),
            apply_ms=round(apply32_ms, 4),
            apply_gbs=round((4.0 * nm * nb * nb + 16.0 * nm * nb + 8.0 * ctx.n_glob) / (apply32_ms * 1e-3) / 1e9, 1))
        # *_inner_graph: the condensed operator for the outer FGMRES, its FP32
        # or BF16 copy for the inner GMRES of the preconditioner
        for name, cp, ip in (("plain_fp64_graph", HDG_FP64, HDG_FP64),
                             ("mixed_fp32_condense_graph", HDG_FP32, HDG_FP64),
                             ("fp64_condense_fp32_inner_graph", HDG_FP64, HDG_FP32),
                             ("fp64_condense_bf16_inner_graph", HDG_FP64, HDG_BF16),
                             ("mixed_fp32_condense_bf16_inner_graph", HDG_FP32, HDG_BF16)):
            gv = run_variant(cp, ip, args.steps, args.warmup, graph_steps=args.graph_steps)
            variants[name] = dict(
                ms_per_stage=round(gv["ms_per_stage"], 3), speedup_vs_plain=round(ms_step / gv["ms_per_stage"], 3),
                phases_ms={k: round(v, 3) for k, v in gv["phase_ms"].items()}, newton_its=gv["newton_its"],
                fgmres=dict(outer_its=gv["outer"], inner_its=gv["inner"]), graph_steps=args.graph_steps,
                stage_solution_rel_diff_vs_plain=dict(
                    u=float((gv["u"] - plain["u"]).abs().max() / plain["u"].abs().max()),
                    uhat=float((gv["uh"] - plain["uh"]).abs().max() / plain["uh"].abs().max())))
        # single-level GMRES: the face-block inverse of A_uh,uh alone as the
        # preconditioner (no inner GMRES), the comparison of the paper's Table 2
        sl = run_variant(HDG_FP64, HDG_FP64, args.steps, args.warmup, inner_its=0, max_outer=5000,
                         graph_steps=args.graph_steps)
        variants["single_level_gmres_fp64_graph"] = dict(
            ms_per_stage=round(sl["ms_per_stage"], 3), speedup_vs_plain=round(ms_step / sl["ms_per_stage"], 3),
            phases_ms={k: round(v, 3) for k, v in sl["phase_ms"].items()}, newton_its=sl["newton_its"],
            fgmres=dict(outer_its=sl["outer"], inner_its=sl["inner"]),
            multi_level_outer_its=outer, multi_level_inner_its=inner,
            stage_solution_rel_diff_vs_plain=dict(
                u=float((sl["u"] - plain["u"]).abs().max() / plain["u"].abs().max()),
                uhat=float((sl["uh"] - plain["uh"]).abs().max() / plain["uh"].abs().max())))
        if not args.no_learned:
            lrn = train_learned(ctx, cfg, dev, dii, dt, args)
            ml = run_variant(HDG_FP32, HDG_FP64, args.steps, args.warmup, use_learned=True)
            variants["mixed_fp32_condense_learned"] = dict(
                ms_per_stage=round(ml["ms_per_stage"], 3),
                speedup_vs_plain=round(ms_step / ml["ms_per_stage"], 3),
                phases_ms={k: round(v, 3) for k, v in ml["phase_ms"].items()},
                newton_its=ml["newton_its"], newton_res=ml["newton_res"],
                fgmres=dict(outer_its=ml["outer"], inner_its=ml["inner"], fallbacks=ml["fallbacks"]),
                stage_solution_rel_diff_vs_plain=dict(
                    u=float((ml["u"] - plain["u"]).abs().max() / plain["u"].abs().max()),
                    uhat=float((ml["uh"] - plain["uh"]).abs().max() / plain["uh"].abs().max())),
                training=lrn)
            ctx.learned_bind(None)
    apply_bytes = 8.0 * nm * nb * nb + 8.0 * nm * nb + 8.0 * nm * nb + 8.0 * ctx.n_glob
    apply_gbs = apply_bytes / (apply_ms * 1e-3) / 1e9
    cond_ms = float(np.mean(cond_calls))
    cond_tflops = flops / (cond_ms * 1e-3) / 1e12
    # dominant work: hdg_condense, one launch sequence per Newton step (MFMA-bound)
    traffic = CONDENSE_TRAFFIC["bytes"] if sources_sha() == CONDENSE_TRAFFIC["sha"] else None
    peak = PEAK_FP64_TFLOPS if main_prec == HDG_FP64 else PEAK_FP32_TFLOPS
    if main_prec != HDG_FP64:
        traffic = None
    roofline = dict(bound="mfma", achieved=round(cond_tflops, 3), peak=peak, unit="TFLOP/s",
                    frac=round(cond_tflops / peak, 4), traffic=traffic,
                    kernel="hdg_condense: k_form + batched FP64 elimination (k_panel, k_uinv, k_u12, k_linv2, "
                           "k_u12lin, k_gemm) + face-preconditioner factorisation",
                    flops_per_launch=flops, ms_per_launch=round(cond_ms, 3), launches=len(cond_calls))
    out = dict(metric=METRIC, value=round(ms_step, 3), unit="ms/DIRK-stage", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=False, scaling="weak",
               vs_baseline=None, dtype="f64" if main_prec == HDG_FP64 else "f32", data="synthetic",
               config=dict(workload=f"{args.config}: Taylor-Green 24^3 periodic hexes on [-pi,pi]^3, 3^3-element "
                                    f"macros (512), p=2, Mach 0.1, Re 1600, 1e-4 seeded noise; DIRK(3,3) stage 1 "
                                    f"solved by Newton to max(1e-10, 1e-8 |R0|), FGMRES(30) rtol {rtol} with "
                                    f"5 inner GMRES steps",
                           n_macros=nm, n_u_macro=nu, n_b_macro=nb, n_glob=ctx.n_glob,
                           variant="plain FP64" if main_prec == HDG_FP64 else "FP32 condensation"),
               phases_ms={k: round(v, 3) for k, v in phase_ms.items()},
               newton_its=newton_its, newton_res=plain["newton_res"],
               fgmres=dict(outer_its=outer, inner_its=inner),
               condense_tflops=round(cond_tflops, 3), condense_ms=round(cond_ms, 3),
               apply_ms=round(apply_ms, 4), apply_gbs=round(apply_gbs, 1),
               apply_frac_hbm=round(apply_gbs / PEAK_HBM_GBS, 4), copy_gbs=round(copy_gbs, 1),
               roofline=roofline, variants=variants, autotune=tuning)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, newton_its)
    # the other workloads need the device memory of the 24^3 workspace
    ctx.close()

    def free_device_memory():
        gc.collect()
        torch.cuda.empty_cache()

    free_device_memory()
    if not args.plain_only and not args.no_uneven:
        uneven_variant(args, dev, variants)
        free_device_memory()
    if args.learned_p3:
        learned_p3_variant(args, dev, variants)
        free_device_memory()
    if args.first_layer:
        first_layer_variant(args, dev, variants)
        free_device_memory()
    if args.tgv_eps > 0:
        tgv_dissipation_variant(args, dev, variants)
        free_device_memory()
    if args.big_steps > 0:
        big_variant(args, dev, variants)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
