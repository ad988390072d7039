"""Benchmark of the macro-element HDG hot path on one MI355X.

Headline: Newton steps of the first DIRK(3,3) stage on the largest
single-GPU workload, Taylor-Green 48^3 periodic hexes on [-pi, pi]^3 with
macros of 4^3 elements (1728 macros), p = 2, Mach 0.1, Re 1600, seeded 1e-4
noise, dt = CFL h / (V0 (p+1)), CFL = 1, plain FP64.  One timed step is one
pass of the whole path from the same initial state: linearise -> second-layer
condensation (in chunks of macros, keeping FP32 copies of the S factors of
the leading chunks for the recovery) -> FGMRES(30) to rtol 1e-8 with 5 inner
GMRES steps -> local recovery -> update.  Extra keys: the mixed-precision
path on the same workload, the 24^3 workload (3^3-element macros, 512) with
its variants (whole stages), and the CPU oracle on a bounded sample.

Prints one JSON line.  Per-phase times come from HIP events recorded on the
library's stream around each C-ABI call; the global apply is also timed on
its own over repeated calls (HBM roofline).
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
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

# HBM bytes per hdg_condense call of the FP64 path, per workload and macros
# per chunk, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by
# what the counters read for a 1 GiB device copy in the same run
# (profiles/newton_step_tgv48_m4_p2_fp64.md), valid only while the kernel
# sources hash to `sha`.
CONDENSE_TRAFFIC = {"sha": "d982f9e5811eff96", "tgv48_m4_p2/122": 20.69e12}
CONDENSE_SOURCES = ("k_form.hip", "k_lu.hip", "k_backsolve.hip", "k_krylov.hip")


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
    from paper_2402_11361_amd.hdg import HDG_FP32, HDG_FP64, Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv48_m4_p2"])
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    free, _ = torch.cuda.mem_get_info()
    ctx.set_chunk_buffers(args.chunk_slots)
    per = ctx.fit_chunking(free - (8 << 30))
    store = None
    if args.factor_store != "none" and per:
        per = max(1, int(per * args.store_chunk_frac))
        ctx.set_chunking(per)
        store = dict(prec=args.factor_store,
                     macros=ctx.fit_factor_store(free - (8 << 30), HDG_FP32 if args.factor_store == "fp32" else HDG_FP64))
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    q, u, uh = dev_fn(q0), dev_fn(u0), dev_fn(uh0)
    dt = inputs.cfl_dt(cfg)
    dii = 1.0 / 0.435866521508459
    ctx.linearize_stage(q, u, uh, -dii * u, dt, dii, norms=False)
    if args.set_tuning:
        ctx.set_tuning(0, HDG_FP32, *[int(v) for v in args.set_tuning.split(",")])
    else:
        ctx.autotune(HDG_FP32, args.tune_cache)
    learned = None
    if args.big_learned:
        # trained on other seeded states (seeds 1..), the timed run starts from seed 0
        learned = train_learned(ctx, cfg, dev_fn, dii, dt, args)
        print(f"[bench] 48^3 learned stage: {learned}", file=sys.stderr, flush=True)
    drv = StageDriver(ctx, rtol=cfg["rtol"], condense_prec=HDG_FP32, inner_prec=HDG_FP32,
                      graph_steps=args.graph_steps, use_learned=args.big_learned)
    steps = []
    for n in range(args.big_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = drv.step(q, u, uh, dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        steps.append(dict(ms=round(1e3 * wall, 1), ms_per_stage=round(1e3 * wall / len(infos), 1),
                          newton_its=[i["newton_its"] for i in infos],
                          fgmres_outer=[[k["outer_its"] for k in i["krylov"]] for i in infos],
                          learned_fallbacks=sum(k.get("fallbacks", 0) for i in infos for k in i["krylov"])))
        print(f"[bench] 48^3 time step {n + 1}: {steps[-1]['ms']} ms", file=sys.stderr, flush=True)
    ms = [st["ms"] for st in steps]
    variants["tgv48_chunked_fp32_graph_steps"] = dict(
        workload="48^3 periodic Taylor-Green, 4^3-element macros (1728), p=2, "
                 f"n_glob {ctx.n_glob}; {per} macros per condensation chunk; FP32 condensation refined by Newton, "
                 "FP32 inner operator, graph-captured FGMRES steps"
                 + ("; learned coarse correction judged by the plain preconditioner" if learned else ""),
        macros_per_chunk=per, chunk_slots=args.chunk_slots, factor_store=store, workspace_gb=round(ctx.workspace_bytes / 1e9, 1), learned=learned,
        ms_per_step_mean=round(float(np.mean(ms)), 1) if ms else None,
        ms_per_stage_mean=round(float(np.mean(ms)) / 3, 1) if ms else None, time_steps=steps)
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


def nested_variant(args, dev_fn, variants):
    """Nested hybridisation inside a macro (third condensation layer) on the
    24^3 Taylor-Green workload at p = 2: every element hybridised on its own
    (one element per macro, 13824 elements), element-level condensation,
    then blocks of 3^3 elements whose internal-face traces (2430 per block)
    are eliminated.  Times per step and the skeleton size, next to the C0
    macro-element method on 3^3-element macros of the same mesh."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.hdg import HDG_FP64, Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv24_m3_p2"])
    cfg["m"] = 1
    spec = mesh_spec_box(3, cfg["n_elem"], 1, cfg["p"], cfg["lo"], cfg["hi"], True)
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    dii = 1.0 / 0.435866521508459
    dt = inputs.cfl_dt(cfg)
    u = dev_fn(u0)
    bhat = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    M = 3
    nb, nI, nB = ctx.nested_dims(M)
    Ag = torch.zeros(nb * nB * nB, dtype=torch.float64, device="cuda")
    bg = torch.zeros(nb * nB, dtype=torch.float64, device="cuda")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    ms_lin = timed(lambda: ctx.linearize_stage(dev_fn(q0), u, dev_fn(uh0), -dii * u, dt, dii, norms=False), 2)
    ms_el = timed(lambda: ctx.condense(bhat, HDG_FP64), 2)
    ms_nest = timed(lambda: ctx.condense_nested(M, Ag, bg), 2)
    x = torch.zeros(ctx.n_glob, dtype=torch.float64, device="cuda")
    dq = torch.zeros(ctx.n_q_tot, dtype=torch.float64, device="cuda")
    du = torch.zeros(ctx.n_u_tot, dtype=torch.float64, device="cuda")
    info = {}

    def solve():
        info.update(ctx.nested_solve(M, x, rtol=cfg["rtol"], restart=30, max_outer=400, inner_its=5))

    ms_solve = timed(solve, 2)
    ms_back = timed(lambda: ctx.local_backsolve(x, dq, du), 2)
    print(f"[bench] nested: linearise {ms_lin:.1f} ms, element condensation {ms_el:.1f} ms, "
          f"block condensation {ms_nest:.1f} ms, skeleton FGMRES + internal traces {ms_solve:.1f} ms "
          f"({info['outer_its']} outer), element recovery {ms_back:.1f} ms", file=sys.stderr, flush=True)
    n_skel_elem = ctx.n_glob - nb * nI
    variants["nested_hdg_in_macro_fp64"] = dict(
        workload="24^3 periodic Taylor-Green, p=2, every element hybridised (13824 elements), blocks of 3^3 "
                 "elements (512) whose internal-face traces are eliminated",
        ms_linearize=round(ms_lin, 1), ms_element_condense=round(ms_el, 1), ms_block_condense=round(ms_nest, 1),
        ms_skeleton_solve_and_internal_traces=round(ms_solve, 1), ms_element_recovery=round(ms_back, 1),
        skeleton_fgmres=dict(outer_its=info["outer_its"], inner_its=info["inner_its"], rtol=cfg["rtol"]),
        ms_newton_step=round(ms_lin + ms_el + ms_nest + ms_solve + ms_back, 1),
        element_trace_unknowns=ctx.n_glob, internal_per_block=nI, boundary_per_block=nB,
        skeleton_unknowns=n_skel_elem, blocks=nb)
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
    at p = 3 (512 macros, chunked FP32 condensation): pairs harvested from
    plain solves on the states of seeds 100, 101, ... (training), evaluated on
    the held-out states of seeds 200, 201, ... (first Newton step): plain
    multi-level preconditioner, learned stage judged by it (fallback on), and
    the learned stage kept for the whole solve (no fallback)."""
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

    train_seeds = list(range(100, 100 + args.learned_train_seeds))
    eval_seeds = list(range(200, 200 + args.learned_eval_seeds))
    t0 = time.perf_counter()
    cc = CoarseCorrection(ctx, hidden=256, max_batch=1024, seed=0, neighbours=args.learned_neighbours)
    for s_ in train_seeds:
        condense_state(s_)
        cc.harvest(bhat, n_vectors=args.train_vectors, inner_prec=HDG_FP32)
        print(f"[bench] p=3 learned: seed {s_} harvested, {cc.n_pairs()} pairs", file=sys.stderr, flush=True)
    X, T = torch.cat(cc.X), torch.cat(cc.T)
    loss0 = cc.eval_loss(X, T)
    cc.train(epochs=args.train_epochs, lr=1e-3, batch=1024)
    loss1 = cc.eval_loss(X, T)
    cc.bind()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] p=3 learned: {cc.n_pairs()} pairs, loss {loss0:.3e} -> {loss1:.3e}", file=sys.stderr, flush=True)
    evals = {}
    for s_ in eval_seeds:
        condense_state(s_)
        ev = {}
        for name, lrn, nofb in (("plain", False, False), ("learned", True, False), ("learned_no_fallback", True, True)):
            x = torch.zeros_like(bhat)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            info = ctx.fgmres_solve(bhat, x, rtol=cfg["rtol"], restart=30, max_outer=300, inner_its=5,
                                    inner_prec=HDG_FP32, use_learned=lrn, no_fallback=nofb, allow_noconv=True)
            torch.cuda.synchronize()
            ev[name] = dict(outer_its=info["outer_its"], inner_its=info["inner_its"],
                            ms=round(1e3 * (time.perf_counter() - ts), 1), fallbacks=info["fallbacks"],
                            converged=info["converged"])
        evals[f"seed_{s_}"] = ev
        print(f"[bench] p=3 learned: held-out seed {s_}: {ev}", file=sys.stderr, flush=True)
    key = "tgv32_m4_p3_learned" + ("_neighbours" if args.learned_neighbours else "")
    variants[key] = dict(
        workload=f"32^3 periodic Taylor-Green, 4^3-element macros (512), p=3, n_glob {ctx.n_glob}; chunked FP32 "
                 f"condensation ({per} macros per chunk); train on seeds {train_seeds}, evaluate on held-out seeds "
                 f"{eval_seeds}; network inputs: own macro" + (" and its face neighbours" if args.learned_neighbours
                                                              else ""),
        n_in=cc.n_in,
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


def cpu_baseline(cfg, gpu, n_sample=1, single_thread=False):
    """Oracle leg on a bounded sample of the headline workload: route-B
    condensation (LAPACK), the condensed apply and the local recovery of
    n_sample macros, and the FGMRES vector work (two classical Gram-Schmidt
    passes) on full-size trace vectors, scaled to one Newton step of the whole
    mesh with the GPU's iteration counts.  The complex-step linearisation of
    the sampled macros is timed on its own (not a fair baseline: it
    differentiates the residual column group by column group).  Returns the
    summary and the oracle's condensed blocks of the sampled macros."""
    from oracle.mesh import box_mesh
    from oracle.physics import Phys
    from oracle.system import System
    from oracle import dirk, krylov
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
    S.geo(S.mclass[0])            # reference matrices of the class (set-up, not timed)
    t0 = time.perf_counter()
    lin = S.linearize(q, u, uh, w=w, dt=dt, dii=dii, macros=sample)
    t1 = time.perf_counter()
    con = S.condense(lin, "B")
    t2 = time.perf_counter()
    x = np.random.default_rng(5).uniform(-1, 1, M.n_glob)
    S.backsolve(lin, con, x)
    t3 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        for i in sample:
            con[i]["Ahat"] @ x[M.macro_trace_index(i)]
    t4 = time.perf_counter()
    # FGMRES vector work: CGS2 of one new vector against j + 1 basis vectors
    # for j = 0 .. outer - 1 (the GPU's outer iterations), plus one face-block
    # preconditioner solve per inner step is left out (small next to these)
    n = M.n_glob
    outer = max(gpu["outer_its"], 1)
    jmax = min(outer, 30)
    V = np.random.default_rng(6).standard_normal((jmax + 1, n))
    wv = np.random.default_rng(7).standard_normal(n)
    t5 = time.perf_counter()
    for j in range(0, jmax, 5):
        krylov._cgs2(V, wv, j)
    t6 = time.perf_counter()
    cgs_per_step = (t6 - t5) / len(range(0, jmax, 5))   # mean over the basis sizes of a cycle, sampled every 5
    nm = M.n_macros
    per_cond = (t2 - t1) / n_sample
    per_back = (t3 - t2) / n_sample
    per_apply = (t4 - t3) / (reps * n_sample)
    applies = gpu["applies"]
    ms = 1e3 * (per_cond * nm + per_back * nm + per_apply * nm * applies + cgs_per_step * outer)
    out = dict(value=round(ms, 1), unit="ms/Newton-step (extrapolated from the sample; linearisation separate)",
               cores=1 if single_thread else blas_threads(), kind="oracle",
               sample=f"{n_sample} of {nm} macros of the headline workload, first Newton step of DIRK stage 1: "
                      f"route-B condensation {1e3 * per_cond:.0f} ms/macro, recovery {1e3 * per_back:.1f} ms/macro, "
                      f"condensed apply {1e3 * per_apply:.2f} ms/macro x {applies} applies, CGS2 on "
                      f"{n}-vectors {1e3 * cgs_per_step:.0f} ms per outer step (x{outer}); scaled to {nm} macros",
               phases_ms=dict(condense=round(1e3 * per_cond * nm, 1), backsolve=round(1e3 * per_back * nm, 1),
                              apply=round(1e3 * per_apply * nm * applies, 1),
                              krylov_vectors=round(1e3 * cgs_per_step * outer, 1)),
               linearisation_not_a_fair_baseline=dict(
                   ms_per_macro=round(1e3 * (t1 - t0) / n_sample, 1),
                   ms_per_newton_step_extrapolated=round(1e3 * (t1 - t0) / n_sample * nm, 1),
                   note="complex-step Jacobian of the residual, column group by column group"))
    blocks = {i: (con[i]["Ahat"], con[i]["bhat"]) for i in sample}
    return out, blocks


def _rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


class NewtonBench:
    """Times whole Newton steps (linearise -> condense -> FGMRES -> recovery ->
    update) from one initial state on one context, with HIP events on the
    library's stream around each phase."""

    def __init__(self, ctx, stream, state, w, dt, dii, rtol):
        import torch
        self.t, self.ctx, self.stream = torch, ctx, stream
        self.q0, self.u0, self.uh0 = state
        self.w, self.dt, self.dii, self.rtol = w, dt, dii, rtol
        dev = dict(dtype=torch.float64, device="cuda")
        self.q, self.u, self.uh = self.q0.clone(), self.u0.clone(), self.uh0.clone()
        self.bhat = torch.zeros(ctx.n_glob, **dev)
        self.x = torch.zeros(ctx.n_glob, **dev)
        self.dq = torch.zeros(ctx.n_q_tot, **dev)
        self.du = torch.zeros(ctx.n_u_tot, **dev)

    def ev(self):
        e = self.t.cuda.Event(enable_timing=True)
        e.record(self.stream)
        return e

    def step(self, marks, cond_prec, inner_prec, graph_steps=0, use_learned=False):
        ctx = self.ctx
        self.q.copy_(self.q0); self.u.copy_(self.u0); self.uh.copy_(self.uh0)
        marks.append(("linearize", self.ev()))
        ctx.linearize_stage(self.q, self.u, self.uh, self.w, self.dt, self.dii, norms=False)
        marks.append(("condense", self.ev()))
        ctx.condense(self.bhat, cond_prec)
        marks.append(("fgmres", self.ev()))
        self.x.zero_()
        info = ctx.fgmres_solve(self.bhat, self.x, rtol=self.rtol, restart=30, max_outer=300, inner_its=5,
                                inner_prec=inner_prec, graph_steps=graph_steps, use_learned=use_learned)
        marks.append(("backsolve", self.ev()))
        ctx.local_backsolve(self.x, self.dq, self.du)
        marks.append(("update", self.ev()))
        ctx.axpy(1.0, self.dq, self.q)
        ctx.axpy(1.0, self.du, self.u)
        ctx.axpy(1.0, self.x, self.uh)
        marks.append(("end", self.ev()))
        return info

    def run(self, steps, warmup, cond_prec, inner_prec, graph_steps=0, use_learned=False, progress=None):
        marks = []
        for k in range(warmup):
            self.step(marks, cond_prec, inner_prec, graph_steps, use_learned)
            if progress:
                progress(f"warm-up step {k + 1}/{warmup}")
        self.t.cuda.synchronize()
        marks.clear()
        infos = []
        t0 = time.perf_counter()
        for k in range(steps):
            infos.append(self.step(marks, cond_prec, inner_prec, graph_steps, use_learned))
            if progress:
                progress(f"timed step {k + 1}/{steps}")
        self.t.cuda.synchronize()
        wall = time.perf_counter() - t0
        phase_ms, cond_calls = {}, []
        for (ph, e), (_, e2) in zip(marks[:-1], marks[1:]):
            if ph == "end":
                continue
            dtm = e.elapsed_time(e2)
            phase_ms[ph] = phase_ms.get(ph, 0.0) + dtm / steps
            if ph == "condense":
                cond_calls.append(dtm)
        return dict(ms_per_step=1e3 * wall / steps, phase_ms=phase_ms, cond_calls=cond_calls,
                    outer=[k["outer_its"] for k in infos], inner=[k["inner_its"] for k in infos],
                    fallbacks=[k["fallbacks"] for k in infos])

    def newton_reduction(self):
        """||R_F|| before and after one step from the initial state (the state
        the last step left)."""
        import numpy as _np
        r1 = self.ctx.linearize_stage(self.q, self.u, self.uh, self.w, self.dt, self.dii)
        r0 = self.ctx.linearize_stage(self.q0, self.u0, self.uh0, self.w, self.dt, self.dii)
        return float(_np.sqrt(_np.sum(r0 ** 2))), float(_np.sqrt(_np.sum(r1 ** 2)))


def time_apply(ctx, stream, reps):
    """Global apply on its own (HBM-bound GEMV over the condensed blocks)."""
    import torch
    xa = torch.randn(ctx.n_glob, dtype=torch.float64, device="cuda")
    ya = torch.zeros_like(xa)
    for _ in range(3):
        ctx.apply_global(xa, ya)
    torch.cuda.synchronize()
    ea = torch.cuda.Event(enable_timing=True); ea.record(stream)
    for _ in range(reps):
        ctx.apply_global(xa, ya)
    eb = torch.cuda.Event(enable_timing=True); eb.record(stream)
    torch.cuda.synchronize()
    return ea.elapsed_time(eb) / reps


def apply_bytes(ctx, w):
    """Algorithmic bytes of one global apply: the condensed blocks (w bytes per
    entry), the gathered and partial local vectors and the output."""
    nb = np.diff(np.asarray(ctx.b_off, dtype=np.float64))
    return float(w * (nb * nb).sum() + 16.0 * nb.sum() + 8.0 * ctx.n_glob)


def c2_variants(args, dev, variants, say):
    """Whole DIRK-stage solves (Newton to max(1e-10, 1e-8 ||R^0||)) on the 24^3
    workload: plain FP64, FP32 condensation with the BF16 inner operator and
    graph-captured FGMRES steps, and the same with the learned coarse
    correction (judged by the plain preconditioner)."""
    import torch
    from paper_2402_11361_amd import inputs
    from paper_2402_11361_amd.driver import StageDriver, alexander_dirk33
    from paper_2402_11361_amd.hdg import HDG_BF16, HDG_FP32, HDG_FP64, Context, mesh_spec_box
    cfg = dict(inputs.CONFIGS["tgv24_m3_p2"])
    spec = mesh_spec_box(3, cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], True)
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    ctx.bind_workspace()
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    q_i, u_i, uh_i = dev(q0), dev(u0), dev(uh0)
    A, _, _ = alexander_dirk33()
    dii = 1.0 / A[0, 0]
    dt = inputs.cfl_dt(cfg)
    w = -dii * u_i
    q, u, uh = q_i.clone(), u_i.clone(), uh_i.clone()
    ctx.linearize_stage(q_i, u_i, uh_i, w, dt, dii, norms=False)
    tuning = {}
    for name, prec in (("fp64", HDG_FP64), ("fp32", HDG_FP32)):
        if args.set_tuning:
            ctx.set_tuning(0, prec, *[int(v) for v in args.set_tuning.split(",")])
        else:
            ctx.autotune(prec, args.tune_cache)
        tuning[name] = list(ctx.tuning(0, prec))
    nm, nu, nb = ctx.n_macros, ctx.n_u_macro, ctx.n_b_macro
    flops = condense_flops(cfg, nu, nb) * nm
    out = dict(workload="tgv24_m3_p2: Taylor-Green 24^3 periodic hexes, 3^3-element macros (512), p=2, Mach 0.1, "
                        "Re 1600, 1e-4 seeded noise; DIRK(3,3) stage 1 solved by Newton to max(1e-10, 1e-8 |R0|)",
               n_macros=nm, n_u_macro=nu, n_b_macro=nb, n_glob=ctx.n_glob, condense_flops=flops, autotune=tuning)
    ref = None

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    def stage_runs(name, cond_prec, inner_prec, graph_steps, use_learned=False):
        marks = []
        drv = StageDriver(ctx, rtol=cfg["rtol"], condense_prec=cond_prec, inner_prec=inner_prec,
                          graph_steps=graph_steps, use_learned=use_learned,
                          mark=lambda ph: marks.append((ph, ev())))
        walls, info = [], None
        for rep in range(1 + args.c2_stages):
            q.copy_(q_i); u.copy_(u_i); uh.copy_(uh_i)
            marks.clear()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = drv.solve_stage(q, u, uh, w, dt, dii)
            torch.cuda.synchronize()
            if rep > 0:
                walls.append(time.perf_counter() - t0)
        cond = [e.elapsed_time(e2) for (ph, e), (_, e2) in zip(marks[:-1], marks[1:]) if ph == "condense"]
        cm = float(np.mean(cond))
        peak = {HDG_FP64: PEAK_FP64_TFLOPS, HDG_FP32: PEAK_FP32_TFLOPS}.get(cond_prec, PEAK_BF16_TFLOPS)
        say(f"c2 {name}: {1e3 * np.mean(walls):.1f} ms per stage")
        return dict(ms_per_stage=round(1e3 * float(np.mean(walls)), 3), stages_timed=len(walls),
                    newton_its=info["newton_its"], newton_res=info["res_hist"],
                    fgmres_outer=[k["outer_its"] for k in info["krylov"]],
                    fallbacks=[k["fallbacks"] for k in info["krylov"]],
                    condense_ms=round(cm, 3), condense_tflops=round(flops / (cm * 1e-3) / 1e12, 3),
                    condense_frac_peak=round(flops / (cm * 1e-3) / 1e12 / peak, 4))

    plain = stage_runs("plain_fp64", HDG_FP64, HDG_FP64, 0)
    u_ref, uh_ref = u.clone(), uh.clone()
    out["plain_fp64"] = plain
    out["plain_fp64"]["apply_ms"] = round(time_apply(ctx, stream, args.applies), 4)
    for name, cp, ip, gs in (("mixed_fp32_condense_bf16_inner_graph", HDG_FP32, HDG_BF16, args.graph_steps),
                             ("mixed_bf16_update_condense_bf16_inner_graph", HDG_BF16, HDG_BF16, args.graph_steps)):
        r = stage_runs(name, cp, ip, gs)
        r["speedup_vs_plain"] = round(plain["ms_per_stage"] / r["ms_per_stage"], 3)
        r["stage_solution_rel_diff_vs_plain_fp64"] = dict(u=_rel_t(u, u_ref), uhat=_rel_t(uh, uh_ref))
        out[name] = r
    if not args.no_learned:
        lrn = train_learned(ctx, cfg, dev, dii, dt, args)
        r = stage_runs("mixed_fp32_condense_learned_graph", HDG_FP32, HDG_BF16, args.graph_steps, use_learned=True)
        r["speedup_vs_plain"] = round(plain["ms_per_stage"] / r["ms_per_stage"], 3)
        r["stage_solution_rel_diff_vs_plain_fp64"] = dict(u=_rel_t(u, u_ref), uhat=_rel_t(uh, uh_ref))
        r["training"] = lrn
        out["mixed_fp32_condense_learned_graph"] = r
        ctx.learned_bind(None)
    variants["tgv24_m3_p2_stages"] = out
    ctx.close()


def _rel_t(a, b):
    return float((a - b).abs().max() / b.abs().max())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="tgv48_m4_p2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--factor-store", default="fp32", choices=("none", "fp32", "fp64"),
                    help="keep the S factors of the leading chunks for the recovery (FP32 copies refined in FP64, "
                         "or FP64)")
    ap.add_argument("--store-chunk-frac", type=float, default=0.35,
                    help="with --factor-store: chunk size as a fraction of the largest that fits")
    ap.add_argument("--progress", action="store_true",
                    help="a line per finished condensation/recovery chunk (for profiled runs; syncs per chunk)")
    ap.add_argument("--chunk-slots", type=int, default=1, choices=(1, 2),
                    help="chunk slots of the condensation buffer (2: the next chunk is formed beside the "
                         "elimination of this one)")
    ap.add_argument("--cpu-sample", type=int, default=1, help="macros of the CPU oracle's sample")
    ap.add_argument("--cpu-single-thread", action="store_true",
                    help="also time the oracle's sample with one BLAS thread")
    ap.add_argument("--applies", type=int, default=20)
    ap.add_argument("--headline-only", action="store_true", help="time only the plain FP64 headline")
    ap.add_argument("--mixed-steps", type=int, default=2, help="timed Newton steps of the mixed-precision variant")
    ap.add_argument("--c2-stages", type=int, default=1, help="timed stages per 24^3 variant (0: skip them)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-correction variant")
    ap.add_argument("--uneven", action="store_true", help="also time the uneven-macro 32^3 variant")
    ap.add_argument("--graph-steps", type=int, default=10, help="FGMRES steps per captured HIP graph")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default elimination launch shapes")
    ap.add_argument("--learned-p3", action="store_true",
                    help="also train and evaluate the learned correction on the 32^3 p=3 workload")
    ap.add_argument("--big-steps", type=int, default=0,
                    help="also time this many DIRK(3,3) steps of the 48^3 workload (chunked FP32 condensation)")
    ap.add_argument("--big-learned", action="store_true",
                    help="--big-steps with the learned coarse correction (trained first on other seeded states)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2402_11361_amd", "tune_mi355x.txt"),
                    help="text file of earlier autotuner choices (read; new choices are appended); the default holds "
                         "the choices measured on MI355X for the bench workloads")
    ap.add_argument("--plain-prec", choices=("fp64", "fp32"), default="fp64",
                    help="condensation precision of the headline (profiling of the FP32 path)")
    ap.add_argument("--uneven-only", action="store_true",
                    help="time only the uneven-macro 32^3 variant (profiling); prints its JSON")
    ap.add_argument("--set-tuning", default=None, metavar="TPW,WIDE,LOOK",
                    help="fixed elimination launch shape for every class instead of the autotuner (profiling)")
    ap.add_argument("--nested", action="store_true",
                    help="also time the nested (third-layer) condensation on the 24^3 workload")
    ap.add_argument("--first-layer", action="store_true",
                    help="also time the standard (first-layer) condensation against the second layer at 24^3")
    ap.add_argument("--tgv-eps", type=float, default=0.0, metavar="T_END",
                    help="also integrate the Re = 100 Taylor-Green flow to t/t_c = T_END on (m,p) = (3,2) and (2,3) "
                         "and report the dissipation rate")
    ap.add_argument("--learned-train-seeds", type=int, default=1, help="training states of --learned-p3 (seeds 100..)")
    ap.add_argument("--learned-eval-seeds", type=int, default=1, help="held-out states of --learned-p3 (seeds 200..)")
    ap.add_argument("--learned-neighbours", action="store_true",
                    help="--learned-p3 with a network that also sees the face neighbours' coarse coefficients")
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
    from paper_2402_11361_amd.driver import alexander_dirk33
    from paper_2402_11361_amd.hdg import HDG_FP32, HDG_FP64, Context, mesh_spec_box
    t_start = time.perf_counter()

    def say(msg):
        print(f"[bench {time.perf_counter() - t_start:7.1f}s] {msg}", file=sys.stderr, flush=True)

    dev = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda")
    if args.uneven_only:
        variants = {}
        uneven_variant(args, dev, variants)
        print(json.dumps(dict(metric=METRIC, unit="ms/DIRK-stage", n_gpus=1, data="synthetic", variants=variants)),
              flush=True)
        return
    cfg = dict(inputs.CONFIGS[args.config])
    spec = mesh_spec_box(cfg["dim"], cfg["n_elem"], cfg["m"], cfg["p"], cfg["lo"], cfg["hi"], cfg["periodic"])
    stream = torch.cuda.current_stream()
    ctx = Context.from_mesh_spec(spec, Re=cfg["Re"], Mach=cfg["mach"], stream=stream.cuda_stream)
    free, _ = torch.cuda.mem_get_info()
    ctx.set_chunk_buffers(args.chunk_slots)
    per_chunk = ctx.fit_chunking(free - (8 << 30))
    store = None
    if args.factor_store != "none" and per_chunk:
        # smaller chunks leave room for the factor store of the leading chunks
        per_chunk = max(1, int(per_chunk * args.store_chunk_frac))
        ctx.set_chunking(per_chunk)
        sprec = HDG_FP32 if args.factor_store == "fp32" else HDG_FP64
        store = dict(prec=args.factor_store, macros=ctx.fit_factor_store(free - (8 << 30), sprec))
    ctx.bind_workspace()
    if args.progress:
        ctx.set_progress(True)
    say(f"{args.config}: {ctx.n_macros} macros, n_glob {ctx.n_glob}, workspace {ctx.workspace_bytes / 1e9:.1f} GB, "
        f"{per_chunk or ctx.n_macros} macros per condensation chunk, factor store {store}")
    u0, q0, uh0 = workload_arrays(ctx, cfg)
    q_init, u_init, uh_init = dev(q0), dev(u0), dev(uh0)
    A, _, _ = alexander_dirk33()
    dii = 1.0 / A[0, 0]
    dt = inputs.cfl_dt(cfg)
    w = -dii * u_init
    main_prec = HDG_FP32 if args.plain_prec == "fp32" else HDG_FP64

    # elimination launch shapes from the autotuner, timed on the linearisation
    # at the initial state (outside the timed region)
    tuning = {}
    ctx.linearize_stage(q_init, u_init, uh_init, w, dt, dii, norms=False)
    if args.set_tuning:
        shape = [int(v) for v in args.set_tuning.split(",")]
        for prec in (HDG_FP64, HDG_FP32):
            for k in range(ctx.class_count()):
                ctx.set_tuning(k, prec, *shape)
        tuning = dict(fixed=shape)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        precs = (("fp64", HDG_FP64),) if args.headline_only else (("fp64", HDG_FP64), ("fp32", HDG_FP32))
        for name, prec in precs:
            ctx.autotune(prec, args.tune_cache)
            tuning[name] = [list(ctx.tuning(k, prec)) for k in range(ctx.class_count())]
        tuning["seconds"] = round(time.perf_counter() - t0, 2)
        say(f"autotune {tuning}")

    # plain copy of 1 GiB: the reference for scaling HBM byte counters
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").uniform_()
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0 = torch.cuda.Event(enable_timing=True); c0.record(stream)
    dst.copy_(src)
    c1 = torch.cuda.Event(enable_timing=True); c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * src.numel() * 8 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    nb_ = NewtonBench(ctx, stream, (q_init, u_init, uh_init), w, dt, dii, cfg["rtol"])
    nm, nu, nb = ctx.n_macros, ctx.n_u_macro, ctx.n_b_macro
    flops = condense_flops(cfg, nu, nb) * nm
    plain = nb_.run(args.steps, args.warmup, main_prec, main_prec, progress=say)
    r0, r1 = nb_.newton_reduction()
    blocks_gpu = {0: ctx.get_condensed(0)}
    apply_ms = time_apply(ctx, stream, args.applies)
    say(f"headline: {plain['ms_per_step']:.1f} ms per Newton step, phases {plain['phase_ms']}")
    variants = {}
    if not args.headline_only and args.mixed_steps > 0:
        mixed = nb_.run(args.mixed_steps, 1, HDG_FP32, HDG_FP32, graph_steps=args.graph_steps, progress=say)
        mr0, mr1 = nb_.newton_reduction()
        blocks32 = {0: ctx.get_condensed(0)}
        apply32_ms = time_apply(ctx, stream, args.applies)
        cm = float(np.mean(mixed["cond_calls"]))
        variants["mixed_fp32_condense_fp32_inner_graph"] = dict(
            workload=args.config, ms_per_step=round(mixed["ms_per_step"], 3),
            speedup_vs_plain=round(plain["ms_per_step"] / mixed["ms_per_step"], 3),
            phases_ms={k: round(v, 3) for k, v in mixed["phase_ms"].items()},
            fgmres=dict(outer_its=mixed["outer"], inner_its=mixed["inner"]), graph_steps=args.graph_steps,
            newton_residual=dict(before=r0, after_step=mr1),
            condense_ms=round(cm, 3), condense_tflops=round(flops / (cm * 1e-3) / 1e12, 3),
            condense_frac_fp32_peak=round(flops / (cm * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
            apply_ms=round(apply32_ms, 4),
            apply_gbs=round(apply_bytes(ctx, 4.0) / (apply32_ms * 1e-3) / 1e9, 1))
        say(f"mixed: {mixed['ms_per_step']:.1f} ms per Newton step")
    bytes64, n_glob = apply_bytes(ctx, 8.0), ctx.n_glob
    ctx.close()
    del nb_
    gc.collect()
    torch.cuda.empty_cache()

    apply_gbs = bytes64 / (apply_ms * 1e-3) / 1e9
    cond_calls = plain["cond_calls"]
    cond_ms = float(np.mean(cond_calls))
    cond_tflops = flops / (cond_ms * 1e-3) / 1e12
    traffic = (CONDENSE_TRAFFIC.get(f"{args.config}/{per_chunk or nm}") if sources_sha() == CONDENSE_TRAFFIC["sha"]
               else None)
    peak = PEAK_FP64_TFLOPS if main_prec == HDG_FP64 else PEAK_FP32_TFLOPS
    if main_prec != HDG_FP64:
        traffic = None
    roofline = dict(bound="mfma", achieved=round(cond_tflops, 3), peak=peak, unit="TFLOP/s",
                    frac=round(cond_tflops / peak, 4), traffic=traffic,
                    kernel="hdg_condense (chunked): k_form + batched elimination (tournament pivoting k_tslu_round/"
                           "k_tslu_final or the register panel k_panel, k_uinv, k_u12, k_linv2, k_u12lin, k_gemm on "
                           "FP64 MFMA) + k_extract + k_store_factors (factor store) + face-preconditioner factorisation",
                    flops_per_launch=flops, ms_per_launch=round(cond_ms, 3), launches=len(cond_calls))
    ms_step = plain["ms_per_step"]
    out = dict(metric=METRIC, value=round(ms_step, 3), unit="ms/Newton-step", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(ms_step, 3), higher_is_better=False, scaling="weak",
               vs_baseline=None, dtype="f64" if main_prec == HDG_FP64 else "f32", data="synthetic",
               config=dict(workload=f"{args.config}: Taylor-Green {cfg['n_elem']}^3 periodic hexes on [-pi,pi]^3, "
                                    f"{cfg['m']}^3-element macros ({nm}), p={cfg['p']}, Mach 0.1, Re 1600, 1e-4 "
                                    f"seeded noise; one Newton step of DIRK(3,3) stage 1 from the initial state: "
                                    f"linearise, second-layer condensation in {(nm + (per_chunk or nm) - 1) // (per_chunk or nm)} "
                                    f"chunks, FGMRES(30) rtol {cfg['rtol']} with 5 inner GMRES steps, recovery, update",
                           n_macros=nm, n_u_macro=nu, n_b_macro=nb, n_glob=n_glob,
                           macros_per_chunk=per_chunk, chunk_slots=args.chunk_slots, factor_store=store,
                           variant="plain FP64" if main_prec == HDG_FP64 else "FP32 condensation"),
               phases_ms={k: round(v, 3) for k, v in plain["phase_ms"].items()},
               fgmres=dict(outer_its=plain["outer"], inner_its=plain["inner"]),
               newton_residual=dict(before=r0, after_step=r1),
               condense_tflops=round(cond_tflops, 3), condense_ms=round(cond_ms, 3),
               apply_ms=round(apply_ms, 4), apply_gbs=round(apply_gbs, 1),
               apply_frac_hbm=round(apply_gbs / PEAK_HBM_GBS, 4), copy_gbs=round(copy_gbs, 1),
               roofline=roofline, variants=variants, autotune=tuning)
    if not args.no_cpu_baseline:
        say("cpu baseline")
        gpu_counts = dict(outer_its=int(np.mean(plain["outer"])),
                          applies=int(np.mean(plain["outer"])) + int(np.mean(plain["inner"])) + 2)
        cb, oblocks = cpu_baseline(cfg, gpu_counts, n_sample=args.cpu_sample)
        if args.cpu_single_thread:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(1):
                cb1, _ = cpu_baseline(cfg, gpu_counts, n_sample=args.cpu_sample, single_thread=True)
            cb["single_thread"] = dict(value=cb1["value"], phases_ms=cb1["phases_ms"], sample=cb1["sample"])
        out["cpu_baseline"] = cb
        # error against the FP64 oracle on the sampled macros' condensed blocks
        err = {}
        for i, (Ao, bo) in oblocks.items():
            Ag, bg = blocks_gpu[i]
            err[f"macro_{i}"] = dict(plain_fp64=dict(ahat=_rel_max(Ag, Ao), bhat=_rel_max(bg, bo)))
            if "mixed_fp32_condense_fp32_inner_graph" in variants:
                A3, b3 = blocks32[i]
                err[f"macro_{i}"]["mixed_fp32"] = dict(ahat=_rel_max(A3, Ao), bhat=_rel_max(b3, bo))
        out["error_vs_fp64_oracle"] = err
        say(f"cpu baseline {cb['value']} ms; block errors {err}")
    if not args.headline_only and args.c2_stages > 0:
        c2_variants(args, dev, variants, say)
        gc.collect()
        torch.cuda.empty_cache()
    if args.uneven:
        uneven_variant(args, dev, variants)
        gc.collect(); torch.cuda.empty_cache()
    if args.learned_p3:
        learned_p3_variant(args, dev, variants)
        gc.collect(); torch.cuda.empty_cache()
    if args.nested:
        nested_variant(args, dev, variants)
        gc.collect(); torch.cuda.empty_cache()
    if args.first_layer:
        first_layer_variant(args, dev, variants)
        gc.collect(); torch.cuda.empty_cache()
    if args.tgv_eps > 0:
        tgv_dissipation_variant(args, dev, variants)
        gc.collect(); torch.cuda.empty_cache()
    if args.big_steps > 0:
        big_variant(args, dev, variants)
    say("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
