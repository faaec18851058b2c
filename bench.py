#!/usr/bin/env python3
"""Benchmark: tet force + stiffness-product evaluations per second on one MI355X.

Workload: 64^3 unit cube, 6 Kuhn tets per cell (1,572,864 tets, 274,625
vertices), compressible neo-Hookean, E=1e6, nu=0.45, FP32 element arithmetic
with FP64 vertex vectors and FP64 accumulation, at a perturbed state
d ~ U(+-0.02h) (seed 10) and direction u ~ U(-1,1) (seed 11), mesh in Morton
order.  Synthetic inputs stand in for the paper's meshes (Vega's
dragon/hose/turtle and the FreeFem++ bunny are not available).

One step = one internal-force call + one stiffness-product call over the whole
mesh.  Headline (cold): before each call a 1 GiB read-only stream evicts the
device caches (including the 256 MB Infinity Cache), so the call's inputs come
from HBM; each call is timed with HIP events on its stream and
value = tets / (median t_force + median t_Kmul).  Also reported: the warm rate (steps
back to back, timed as a whole), the implicit step (100 CG iterations), the
roofline of the dominant call and the CPU oracle baseline.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cube64_nh_f32.json")


def canonical_bytes(nt, nv, op, prec_bytes=4):
    """Algorithmic bytes of one call: per tet 4 int32 keys + 9 B entries + V0 at
    element precision; per vertex each FP64 vec3 touched once (force: d read,
    f written; Kmul: d, u read, y written)."""
    per_tet = 16 + 10 * prec_bytes
    per_vert = 48 if op == "force" else 72
    return nt * per_tet + nv * per_vert


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("elem.hip", "fem.hip", "fem.h", "tetmath.h"):
        with open(os.path.join(ROOT, "paper_1506_07577_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--strategy", default="block", choices=["atomic", "seg", "block", "block_lds", "owner", "pipe", "lanes"])
    ap.add_argument("--order", default="morton", choices=["lattice", "morton"])
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--block", type=int, default=0,
                    help="tets per block (block strategies) or threads per workgroup (others); 0 = default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-step", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--all-strategies", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (counter calibration)")
    ap.add_argument("--workload", default="plain", choices=["plain", "locality"],
                    help="plain: the headline 64^3 line; locality: the 128^3 StVK FP64 mesh, scrambled "
                         "then Morton-ordered, every strategy (a separate JSON line)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-step section")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint section")
    ap.add_argument("--no-assembled", action="store_true", help="skip the assembled-stiffness section")
    ap.add_argument("--no-springs", action="store_true", help="skip the spring-mass section")
    ap.add_argument("--no-autotune", action="store_true", help="skip the autotuner section")
    ap.add_argument("--no-small", action="store_true", help="skip the 8^3 latency section")
    ap.add_argument("--no-cpu-adjoint", action="store_true", help="skip the oracle's adjoint sample")
    ap.add_argument("--no-cpu-batch", action="store_true", help="skip the oracle's 16-mesh batch sample")
    ap.add_argument("--only", default="",
                    help="locality workload: comma-separated order/strategy rows to run (e.g. morton/block)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_events(fn, stream, reps):
    """Run fn() reps times, each bracketed by HIP events on `stream`; returns ms per run."""
    import torch
    out = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def bench_springs(stream, flush_bytes):
    """Spring-mass example on the 64^3 cube (vertices and edges in Morton order): force pass cold,
    and steps replayed from the graph."""
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg
    w = mg.workload_springs(64)
    m = w.mesh
    sm = ebbx.SpringMesh(m.X, w.tail, w.head, w.K, morton=True)
    sp = sm.springs
    md = sm.scalar_to_dev(w.mass)
    q, qd = sm.to_dev(w.q0), sm.to_dev(w.qd0)
    f = torch.zeros_like(q)
    nv, ne = sm.nv, len(w.tail)
    tf = []
    for _ in range(10):
        ebbx.cache_flush(flush_bytes, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sp.forces(q, f, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        tf.append(e0.elapsed_time(e1))
    f.zero_()
    steps = 320
    sp.run(md, w.dt, steps, q, qd, f, stream=stream)   # capture + warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sp.run(md, w.dt, steps, q, qd, f, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / steps
    # per step, the least a step must move: heads and rest lengths per edge, row offsets, q read
    # once (own and neighbour positions), the new q written, qd read and written, mass read
    step_bytes = 12 * ne + 4 * (nv + 1) + 104 * nv
    sp.close()
    return {"mesh": "cube64 directed edges", "n_verts": nv, "n_edges": ne,
            "forces_cold_us": round(1e3 * statistics.median(tf), 2),
            "graph_step_us": round(1e3 * step_ms, 2),
            "edge_evals_per_s": round(ne / (step_ms * 1e-3), 1),
            "step_algorithmic_bytes": step_bytes,
            "step_hbm_frac": round(step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_small(stream):
    """Latency on the small case (8^3 jittered cube, 3,072 tets, StVK FP64, bottom pinned): one
    force call, one stiffness-product call (warm, medians of 50), and one implicit step with 50
    CG iterations (dt = 1e-3, tol = 0) replayed from its graphs (median of 20)."""
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg
    w = mg.workload_small()
    m = w.mesh
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=w.model, elem_prec=ebbx.F64, E=w.E, nu=w.nu,
                        strategy=ebbx.STRAT_BLOCK, morton=True)
    d = mesh.to_dev(mg.perturbed_state(m, 0.02, seed=10))
    u = mesh.to_dev(mg.direction(m, 11))
    f, y = torch.empty_like(d), torch.empty_like(d)
    tf = time_events(lambda: mesh.fem.forces(d, f, stream=stream), stream, 50)
    tk = time_events(lambda: mesh.fem.kmul(d, u, y, stream=stream), stream, 50)
    dd, vv = torch.zeros_like(d), torch.zeros_like(d)

    def step():
        mesh.fem.implicit_step(dd, vv, 1e-3, tol=0.0, maxit=w.maxit, stream=stream)

    step()   # graph capture
    ts = []
    for _ in range(20):
        dd.zero_()
        vv.zero_()
        ts += time_events(step, stream, 1)
    mesh.fem.close()
    return {"mesh": "8^3 jittered, 3072 tets, StVK FP64", "force_us": round(1e3 * statistics.median(tf), 2),
            "kmul_us": round(1e3 * statistics.median(tk), 2),
            "step_50_cg_iters_us": round(1e3 * statistics.median(ts), 1),
            "note": "warm calls, HIP events per call (launch latency included); no roofline at this size"}


def cand_name(names, sid, blk):
    """strategy/block, with "x2" for two tets per thread"""
    two = blk & 0x10000
    return f"{names.get(sid, sid)}/{blk & 0xffff}" + ("x2" if two else "")


def bench_autotune(stream, n):
    """The autotuner on the headline mesh (64^3 neo-Hookean FP32, Morton order): every strategy
    and block size timed on the stiffness product, the fastest kept; no cache."""
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg
    w = mg.workload_plain(n)
    m = w.mesh
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=w.model, elem_prec=ebbx.F32 if w.prec == "f32" else ebbx.F64,
                        E=w.E, nu=w.nu, strategy=ebbx.STRAT_AUTO, morton=True)
    d = mesh.to_dev(mg.perturbed_state(m, 0.02, seed=10))
    u = mesh.to_dev(mg.direction(m, 11))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = mesh.fem.autotune(d, u, stream=stream)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    names = {ebbx.STRAT_ATOMIC: "atomic", ebbx.STRAT_SEG: "seg", ebbx.STRAT_BLOCK: "block",
             ebbx.STRAT_BLOCK_LDS: "block_lds", ebbx.STRAT_OWNER: "owner", ebbx.STRAT_PIPE: "pipe",
             ebbx.STRAT_LANES: "lanes"}
    chosen = mesh.fem.get_strategy()
    out = {"mesh": f"{n}^3 Morton", "tune_s": round(tune_s, 2),
           "chosen": cand_name(names, chosen[0], chosen[1]),
           "candidates_us": {cand_name(names, sid, blk): round(us, 2) for sid, blk, us in res},
           "note": "stiffness product, warm calls timed by the tuner (5 after 2 warm-up, HIP events)"}
    mesh.fem.close()
    return out


def bench_batch(stream, plain_rate, plain_loop_rate=None):
    """256 Kuhn cubes (sides 8..40), neo-Hookean, FP32 elements, per-mesh E and nu, each mesh in
    lattice order, one implicit step of every mesh with per-mesh CG to 1e-8 (maxit 1000)."""
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg
    t0 = time.perf_counter()
    meshes, E, nu = mg.workload_batch()
    un = mg.union(meshes)
    bm = ebbx.BatchMesh(un, E, nu, model=ebbx.NH, elem_prec=ebbx.F32)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    log(f"batch: {bm.nm} meshes, {bm.nt} tets, {bm.nv} verts, setup {setup:.1f} s")
    tuned = tune_batch(stream, meshes, E, nu)
    bm.batch.fem.set_strategy(*tuned["chosen_raw"])
    log(f"batch autotune: {tuned['chosen']} in {tuned['tune_s']} s")
    d0 = torch.zeros(3, bm.nv, dtype=torch.float64, device="cuda")
    d, v = d0.clone(), d0.clone()
    stats = torch.zeros(bm.nm, 3, dtype=torch.int64, device="cuda")

    def step():
        bm.batch.implicit_step(d, v, 1e-3, tol=1e-8, maxit=1000, stats=stats, stream=stream)

    def reset():
        d.zero_()
        v.zero_()

    reset()
    step()   # graph capture
    times = []
    for _ in range(3):
        reset()
        times += time_events(step, stream, 1)
    st = ebbx.stats_parse(stats)
    nts = np.diff(un.tptr)
    iters = np.array([s.iters for s in st])
    ms = min(times)
    useful = float(np.sum(nts * iters))
    rate = useful / (ms * 1e-3)

    # the same step with no CG iteration (force, K v, diagonal, right-hand side, state copies)
    def step0():
        bm.batch.implicit_step(d, v, 1e-3, tol=1e-8, maxit=0, stats=stats, stream=stream)

    reset()
    step0()
    pre = []
    for _ in range(3):
        reset()
        pre += time_events(step0, stream, 1)
    ms_pre = min(pre)
    loop_rate = useful / ((ms - ms_pre) * 1e-3)
    one = bench_one_by_one(stream, meshes[::8], E[::8], nu[::8])
    return {"meshes": bm.nm, "tets": bm.nt, "verts": bm.nv, "setup_s": round(setup, 1),
            "step_ms": round(ms, 3), "cg_iters_min": int(iters.min()), "cg_iters_max": int(iters.max()),
            "cg_iters_mean": round(float(iters.mean()), 2),
            "all_converged": bool(all(s.status == ebbx.OK for s in st)),
            "max_rel_res": max(s.rel_res for s in st),
            "tet_cg_iters_per_s": round(rate, 1),
            "vs_plain_tet_cg_iters_per_s": round(rate / plain_rate, 4) if plain_rate else None,
            "preamble_ms": round(ms_pre, 3),
            "loop_tet_cg_iters_per_s": round(loop_rate, 1),
            "loop_vs_plain_loop": round(loop_rate / plain_loop_rate, 4) if plain_loop_rate else None,
            "one_by_one": one,
            "vs_one_by_one_tet_cg_iters_per_s": round(rate / one["tet_cg_iters_per_s"], 3),
            "autotune": {k: v for k, v in tuned.items() if k != "chosen_raw"}}


def tune_batch(stream, meshes, E, nu):
    """The autotuner on a batched union domain: every 16th mesh of the batch (16 meshes, sides,
    E and nu as drawn), its stiffness product timed under every candidate; the choice is then
    set on the whole batch.  (Tuning the whole 31.8M-tet union would rebuild its block tables
    for every candidate, most of a minute.)"""
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg
    sub = meshes[::16]
    un = mg.union(sub)
    bm = ebbx.BatchMesh(un, E[::16], nu[::16], model=ebbx.NH, elem_prec=ebbx.F32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = bm.batch.fem.autotune(stream=stream)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t0
    names = {ebbx.STRAT_ATOMIC: "atomic", ebbx.STRAT_SEG: "seg", ebbx.STRAT_BLOCK: "block",
             ebbx.STRAT_BLOCK_LDS: "block_lds", ebbx.STRAT_OWNER: "owner", ebbx.STRAT_PIPE: "pipe",
             ebbx.STRAT_LANES: "lanes"}
    chosen = bm.batch.fem.get_strategy()
    out = {"sample": f"every 16th mesh of the batch: {len(sub)} meshes, {un.nt} tets",
           "tune_s": round(tune_s, 2), "chosen": cand_name(names, chosen[0], chosen[1]), "chosen_raw": chosen,
           "candidates_us": {cand_name(names, sid, blk): round(us, 2) for sid, blk, us in res},
           "note": "stiffness product over the union, warm calls timed by the tuner (5 after 2 warm-up)"}
    bm.batch.close()
    return out


def bench_one_by_one(stream, meshes, E, nu):
    """The plain path on a sample of the batch's meshes, each its own Fem (block strategy, Morton
    order, graph captured on its first step), stepped one after another with the batch's
    per-mesh E, nu, tolerance and iteration cap: the work a caller without the batched entry
    point would launch."""
    import torch

    from paper_1506_07577_amd import ebbx
    fems, state = [], []
    for m, Em, num in zip(meshes, E, nu):
        fm = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.NH, elem_prec=ebbx.F32, E=float(Em), nu=float(num),
                          strategy=ebbx.STRAT_BLOCK, morton=True)
        z = torch.zeros(3, fm.nv, dtype=torch.float64, device="cuda")
        fems.append(fm)
        state.append((z, z.clone()))

    def steps():
        return [fm.fem.implicit_step(d, v, 1e-3, tol=1e-8, maxit=1000, stream=stream)
                for fm, (d, v) in zip(fems, state)]

    def reset():
        for d, v in state:
            d.zero_()
            v.zero_()

    steps()   # graph capture per mesh
    best, st = None, None
    for _ in range(3):
        reset()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = steps()
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1)
        if best is None or t < best:
            best, st = t, [ebbx.stats_fetch(o) for o in out]
    useful = float(sum(fm.nt * s.iters for fm, s in zip(fems, st)))
    res = {"meshes": len(fems), "tets": int(sum(fm.nt for fm in fems)), "ms": round(best, 3),
           "all_converged": bool(all(s.status == ebbx.OK for s in st)),
           "tet_cg_iters_per_s": round(useful / (best * 1e-3), 1),
           "sample": "every 8th mesh of the batch (sides, E and nu as drawn)"}
    for fm in fems:
        fm.fem.close()
    return res


def bench_adjoint(stream, plain_step_rate, morton=True):
    """48^3 cube, neo-Hookean FP64, per-tet log-normal E, Morton order: 20 implicit steps (CG to
    1e-10) forward, then dL/dE and dL/dd0 of ||x_T - target||^2 with checkpoints every 5 steps."""
    import torch

    from paper_1506_07577_amd import adjoint, ebbx
    from paper_1506_07577_amd import meshgen as mg
    m = mg.kuhn_cube(48)
    E_tet, target, _ = mg.adjoint_recipe(m, seed=2)
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=ebbx.NH, elem_prec=ebbx.F64, E=1e5, nu=0.3, E_tet=E_tet,
                        strategy=ebbx.STRAT_BLOCK, morton=morton)
    sim = adjoint.Simulation(fem=mesh.fem, steps=20, dt=1e-3, tol=1e-10, maxit=2000, checkpoint_every=5)
    X = mesh.to_dev(m.X)
    tgt = mesh.to_dev(target)
    Et = mesh.tet_to_dev(E_tet)

    def run():
        d0 = torch.zeros(3, mesh.nv, dtype=torch.float64, device="cuda", requires_grad=True)
        v0 = torch.zeros(3, mesh.nv, dtype=torch.float64, device="cuda")
        Eg = Et.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dT, _ = adjoint.trajectory(sim, d0, v0, Eg)
        L = adjoint.position_loss(X, dT, tgt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return t1 - t0, t2 - t1

    run()   # graph capture
    fw, bw = min(run() for _ in range(3))
    fwd_rate = mesh.nt * 20 / fw
    return {"tets": mesh.nt, "verts": mesh.nv, "steps": 20, "checkpoint_every": 5,
            "forward_ms": round(1e3 * fw, 2), "backward_ms": round(1e3 * bw, 2),
            "backward_over_forward": round(bw / fw, 3),
            "forward_backward_over_forward": round((fw + bw) / fw, 3),
            "forward_tet_steps_per_s": round(fwd_rate, 1),
            "forward_backward_tet_steps_per_s": round(mesh.nt * 20 / (fw + bw), 1),
            "plain_step_tet_steps_per_s": round(plain_step_rate, 1) if plain_step_rate else None,
            "forward_vs_plain_step": round(fwd_rate / plain_step_rate, 3) if plain_step_rate else None,
            "vs_plain_note": "plain = one 64^3 NH FP32 step with 100 fixed CG iterations on the same GPU; the "
                             "adjoint's steps are FP64 and stop at 1e-10 (different iteration counts)",
            "note": "wall clock with device syncs; forward = 20 implicit steps (CG to 1e-10), backward = "
                    "segment recompute + 20 step VJPs (adjoint CG, K w, T[v, w], dL/dE)"}


def bench_locality(args):
    """Cold force and K u calls on the 128^3 StVK FP64 mesh (12,582,912 tets) with scrambled
    vertex and tet order, then Morton order, under every scatter strategy."""
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg
    w = mg.workload_locality(args.n if args.n != 64 else 128)
    m = w.mesh
    stream = torch.cuda.current_stream()
    strat = {"atomic": (ebbx.STRAT_ATOMIC, 0), "seg": (ebbx.STRAT_SEG, 0), "block": (ebbx.STRAT_BLOCK, 0),
             "owner": (ebbx.STRAT_OWNER, 64), "lanes": (ebbx.STRAT_LANES, 0), "lanes/128": (ebbx.STRAT_LANES, 128),
             "pipe": (ebbx.STRAT_PIPE, 0)}
    rows = {}
    only = {x for x in args.only.split(",") if x}
    for order in ("scrambled", "morton"):
        if only and not any(x.startswith(order + "/") for x in only):
            continue
        mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=w.model, elem_prec=ebbx.F64, E=w.E, nu=w.nu,
                            strategy=ebbx.STRAT_SEG, morton=(order == "morton"))
        d = mesh.to_dev(mg.perturbed_state(m, 0.02, seed=10))
        u = mesh.to_dev(mg.direction(m, 11))
        f = torch.empty_like(d)
        y = torch.empty_like(d)
        for name, (sid, blk) in strat.items():
            if only and f"{order}/{name}" not in only:
                continue
            try:
                mesh.fem.set_strategy(sid, blk)
            except ebbx.EbbxError as e:   # pipelined blocks need a well-ordered mesh
                rows[f"{order}/{name}"] = {"unavailable": str(e)}
                continue
            tf = time_events(lambda: (ebbx.cache_flush(1 << 30, stream), mesh.fem.forces(d, f, stream=stream)),
                             stream, 1)   # warm-up
            tf, tk = [], []
            for _ in range(args.steps):
                ebbx.cache_flush(1 << 30, stream)
                tf += time_events(lambda: mesh.fem.forces(d, f, stream=stream), stream, 1)
                ebbx.cache_flush(1 << 30, stream)
                tk += time_events(lambda: mesh.fem.kmul(d, u, y, stream=stream), stream, 1)
            bk = canonical_bytes(mesh.nt, mesh.nv, "kmul", 8)
            tk_ms = statistics.mean(tk)
            rows[f"{order}/{name}"] = {"force_us": round(1e3 * statistics.mean(tf), 1),
                                       "kmul_us": round(1e3 * tk_ms, 1),
                                       "kmul_GBps": round(bk / (tk_ms * 1e-3) / 1e9, 1),
                                       "kmul_frac": round(bk / (tk_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"{order}/{name}: {rows[f'{order}/{name}']}")
        mesh.fem.close()
        del mesh, d, u, f, y
        torch.cuda.empty_cache()
    out = {"metric": "tet force+Kmul cold call time by scatter strategy and vertex order", "unit": "us",
           "workload": f"{m.n}^3 Kuhn cube, StVK FP64, E=1e5 nu=0.3, {m.nt} tets, {m.nv} verts",
           "protocol": "1 GiB read-only cache flush before each call; HIP events on the launch stream; "
                       f"mean of {args.steps} calls",
           "algorithmic_bytes_kmul": canonical_bytes(m.nt, m.nv, "kmul", 8), "rows": rows}
    print(json.dumps(out), flush=True)


def host_cpu():
    """(threads for the oracle, CPU model): the cores this process may run on, capped by
    OMP_NUM_THREADS when set (the machine's CPU share), and /proc/cpuinfo's model name."""
    cores = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        cores = min(cores, int(omp))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def timed(fn, seconds, min_reps=1):
    """(repetitions, elapsed s) of fn run until `seconds` have passed (at least min_reps)."""
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if reps >= min_reps and el >= seconds:
            return reps, el


def cpu_baseline(args, w, m, nt, extra):
    """The oracle timed on this host's cores beside the GPU rows, on bounded samples of the same
    workloads.  The headline value is the oracle's force + K u on `cores` OpenMP threads (per-corner
    partials, then a vertex gather over the grouping: bit-for-bit the serial oracle's result); the
    serial figure and the other rows are the serial oracle as the tests use it."""
    import oracle
    from paper_1506_07577_amd import meshgen as mg
    cores, model = host_cpu()
    ref = oracle.FEM.create(w.model, m.X, m.tets, w.E, w.nu, pinned=m.pinned)
    dh = mg.perturbed_state(m, 0.02, seed=10)
    uh = mg.direction(m, 11)
    ref.kmul_mt(dh, uh, cores)   # builds the grouping once
    sec = args.cpu_seconds
    reps, el = timed(lambda: (ref.forces_mt(dh, cores), ref.kmul_mt(dh, uh, cores)), 0.35 * sec)
    cpu = {"value": round(reps * nt / el, 1), "unit": "tet force+Kmul evals/s", "cores": cores,
           "kind": "oracle", "cpu_model": model,
           "sample": f"{reps} force+Kmul passes over the full {nt}-tet mesh (FP64 C oracle, OpenMP over "
                     f"tets then a vertex gather, {cores} threads) in {el:.1f} s"}
    rows = {}
    reps1, el1 = timed(lambda: (ref.forces(dh), ref.kmul(dh, uh)), 0.25 * sec)
    rows["single_thread"] = {"value": round(reps1 * nt / el1, 1), "unit": "tet force+Kmul evals/s",
                             "cores": 1, "sample": f"{reps1} serial passes, full mesh, {el1:.1f} s"}
    # one implicit step: the per-iteration cost from two iteration counts (the force, K v and
    # diagonal passes of the step's setup cancel)
    t = []
    for it in (2, 5):
        t0 = time.perf_counter()
        ref.implicit_step(dh, np.zeros_like(dh), w.dt, tol=0.0, maxit=it)
        t.append(time.perf_counter() - t0)
    per_it = max((t[1] - t[0]) / 3.0, 1e-9)
    rows["implicit_step"] = {"value": round(nt / per_it, 1), "unit": "tet CG iterations/s",
                             "sample": f"full mesh, serial; (t(5 iterations) - t(2 iterations)) / 3 = "
                                       f"{1e3 * per_it:.0f} ms per iteration, setup passes excluded"}
    if "implicit_step" in extra:
        rows["implicit_step"]["gpu_over_oracle"] = round(
            extra["implicit_step"]["tet_cg_iters_per_s"] / rows["implicit_step"]["value"], 1)
    if "assembled" in extra:
        rp, col = oracle.edges(m.nv, m.tets)
        blocks = ref.assemble(dh, rp, col)
        t0 = time.perf_counter()
        for _ in range(5):
            oracle.spmv(rp, col, blocks, uh)
        el = time.perf_counter() - t0
        rows["assembled_spmv"] = {"value": round(5 * nt / el, 1), "unit": "tet-equivalent products/s",
                                  "sample": f"5 block-CSR products, full mesh, serial, {el:.2f} s"}
        rows["assembled_spmv"]["gpu_over_oracle"] = round(
            (nt / (extra["assembled"]["spmv_us"] * 1e-6)) / rows["assembled_spmv"]["value"], 1)
    if "springs" in extra:
        sw = mg.workload_springs(64)
        sref = oracle.Springs(sw.mesh.X, sw.tail, sw.head, sw.mass, sw.K)
        q1, qd1 = sw.q0, sw.qd0
        t0 = time.perf_counter()
        for _ in range(5):
            q1, qd1 = sref.step(q1, qd1, sw.dt)
        el = time.perf_counter() - t0
        rows["springs"] = {"value": round(5 * len(sw.tail) / el, 1), "unit": "spring evals/s",
                           "sample": f"5 steps, full 64^3 edge set, serial, {el:.2f} s"}
        rows["springs"]["gpu_over_oracle"] = round(extra["springs"]["edge_evals_per_s"] /
                                                   rows["springs"]["value"], 1)
    if "adjoint" in extra and not args.no_cpu_adjoint:
        # the 48^3 adjoint workload, first step only: forward (CG to 1e-10) and its step VJP
        ma = mg.kuhn_cube(48)
        E_tet, target, _ = mg.adjoint_recipe(ma, seed=2)
        aref = oracle.FEM.create(oracle.NH, ma.X, ma.tets, E_tet, 0.3, pinned=ma.pinned)
        z = np.zeros((ma.nv, 3))
        t0 = time.perf_counter()
        d1, v1, _dv, so = aref.implicit_step(z, z, 1e-3, tol=1e-10, maxit=2000)
        t1 = time.perf_counter()
        aref.step_vjp(z, v1, 2.0 * (d1 + ma.X - target), np.zeros_like(z), 1e-3, tol=1e-10, maxit=2000)
        t2 = time.perf_counter()
        steps = extra["adjoint"]["steps"]
        fw_est, bw_est = steps * (t1 - t0), steps * (t2 - t1)
        rows["adjoint"] = {
            "forward_tet_steps_per_s": round(ma.nt / (t1 - t0), 1),
            "forward_backward_tet_steps_per_s": round(ma.nt / (t2 - t0), 1),
            "unit": "tet steps/s",
            "forward_s_extrapolated": round(fw_est, 2), "backward_s_extrapolated": round(bw_est, 2),
            "sample": f"first of the {steps} steps only (forward {so.iters} CG iterations to 1e-10, then its "
                      f"step VJP; no checkpoint recompute), serial, {t2 - t0:.1f} s; the extrapolated "
                      f"times are {steps} x the sampled step",
            "gpu_over_oracle_forward": round(extra["adjoint"]["forward_tet_steps_per_s"] /
                                             (ma.nt / (t1 - t0)), 1)}
    if "batched" in extra and not args.no_cpu_batch:
        # 16 meshes of the batch (every 16th, sides, E and nu as drawn), one step each, CG to 1e-8
        meshes, E, nu = mg.workload_batch()
        sel = list(range(0, len(meshes), 16))
        useful, el = 0.0, 0.0
        for i in sel:
            mm = meshes[i]
            bref = oracle.FEM.create(oracle.NH, mm.X, mm.tets, float(E[i]), float(nu[i]), pinned=mm.pinned)
            z = np.zeros((mm.nv, 3))
            t0 = time.perf_counter()
            _d1, _v1, _dv, so = bref.implicit_step(z, z, 1e-3, tol=1e-8, maxit=1000)
            el += time.perf_counter() - t0
            useful += mm.nt * so.iters
        rate = useful / el
        rows["batched"] = {"value": round(rate, 1), "unit": "tet CG iterations/s",
                           "sample": f"{len(sel)} of the {len(meshes)} meshes (every 16th), one step each, serial, "
                                     f"{el:.1f} s; the whole batch would take about "
                                     f"{el * len(meshes) / len(sel):.0f} s (extrapolated by mesh count)",
                           "gpu_over_oracle": round(extra["batched"]["tet_cg_iters_per_s"] / rate, 1)}
    cpu["rows"] = rows
    return cpu


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.workload == "locality":
        from paper_1506_07577_amd import ebbx
        if not os.path.exists(ebbx.LIB_PATH):
            raise SystemExit(f"{ebbx.LIB_PATH} is missing: run __graft_entry__.build() first")
        torch.cuda.set_device(0)
        bench_locality(args)
        return

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg

    if not os.path.exists(ebbx.LIB_PATH):
        from paper_1506_07577_amd import build as hb
        hb.build()
    torch.cuda.set_device(0)
    w = mg.workload_plain(args.n)
    m = w.mesh
    strat_id = {"atomic": ebbx.STRAT_ATOMIC, "seg": ebbx.STRAT_SEG, "block": ebbx.STRAT_BLOCK,
                "block_lds": ebbx.STRAT_BLOCK_LDS, "owner": ebbx.STRAT_OWNER, "pipe": ebbx.STRAT_PIPE,
                "lanes": ebbx.STRAT_LANES}
    t_setup = time.perf_counter()
    mesh = ebbx.FemMesh(m.X, m.tets, m.pinned, model=w.model, elem_prec=ebbx.F32, E=w.E, nu=w.nu,
                        strategy=strat_id[args.strategy], block=args.block, morton=(args.order == "morton"))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    fem = mesh.fem
    nt, nv = mesh.nt, mesh.nv
    d = mesh.to_dev(mg.perturbed_state(m, 0.02, seed=10))
    u = mesh.to_dev(mg.direction(m, 11))
    f = torch.empty_like(d)
    y = torch.empty_like(d)
    stream = torch.cuda.current_stream()
    flush_bytes = 1 << 30
    if args.calib_copy:
        a = torch.zeros(1 << 25, dtype=torch.float64, device="cuda")   # 256 MiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def cold_run(steps):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ebbx.cache_flush(flush_bytes, stream)
            ev[k][0].record(stream)
            fem.forces(d, f, stream=stream)
            ev[k][1].record(stream)
            ebbx.cache_flush(flush_bytes, stream)
            ev[k][2].record(stream)
            fem.kmul(d, u, y, stream=stream)
            ev[k][3].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return [e[0].elapsed_time(e[1]) for e in ev], [e[2].elapsed_time(e[3]) for e in ev], wall

    def warm_run(steps):
        # steps back to back, one event pair around all of them
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fem.forces(d, f, stream=stream)
            fem.kmul(d, u, y, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def graph_run(calls=100):
        # warm steady state: `calls` force+Kmul pairs captured in one HIP graph, replayed
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            fem.forces(d, f, stream=side)   # warm-up outside the capture
            fem.kmul(d, u, y, stream=side)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            for _ in range(calls):
                fem.forces(d, f, stream=side)
                fem.kmul(d, u, y, stream=side)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / calls

    def measure(strategy, block):
        fem.set_strategy(strat_id[strategy], block)
        cold_run(max(args.warmup, 1))
        tf, tk, wall = cold_run(args.steps)
        warm_ms = warm_run(args.steps)
        return dict(tf=tf, tk=tk, wall=wall, warm_ms=warm_ms)

    others = {}
    if args.all_strategies:
        for s in ["atomic", "seg", "block", "block_lds", "owner"]:
            if s != args.strategy:
                r = measure(s, 0)
                others[s] = {"cold_force_us": round(1e3 * statistics.median(r["tf"]), 2),
                             "cold_kmul_us": round(1e3 * statistics.median(r["tk"]), 2),
                             "warm_step_us": round(1e3 * r["warm_ms"], 2)}
    r = measure(args.strategy, args.block)
    log(f"force+Kmul cold {statistics.median(r['tf']) + statistics.median(r['tk']):.4f} ms")
    # headline: nt / (median force call + median Kmul call), each call cold
    tf_med = statistics.median(r["tf"])
    tk_med = statistics.median(r["tk"])
    tf_ms = statistics.mean(r["tf"])
    tk_ms = statistics.mean(r["tk"])
    ms_per_step = tf_med + tk_med
    value = nt / (ms_per_step * 1e-3)
    graph_ms = graph_run()

    # roofline of the dominant call (the stiffness product): algorithmic bytes / mean duration
    bk = canonical_bytes(nt, nv, "kmul")
    bf = canonical_bytes(nt, nv, "force")
    achieved = bk / (tk_ms * 1e-3) / 1e9
    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        key = f"{args.strategy}_{args.order}_{fem.get_strategy()[1]}"
        if tr.get("source_hash") == kernel_source_hash() and args.n == 64 and key in tr.get("kmul_bytes", {}):
            traffic = tr["kmul_bytes"][key]
    except (OSError, ValueError):
        pass
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": (f"not measured in this run: FETCH_SIZE + WRITE_SIZE counters from "
                                   f"{os.path.relpath(TRAFFIC_FILE, ROOT)} for kernel sources {kernel_source_hash()}"
                                   if traffic is not None else None),
                "kernel": "stiffness-product call (block kernel + halo pass), cold, mean over the timed calls",
                "algorithmic_bytes": bk, "mean_us": round(1e3 * tk_ms, 2)}

    extra = {}
    if not args.no_step:
        # one implicit step, 100 CG iterations, tol = 0 (fixed count), captured graph;
        # then the same step with Rayleigh damping (alpha = 2.5 / s, beta = 4e-3 s)
        def time_step(alpha, beta, maxit=w.maxit):
            dd = d.clone()
            vv = torch.zeros_like(d)
            fem.implicit_step(dd, vv, w.dt, tol=0.0, maxit=maxit, alpha=alpha, beta=beta)   # capture + warm-up
            torch.cuda.synchronize()
            times = []
            st = None
            for _ in range(3):
                dd.copy_(d)
                vv.zero_()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                st = fem.implicit_step(dd, vv, w.dt, tol=0.0, maxit=maxit, stream=stream, alpha=alpha, beta=beta)
                e1.record(stream)
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            return min(times), ebbx.stats_fetch(st)

        t_step, s = time_step(0.0, 0.0)
        plain_rate = nt * s.iters / (t_step * 1e-3)
        plain_step_rate = nt / (t_step * 1e-3)
        # the same step with no CG iteration: the force, K v and diagonal passes, the right-hand
        # side and the state copies, so that the CG loop's own rate can be compared with a batch's
        t_pre, _s0 = time_step(0.0, 0.0, maxit=0)
        plain_loop_rate = nt * s.iters / ((t_step - t_pre) * 1e-3)
        # per CG iteration: the K p element map (same bytes as a K u call) plus the vector
        # kernels (q = A p: y, p, mass, pinned in, q out; update: x, p, r, q, diag in, x, r, z
        # out; p = z + beta p: z, p in, p out)
        cg_bytes = bk + nv * (24 * 4 + 9 + 24 * 8 + 24 * 3)
        extra["implicit_step"] = {"ms": round(t_step, 3), "cg_iters": s.iters,
                                  "us_per_cg_iter": round(1e3 * t_step / max(s.iters, 1), 2),
                                  "cg_iter_algorithmic_bytes": cg_bytes,
                                  "cg_iter_hbm_frac": round(cg_bytes / (t_step * 1e-3 / max(s.iters, 1)) / 1e9
                                                            / HBM_PEAK_GBS, 4),
                                  "tet_cg_iters_per_s": round(plain_rate, 1),
                                  "preamble_ms": round(t_pre, 3),
                                  "loop_tet_cg_iters_per_s": round(plain_loop_rate, 1),
                                  "rel_res": s.rel_res, "status": s.status}
        t_damp, sd = time_step(2.5, 4e-3)
        extra["implicit_step"]["damped"] = {"alpha": 2.5, "beta": 4e-3, "ms": round(t_damp, 3),
                                            "cg_iters": sd.iters, "rel_res": sd.rel_res, "status": sd.status}
        log(f"implicit step {t_step:.3f} ms, damped {t_damp:.3f} ms")
    else:
        plain_rate = plain_step_rate = plain_loop_rate = None
    if not args.no_assembled:
        # the stiffness assembled on the edges relation (Vega's representation): one-time edge
        # build, assembly of K(d), and the block-CSR product against the matrix-free K u call
        t0 = time.perf_counter()
        ne = fem.edge_count()
        build_s = time.perf_counter() - t0
        fem.assemble(d, stream=stream)
        fem.spmv(u, y, stream=stream)
        torch.cuda.synchronize()
        reps = max(3, min(args.steps, 20))
        ta, ts = [], []
        for _ in range(reps):
            ebbx.cache_flush(flush_bytes, stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fem.assemble(d, stream=stream)
            e1.record(stream)
            ebbx.cache_flush(flush_bytes, stream)
            e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e2.record(stream)
            fem.spmv(u, y, stream=stream)
            e3.record(stream)
            torch.cuda.synchronize()
            ta.append(e0.elapsed_time(e1))
            ts.append(e2.elapsed_time(e3))
        esz = 4 if w.prec == "f32" else 8
        sp_bytes = (nv + 1) * 4 + ne * (4 + 9 * esz) + 72 * nv
        sp_ms = statistics.median(ts)
        extra["assembled"] = {
            "n_edges": ne, "edge_build_s": round(build_s, 3),
            "assemble_ms": round(statistics.median(ta), 3),
            "spmv_us": round(1e3 * sp_ms, 2), "matrix_free_kmul_us": round(1e3 * tk_med, 2),
            "spmv_over_matrix_free": round(sp_ms / tk_med, 3),
            "spmv_algorithmic_bytes": sp_bytes,
            "spmv_hbm_frac": round(sp_bytes / (sp_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "block_bytes": ne * 9 * esz, "scratch_bytes": nt * 144 * esz,
            "note": "cold calls (1 GiB flush before each); per-tet records and edge blocks at the element precision, FP64 sums"}
        log(f"assembled: build {build_s:.2f} s, assemble {statistics.median(ta):.3f} ms, spmv {1e3 * sp_ms:.1f} us")
    if not args.no_springs:
        extra["springs"] = bench_springs(stream, flush_bytes)
        log(f"springs: {extra['springs']['graph_step_us']} us per step")
    if not args.no_small:
        extra["small"] = bench_small(stream)
        log(f"small: force {extra['small']['force_us']} us, step {extra['small']['step_50_cg_iters_us']} us")
    if not args.no_autotune:
        extra["autotune"] = bench_autotune(stream, args.n)
        log(f"autotune: {extra['autotune']['chosen']} in {extra['autotune']['tune_s']} s")
    if not args.no_batch:
        extra["batched"] = bench_batch(stream, plain_rate, plain_loop_rate)
        log(f"batched step {extra['batched']['step_ms']} ms")
    if not args.no_adjoint:
        extra["adjoint"] = bench_adjoint(stream, plain_step_rate)
        log(f"adjoint fwd {extra['adjoint']['forward_ms']} ms bwd {extra['adjoint']['backward_ms']} ms")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, w, m, nt, extra)

    out = {
        "metric": "tet force+Kmul evals/s (1.6M tets); batched & adjoint vs plain, same GPU",
        "value": round(value, 1),
        "unit": "tet force+Kmul evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 element math, f64 vertex vectors and accumulation",
        "data": "synthetic",
        "config": {"workload": f"{args.n}^3 Kuhn cube (6 tets/cell), neo-Hookean E=1e6 nu=0.45, "
                               f"1 force + 1 Kmul per step, cold caches",
                   "tets": nt, "verts": nv, "strategy": args.strategy, "order": args.order,
                   "block": fem.get_strategy()[1],
                   "protocol": "1 GiB read-only cache flush before each call; HIP events on the launch stream"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "force_us_median": round(1e3 * tf_med, 2),
        "kmul_us_median": round(1e3 * tk_med, 2),
        "force_us_mean": round(1e3 * tf_ms, 2),
        "kmul_us_mean": round(1e3 * tk_ms, 2),
        "force_tets_per_s": round(nt / (tf_med * 1e-3), 1),
        "kmul_tets_per_s": round(nt / (tk_med * 1e-3), 1),
        "combined_hbm_frac": round((bf + bk) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "warm_evals_per_s": round(nt / (r["warm_ms"] * 1e-3), 1),
        "warm_step_us": round(1e3 * r["warm_ms"], 2),
        "warm_graph_step_us": round(1e3 * graph_ms, 2),
        "warm_note": "warm = calls back to back (inputs in the 256 MB Infinity Cache, so not an HBM figure); "
                     "graph = 100 force+Kmul pairs captured in one HIP graph",
        "timed_wall_s": round(r["wall"], 4),
        "setup_s": round(t_setup, 3),
        "kernel_source": kernel_source_hash(),
    }
    out.update(extra)
    if others:
        out["other_strategies"] = others
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
