#!/usr/bin/env python3
"""Benchmark: tet force + stiffness-product evaluations per second on one MI355X.

Workload: 64^3 unit cube, 6 Kuhn tets per cell (1,572,864 tets, 274,625
vertices), compressible neo-Hookean, E=1e6, nu=0.45, FP32 element arithmetic
with FP64 vertex vectors, at a perturbed state d ~ U(+-0.02h) (seed 10) and
direction u ~ U(-1,1) (seed 11).  Synthetic inputs stand in for the paper's
meshes (Vega's dragon/hose/turtle and the FreeFem++ bunny are not available).

One step = one internal-force call + one stiffness-product call over the whole
mesh.  Headline (cold): the device caches, including the 256 MB Infinity
Cache, are flushed before each call, so the inputs come from HBM; each call is
timed with HIP events on its stream.  value = tets / (t_force + t_Kmul).
Also reported: the warm back-to-back rate, the implicit step (100 CG
iterations), the roofline of the dominant call and the CPU oracle baseline.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def canonical_bytes(nt, nv, op, prec_bytes=4):
    """Algorithmic bytes of one call: per tet 4 int32 keys + 9 B entries + V0 at
    element precision; per vertex each FP64 vec3 touched once (force: d read,
    f written; Kmul: d, u read, y written)."""
    per_tet = 16 + 10 * prec_bytes
    per_vert = 48 if op == "force" else 72
    return nt * per_tet + nv * per_vert


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--strategy", default="block", choices=["atomic", "seg", "block", "block_lds"])
    ap.add_argument("--order", default="morton", choices=["lattice", "morton"])
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-step", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--all-strategies", action="store_true")
    ap.add_argument("--block", type=int, default=0,
                    help="tets per block (block strategy) or threads per workgroup (others); 0 = default")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1506_07577_amd import ebbx
    from paper_1506_07577_amd import meshgen as mg

    if not os.path.exists(ebbx.LIB_PATH):
        from paper_1506_07577_amd import build as hb
        hb.build()
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    w = mg.workload_plain(args.n)
    m = w.mesh
    strat_id = {"atomic": ebbx.STRAT_ATOMIC, "seg": ebbx.STRAT_SEG, "block": ebbx.STRAT_BLOCK,
                "block_lds": ebbx.STRAT_BLOCK_LDS}
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
        tf = [e[0].elapsed_time(e[1]) for e in ev]
        tk = [e[2].elapsed_time(e[3]) for e in ev]
        return tf, tk, wall

    def warm_run(steps):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            fem.forces(d, f, stream=stream)
            ev[k][1].record(stream)
            fem.kmul(d, u, y, stream=stream)
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tf = [e[0].elapsed_time(e[1]) for e in ev]
        tk = [e[1].elapsed_time(e[2]) for e in ev]
        return tf, tk, wall

    def measure(strategy):
        fem.set_strategy(strat_id[strategy], args.block if strategy == args.strategy else 0)
        cold_run(max(args.warmup, 1))
        tf, tk, wall = cold_run(args.steps)
        wtf, wtk, wwall = warm_run(args.steps)
        return dict(tf=tf, tk=tk, wall=wall, wtf=wtf, wtk=wtk, wwall=wwall)

    others = {}
    if args.all_strategies:
        for s in ["atomic", "seg", "block", "block_lds"]:
            if s != args.strategy:
                r = measure(s)
                others[s] = {
                    "cold_force_us": round(1e3 * statistics.median(r["tf"]), 2),
                    "cold_kmul_us": round(1e3 * statistics.median(r["tk"]), 2),
                    "warm_force_us": round(1e3 * statistics.median(r["wtf"]), 2),
                    "warm_kmul_us": round(1e3 * statistics.median(r["wtk"]), 2),
                }
    r = measure(args.strategy)
    tf_ms = statistics.mean(r["tf"])
    tk_ms = statistics.mean(r["tk"])
    ms_per_step = tf_ms + tk_ms
    value = nt / (ms_per_step * 1e-3)
    med_f, med_k = statistics.median(r["tf"]), statistics.median(r["tk"])
    warm_ms = statistics.mean(r["wtf"]) + statistics.mean(r["wtk"])

    # roofline of the dominant call (the stiffness product): algorithmic bytes / mean duration
    bk = canonical_bytes(nt, nv, "kmul")
    bf = canonical_bytes(nt, nv, "force")
    achieved = bk / (tk_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "stiffness product call (ebbx_fem_Kmul)",
                "algorithmic_bytes": bk, "mean_us": round(1e3 * tk_ms, 2)}
    combined_frac = (bf + bk) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS

    extra = {}
    if not args.no_step:
        # one implicit step, 100 CG iterations, tol = 0 (fixed count)
        dd = d.clone()
        vv = torch.zeros_like(d)
        fem.implicit_step(dd, vv, w.dt, tol=0.0, maxit=w.maxit)   # graph capture + warm-up
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            dd.copy_(d)
            vv.zero_()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            st = fem.implicit_step(dd, vv, w.dt, tol=0.0, maxit=w.maxit, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        s = ebbx.stats_fetch(st)
        extra["implicit_step"] = {"ms": round(min(times), 3), "cg_iters": s.iters,
                                  "us_per_cg_iter": round(1e3 * min(times) / max(s.iters, 1), 2),
                                  "rel_res": s.rel_res, "status": s.status}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        X = m.X
        ref = oracle.FEM.create(w.model, X, m.tets, w.E, w.nu, pinned=m.pinned)
        dh = mg.perturbed_state(m, 0.02, seed=10)
        uh = mg.direction(m, 11)
        reps = 0
        t0 = time.perf_counter()
        while True:
            ref.forces(dh)
            ref.kmul(dh, uh)
            reps += 1
            if time.perf_counter() - t0 >= args.cpu_seconds:
                break
        el = time.perf_counter() - t0
        cpu = {"value": round(reps * nt / el, 1), "unit": "tet force+Kmul evals/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{reps} force+Kmul passes over the full {nt}-tet mesh, FP64, serial C, "
                         f"{el:.1f} s"}

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
        "dtype": "f32 element math, f64 vertex vectors",
        "data": "synthetic",
        "config": {"workload": f"{args.n}^3 Kuhn cube, neo-Hookean, 1 force + 1 Kmul per step, cold caches",
                   "tets": nt, "verts": nv, "strategy": args.strategy, "order": args.order,
                   "block": fem.get_strategy()[1],
                   "protocol": "1 GiB cache flush before each call; HIP events on the launch stream"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "force_us_median": round(1e3 * med_f, 2),
        "kmul_us_median": round(1e3 * med_k, 2),
        "combined_hbm_frac": round(combined_frac, 4),
        "warm_evals_per_s": round(nt / (warm_ms * 1e-3), 1),
        "warm_force_us": round(1e3 * statistics.mean(r["wtf"]), 2),
        "warm_kmul_us": round(1e3 * statistics.mean(r["wtk"]), 2),
        "timed_wall_s": round(r["wall"], 4),
        "setup_s": round(t_setup, 3),
    }
    out.update(extra)
    if others:
        out["other_strategies"] = others
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
