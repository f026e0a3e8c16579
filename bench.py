"""Smooth-distance value+gradient throughput on one MI355X.

Workload: the bumpy level-7 icosphere (327,680 triangles, 163,842 vertices,
radial sinusoid bumps) with 1,000,000 FP32 queries, half uniform in
[-1.5, 1.5]^3 and half within +-0.02 of the surface along face normals;
alpha = 50, beta = 0.5 (Barnes-Hut), the paper's blending weights.

One step = Morton ordering of the queries + Alg. 1/Alg. 2 traversal with
value and gradient for every query (sd_query_order + sd_eval_grad_ordered),
inputs resident in HBM.  The hierarchy build is timed separately (build_ms).

Prints one JSON line (see the keys below).  --gpus N > 1 is not supported:
the library runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector issue rate of the code as built (packed FP32 instructions are
# disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6
ALU_PEAK_PACKED_TFLOPS = 157.3
# algorithmic FLOPs per unit of work, value + gradient (see the design notes):
F_QUERY = 50        # load, seed bookkeeping, finalisation
F_NODE = 26         # box distance, box diagonal, opening and pruning tests
F_FAR = 35          # sqrt, rcp, direction, exponent, compensated sums
F_TRI_LEAF = 636    # distance + region, de Casteljau weight, gradient, sums
METRIC = "smooth-distance+grad queries/s on 1 MI355X: BH vs surrogate at ≤1e-5 rel / 1e-3 abs"
# algorithmic bytes per unit of work (see the design notes)
B_QUERY = 12 + 16 + 4        # query in, value + gradient out, order index
B_NODE = 32                  # one hierarchy node record
B_TRI_LEAF = 48              # one triangle leaf record


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_src):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic_k_eval_icosphere_l7_1M.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha") != _sha(kernel_src):
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=50.0)
    ap.add_argument("--beta", type=float, default=0.5)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--nq", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample", type=int, default=250000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run 3 plain device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        x = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; this build runs on one GPU "
              "(queries shard with no communication; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_10480_amd import api, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t_gen = time.time()
    sc = scenes.bumpy_icosphere(level=args.level, seed=2)
    Q = scenes.icosphere_queries(sc, args.nq, seed_box=3, seed_surf=4)
    t_gen = time.time() - t_gen
    V = torch.as_tensor(sc.V, device=dev)
    T = torch.as_tensor(sc.T, device=dev)
    Qd = torch.as_tensor(Q, device=dev)
    torch.cuda.synchronize()

    # hierarchy build (a1-a3), timed on its own
    builds = []
    for _ in range(2):
        t0 = time.perf_counter()
        scene = api.sd_build_bvh(V, T=T)
        torch.cuda.synchronize()
        builds.append((time.perf_counter() - t0) * 1e3)
    info = scene.info()

    n = args.nq
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    d = torch.empty(n, dtype=torch.float32, device=dev)
    g = torch.empty((n, 3), dtype=torch.float32, device=dev)

    def step():
        api.sd_query_order(scene, Qd, out=perm)
        api.sd_eval_grad_ordered(scene, Qd, perm, args.alpha, args.beta, out=d, grad_out=g)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for k in range(args.steps):
        ev[k][0].record(s)
        api.sd_query_order(scene, Qd, out=perm)
        ev[k][1].record(s)
        api.sd_eval_grad_ordered(scene, Qd, perm, args.alpha, args.beta, out=d, grad_out=g)
        ev[k][2].record(s)
    e1.record(s)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ms_step = total_ms / args.steps
    order_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    eval_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))   # the traversal kernel alone
    qps = n / (ms_step * 1e-3)

    # the same step visiting every node of Alg. 1's cut (no negligible-subtree skipping)
    e2 = torch.cuda.Event(enable_timing=True)
    e3 = torch.cuda.Event(enable_timing=True)
    e2.record(s)
    for k in range(args.steps):
        api.sd_query_order(scene, Qd, out=perm)
        api.sd_eval_grad_ordered(scene, Qd, perm, args.alpha, args.beta, flags=api.SD_NO_PRUNE,
                                 out=d, grad_out=g)
    e3.record(s)
    torch.cuda.synchronize()
    ms_step_noprune = e2.elapsed_time(e3) / args.steps
    cnt_np = api.sd_eval_counters(scene, Qd, args.alpha, args.beta, flags=api.SD_NO_PRUNE).double()
    api.sd_query_order(scene, Qd, out=perm)
    api.sd_eval_grad_ordered(scene, Qd, perm, args.alpha, args.beta, out=d, grad_out=g)

    # work counters on the same inputs -> algorithmic bytes
    cnt = api.sd_eval_counters(scene, Qd, args.alpha, args.beta).double()
    nodes, far, leaves = [float(x) for x in cnt.mean(0).cpu()]
    p99 = [float(x) for x in torch.quantile(cnt[:200000], 0.99, dim=0).cpu()]
    bytes_per_query = B_QUERY + B_NODE * nodes + B_TRI_LEAF * leaves
    achieved = n * bytes_per_query / (eval_ms * 1e-3) / 1e9
    flops_per_query = F_QUERY + F_NODE * nodes + F_FAR * far + F_TRI_LEAF * leaves
    tflops = n * flops_per_query / (eval_ms * 1e-3) / 1e12
    traffic = _traffic(os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "eval.hip"))

    out = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"bumpy icosphere level {args.level} ({info['n_prims'][2]} triangles), "
                        f"{n} queries (half uniform in [-1.5,1.5]^3, half within 0.02 of the "
                        f"surface), alpha={args.alpha:g}, beta={args.beta:g}, Barnes-Hut, "
                        "value+gradient",
            "mode": "barnes_hut",
            "n_triangles": info["n_prims"][2],
            "n_queries": n,
            "alpha": args.alpha,
            "beta": args.beta,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_eval (Barnes-Hut traversal, value+gradient)",
            "achieved": tflops,
            "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": tflops / ALU_PEAK_TFLOPS,
            "frac_of_packed_peak": tflops / ALU_PEAK_PACKED_TFLOPS,
            "traffic": traffic,
            "flops_per_query": flops_per_query,
            "kernel_ms": eval_ms,
            "hbm_algorithmic": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": achieved / HBM_PEAK_GBS,
                                "bytes_per_query": bytes_per_query},
        },
        "stages_ms": {"query_order": order_ms, "traversal": eval_ms, "build": min(builds)},
        "work_per_query": {"nodes": nodes, "far_terms": far, "leaves": leaves,
                           "p99_nodes": p99[0], "p99_far": p99[1], "p99_leaves": p99[2]},
        "no_prune": {"value": n / (ms_step_noprune * 1e-3), "ms_per_step": ms_step_noprune,
                     "nodes": float(cnt_np[:, 0].mean()), "far_terms": float(cnt_np[:, 1].mean()),
                     "leaves": float(cnt_np[:, 2].mean())},
    }

    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rng = np.random.default_rng(123)
        idx = np.sort(rng.choice(n, size=min(args.cpu_sample, n), replace=False))
        trees = [None, None, O.OracleTree(*api.sd_export_bvh(scene, 2))]
        osc = O.OracleScene(sc.V, T=sc.T)
        Qs = Q[idx].astype(np.float64)
        t0 = time.perf_counter()
        dr, gr, st = O.barnes_hut(osc, trees, Qs, args.alpha, args.beta)
        dt = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        d_s = d.cpu().numpy()[idx]
        dm_floor = 1e-3 * float(np.linalg.norm(sc.V.max(0) - sc.V.min(0)))
        ok = st[:, 0] > 1e-6
        err = O.value_error(d_s, dr, dm_floor)[ok]
        out["cpu_baseline"] = {
            "value": len(idx) / dt, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} random queries of the same workload, FP64 Barnes-Hut oracle "
                      f"on the exported hierarchy ({dt:.1f} s)",
        }
        out["parity_sample"] = {"max_rel_err_vs_oracle": float(err.max()),
                                "n": int(ok.sum()), "cut_ties_excluded": int((~ok).sum())}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
