"""Smooth-distance value+gradient throughput on one MI355X.

Headline workload (the largest single-GPU configuration): a 20M-point noisy
fBm terrain over [-1, 1]^2, a 1M-triangle torus above it and a 199,200-edge
hemispherical net; 32M FP32 queries uniform in the scene box enlarged by 10 %;
alpha = 100, beta = 0.5 (Barnes-Hut), the paper's blending weights, value and
gradient.  One step = Morton ordering of the queries + Alg. 1/Alg. 2 traversal
with value and gradient for every query (sd_query_order +
sd_eval_grad_ordered), inputs resident in HBM.  The hierarchy build is timed
separately.

Further legs (extra keys of the same JSON line): the 2,000-point sphere
(Barnes-Hut against brute force), the bumpy level-7 icosphere at alpha 50 and
500, the alpha sweep 10 / 100 / 1000 / 5000 on the headline scene, the learned
surrogate, the rigid-body street step; --headline-only skips them.

Prints one JSON line.  --gpus N > 1 is not supported: the library runs on one
GPU.
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
METRIC = "smooth-distance+grad queries/s on 1 MI355X: BH vs surrogate at ≤1e-5 rel / 1e-3 abs"
# Algorithmic work per query, value + gradient (not the instructions the
# kernel issues):
#   FLOPs = 20 per node visited + 25 per far-field term + 30 / 80 / 200 per
#           exact point / edge / triangle leaf term
#   bytes = 12 (query) + 16 (value, gradient) + 32 per node record
#           + 12 / 32 / 40 per point / edge / triangle leaf record
F_NODE, F_FAR, F_LEAF = 20, 25, (30, 80, 200)
B_QUERY, B_NODE, B_LEAF = 12 + 16, 32, (12, 32, 40)
ICO_ALPHAS = (50.0, 500.0)
SWEEP_ALPHAS = (10.0, 100.0, 1000.0, 5000.0)


def _progress(msg):
    """One line on stderr as each stage of the run starts (stdout keeps the
    single JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _sha(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(kernel_src, name, units):
    """HBM bytes of one launch over `units` work units (queries) from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by
    the same counters on a plain copy), or None when the kernel source changed
    since the counters were taken."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha") != _sha(kernel_src):
        return None
    return t["hbm_bytes_per_launch"] / t["units_per_launch"] * units


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _work(np, cnt):
    """Mean per-query work from the by-class counters (n x 5: nodes, far
    terms, point / edge / triangle leaves) -> (work dict, FLOPs, bytes)."""
    m = [float(x) for x in cnt.mean(0)]
    flops = F_NODE * m[0] + F_FAR * m[1] + sum(f * x for f, x in zip(F_LEAF, m[2:5]))
    nbytes = B_QUERY + B_NODE * m[0] + sum(b * x for b, x in zip(B_LEAF, m[2:5]))
    k = min(len(cnt), 200_000)
    p99 = np.quantile(cnt[:k], 0.99, axis=0)
    work = {"nodes": m[0], "far_terms": m[1], "point_leaves": m[2], "edge_leaves": m[3],
            "triangle_leaves": m[4], "p99_nodes": float(p99[0]), "p99_far": float(p99[1]),
            "p99_leaves": float(np.quantile(cnt[:k, 2:5].sum(1), 0.99))}
    return work, flops, nbytes


def _roofline(kernel, n, kernel_ms, flops_q, bytes_q, traffic):
    t = kernel_ms * 1e-3
    tflops = n * flops_q / t / 1e12
    out = {"bound": "alu", "kernel": kernel, "achieved": tflops, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": tflops / ALU_PEAK_TFLOPS, "traffic": traffic,
           "peak_note": "FP32 vector FMA rate of code built without packed-FP32 instructions "
                        "(256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz); the FP64 vector rate is the same",
           "frac_of_packed_peak": tflops / ALU_PEAK_PACKED_TFLOPS,
           "flops_per_query": flops_q,
           "flop_model": "20 per node + 25 per far-field term + 30/80/200 per point/edge/triangle leaf",
           "kernel_ms": kernel_ms,
           "algorithmic_bytes": {"per_query": bytes_q, "GB_per_s": n * bytes_q / t / 1e9,
                                 "note": "node and leaf records as read by the algorithm; most are served "
                                         "by L1/L2/MALL, so this is not an HBM figure"}}
    if traffic is not None:
        gbs = traffic / t / 1e9
        out["hbm_measured"] = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    return out


def _timed_steps(torch, step, steps, warmup):
    """warmup untimed steps, then `steps` timed ones between two events on the
    current stream; per-step events around the traversal (stage 1 -> 2)."""
    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for k in range(steps):
        step(ev[k])
    e1.record(s)
    torch.cuda.synchronize()
    total = e0.elapsed_time(e1)
    order = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    trav = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    return total / steps, order, trav


def _ordered_step(api, scene, Q, perm, d, g, alpha, beta, flags=0):
    def step(evs):
        if evs: evs[0].record()
        api.sd_query_order(scene, Q, out=perm)
        if evs: evs[1].record()
        api.sd_eval_grad_ordered(scene, Q, perm, alpha, beta, flags=flags, out=d, grad_out=g)
        if evs: evs[2].record()
    return step


def _parity(np, O, osc, trees, Qs, d, g, alpha, beta, floor, chunk=2_000_000):
    """Default outputs d, g of the sample Qs against the oracle (Barnes-Hut on
    the exported hierarchies, FP32 opening decisions), and d <= d_min against
    the oracle's exact nearest distance; in chunks with a progress line each,
    so that a large sample keeps reporting.  Returns (summary, seconds spent
    in the Barnes-Hut oracle)."""
    n = len(Qs)
    ev = np.empty(n)
    eg = np.empty(n)
    above = 0
    dt = 0.0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        t0 = time.perf_counter()
        dr, gr, _ = O.barnes_hut(osc, trees, Qs[a:b], alpha, beta, cut_f32=True)
        dt += time.perf_counter() - t0
        dm = O.dmin_tree(osc, trees, Qs[a:b])
        ev[a:b] = O.value_error(d[a:b], dr, floor)
        eg[a:b] = O.grad_error(g[a:b], gr)
        above += int(np.sum(d[a:b].astype(np.float64) > dm))
        if n > chunk:
            _progress(f"oracle parity {b}/{n}")
    return {"n": int(n), "max_err_vs_oracle": float(ev.max()), "max_grad_err_vs_oracle": float(eg.max()),
            "p999_err_vs_oracle": float(np.quantile(ev, 0.999)),
            "p9999_grad_err_vs_oracle": float(np.quantile(eg, 0.9999)),
            "metric": "|d - d_oracle| / max(|d_oracle|, 1e-3 scene diagonal); gradient "
                      "|g - g_oracle| / max(|g_oracle|, 1e-2); default (conservative) output",
            "gate_1e-5_met": bool(ev.max() <= 1e-5 and eg.max() <= 1e-5),
            "conservative_violations": above}, dt


def _compensated_row(np, torch, api, scene, Qd, perm, d, g, alpha, beta, steps, par_fn):
    """The same step with the running sums in compensated FP32
    (SD_LSE_COMPENSATED_F32) instead of FP64: time, and the parity sample
    (par_fn on the new outputs) when given."""
    ms, order_ms, trav = _timed_steps(torch, _ordered_step(api, scene, Qd, perm, d, g, alpha, beta,
                                                           flags=api.SD_LSE_COMPENSATED_F32), steps, 1)
    row = {"queries_per_s": len(Qd) / (ms * 1e-3), "ms_per_step": ms, "traversal_ms": trav}
    if par_fn is not None:
        row["parity_sample"] = par_fn()
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=100.0)
    ap.add_argument("--beta", type=float, default=0.5)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="headline scene size relative to 20M points, 1M triangles, 200k edges, 32M queries")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000,
                    help="queries of the headline workload timed on the FP64 oracle and checked against it")
    ap.add_argument("--headline-only", action="store_true", help="only the headline workload (for profiling)")
    ap.add_argument("--icosphere-only", type=float, default=None, metavar="ALPHA",
                    help="only the icosphere workload at this alpha (for profiling); prints its record")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate comparison")
    ap.add_argument("--no-rigid", action="store_true", help="skip the rigid-body street workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the alpha sweep on the headline scene")
    ap.add_argument("--rigid-steps", type=int, default=5)
    ap.add_argument("--sweep-oracle", type=int, default=20_000,
                    help="queries of each sweep alpha checked against the oracle")
    ap.add_argument("--beta-ablation", action=argparse.BooleanOptionalAction, default=True,
                    help="sphere-trace renders of vertex, edge and triangle scenes over beta (Sec. 4.3 analogue)")
    ap.add_argument("--ablation-res", type=int, default=256, help="image side of the beta ablation renders")
    ap.add_argument("--prims", action=argparse.BooleanOptionalAction, default=True,
                    help="edges and triangles as query primitives on the icosphere scene (Sec. 3.4)")
    ap.add_argument("--contact", action=argparse.BooleanOptionalAction, default=True,
                    help="rigid-body contact steps of the street body dropped on the street (Sec. 4.5)")
    ap.add_argument("--switch-study", action=argparse.BooleanOptionalAction, default=True,
                    help="near/far switch discrepancy beta 0.5 vs 0.5001 on the street points (Sec. 4.3 analogue)")
    ap.add_argument("--sur-train", type=int, default=20_000_000, help="surrogate training samples")
    ap.add_argument("--sur-epochs", type=int, default=80)
    ap.add_argument("--sur-c5-epochs", type=int, default=40, help="surrogate epochs on the terrain scene")
    ap.add_argument("--no-surrogate-c5", action="store_true", help="skip the surrogate on the terrain scene")
    ap.add_argument("--sur-nq", type=int, default=16_000_000, help="surrogate inference queries")
    ap.add_argument("--sur-oracle", type=int, default=20000, help="oracle-checked queries of the surrogate path")
    ap.add_argument("--sur-grid", type=int, default=32, help="cells per axis of the local certificate")
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
        print(f"bench.py: --gpus {args.gpus} is not supported; the library runs on one GPU "
              "(queries are independent: several GPUs would each take a share of them against a "
              "replicated scene)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2108_10480_amd import api, scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.icosphere_only is not None:
        res, _, scene = icosphere_leg(args, np, torch, api, scenes, alphas=(args.icosphere_only,))
        scene.free()
        print(json.dumps(res))
        return
    dev = torch.device("cuda:0")
    _progress("terrain scene and queries")
    sc = scenes.terrain_scene(args.scale)
    nq = max(int(round(32_000_000 * args.scale)), 1000)
    Q = scenes.terrain_queries(sc, nq, seed=10)
    cnt_cls = sc.counts()
    V = torch.as_tensor(sc.V, device=dev)
    P = torch.as_tensor(sc.P, device=dev)
    E = torch.as_tensor(sc.E, device=dev)
    T = torch.as_tensor(sc.T, device=dev)
    Qd = torch.as_tensor(Q, device=dev)
    torch.cuda.synchronize()

    _progress("hierarchy build")
    builds = []
    for _ in range(2):
        t0 = time.perf_counter()
        scene = api.sd_build_bvh(V, P=P, E=E, T=T)
        torch.cuda.synchronize()
        builds.append((time.perf_counter() - t0) * 1e3)
    del V, P, E, T

    _progress("headline steps")
    perm = torch.empty(nq, dtype=torch.int32, device=dev)
    d = torch.empty(nq, dtype=torch.float32, device=dev)
    g = torch.empty((nq, 3), dtype=torch.float32, device=dev)
    ms_step, order_ms, eval_ms = _timed_steps(torch, _ordered_step(api, scene, Qd, perm, d, g, args.alpha,
                                                                     args.beta), args.steps, args.warmup)
    qps = nq / (ms_step * 1e-3)
    workload = (f"terrain {cnt_cls[0]} points (fBm heightfield + noise) + torus {cnt_cls[2]} triangles + "
                f"hemisphere net {cnt_cls[1]} edges; {nq} queries uniform in the scene box enlarged by 10 %; "
                f"alpha={args.alpha:g}, beta={args.beta:g}, Barnes-Hut, value+gradient")
    out = {
        "metric": METRIC, "value": qps, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "mode": "barnes_hut", "n_points": cnt_cls[0], "n_edges": cnt_cls[1],
                   "n_triangles": cnt_cls[2], "n_queries": nq, "alpha": args.alpha, "beta": args.beta},
        "stages_ms": {"query_order": order_ms, "traversal": eval_ms, "build": min(builds)},
    }
    if args.headline_only:
        print(json.dumps(out))
        return

    _progress("work counters")
    cnt = api.sd_eval_counters(scene, Qd, args.alpha, args.beta, flags=api.SD_COUNTERS_BY_CLASS).cpu().numpy()
    work, flops_q, bytes_q = _work(np, cnt)
    del cnt
    out["work_per_query"] = work
    out["roofline"] = _roofline("k_eval (Barnes-Hut traversal, value+gradient, three classes)", nq, eval_ms,
                                flops_q, bytes_q,
                                _traffic(os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "eval.hip"),
                                         "traffic_k_eval_terrain_32M.json", nq))
    lo, hi = scenes.scene_aabb(sc)
    floor = 1e-3 * float(np.linalg.norm(hi - lo))
    O = osc = trees = None
    if not args.no_cpu_baseline:
        _progress("FP64 oracle on the host (cpu baseline, parity sample)")
        from oracle import oracle as O
        osc = O.OracleScene(sc.V, P=sc.P, E=sc.E, T=sc.T)
        trees = [O.OracleTree(*api.sd_export_bvh(scene, c)) for c in range(3)]
        rng = np.random.default_rng(123)
        k = min(args.cpu_sample, nq)
        idx = np.sort(rng.choice(nq, size=k, replace=False))
        idx_d = torch.as_tensor(idx, device=dev)
        par, dt = _parity(np, O, osc, trees, Q[idx].astype(np.float64), d[idx_d].cpu().numpy(),
                          g[idx_d].cpu().numpy(), args.alpha, args.beta, floor)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {
            "value": k / dt, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} random queries of the headline workload, FP64 Barnes-Hut oracle on the exported "
                      f"hierarchies (Alg. 1/Alg. 2, every term in FP64), {dt:.1f} s",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}
        out["parity_sample"] = par
    _progress("compensated FP32 sums")
    par_fn = None
    if not args.no_cpu_baseline:
        sub, sub_d = idx[:100_000], idx_d[:100_000]
        par_fn = lambda: _parity(np, O, osc, trees, Q[sub].astype(np.float64), d[sub_d].cpu().numpy(),
                                 g[sub_d].cpu().numpy(), args.alpha, args.beta, floor)[0]
    out["lse_compensated_f32"] = {
        "what": "the headline step with the running sums of Eq. 3-4 in compensated FP32 (Neumaier, product "
                "errors by FMA) instead of FP64; log-terms FP64 in both",
        "fp64_sums": {"queries_per_s": qps, "ms_per_step": ms_step, "traversal_ms": eval_ms},
        "compensated_f32_sums": _compensated_row(np, torch, api, scene, Qd, perm, d, g, args.alpha, args.beta,
                                                 max(3, args.steps // 4), par_fn)}
    if not args.no_surrogate and not args.no_surrogate_c5:
        _progress("surrogate on the terrain scene")
        out["surrogate_terrain"] = surrogate_leg(args, sc, scene, np, torch, api, scenes, terrain=True, Xin=Qd)
    if not args.no_sweep:
        out["alpha_sweep"] = alpha_sweep_leg(args, np, torch, api, scene, Qd, perm, d, g, O, osc, trees, Q,
                                             floor)
    del d, g, perm
    if not args.no_cpu_baseline:
        del trees
    scene.free()
    del Qd

    out["point_sphere"] = point_sphere_leg(args, np, torch, api, scenes)
    ico, ico_sc, ico_scene = icosphere_leg(args, np, torch, api, scenes)
    out["icosphere"] = ico
    if not args.no_surrogate:
        _progress("surrogate")
        out["surrogate"] = surrogate_leg(args, ico_sc, ico_scene, np, torch, api, scenes)
    if args.prims:
        _progress("query primitives")
        out["query_primitives"] = prims_leg(args, np, torch, api, scenes, ico_sc, ico_scene)
    ico_scene.free()
    if not args.no_rigid:
        _progress("rigid")
        out["rigid"] = rigid_leg(args, np, torch, api, scenes)
    if args.contact:
        _progress("contact")
        out["contact"] = contact_leg(args, np, torch, api, scenes)
    if args.beta_ablation:
        _progress("beta ablation")
        out["beta_ablation"] = beta_ablation_leg(args, np, torch, api, scenes)
    if args.switch_study:
        _progress("switch study")
        out["switch_study"] = switch_study_leg(args, np, torch, api, scenes)
    print(json.dumps(out))


def alpha_sweep_leg(args, np, torch, api, scene, Qd, perm, d, g, O, osc, trees, Q, floor):
    """alpha = 10, 100, 1000, 5000 on the headline scene and queries:
    throughput (ordering + traversal), work per query and, on a random
    sample, the default output against the oracle and d <= d_min."""
    nq = len(Q)
    rng = np.random.default_rng(456)
    k = min(args.sweep_oracle, nq)
    idx = np.sort(rng.choice(nq, size=k, replace=False))
    idx_d = torch.as_tensor(idx, device="cuda")
    Qs = Q[idx].astype(np.float64)
    res = {"workload": "headline scene and queries; oracle sample of "
                       f"{k} random queries per alpha", "alphas": {}}
    for alpha in SWEEP_ALPHAS:
        _progress(f"alpha sweep: {alpha:g}")
        ms, _, trav = _timed_steps(torch, _ordered_step(api, scene, Qd, perm, d, g, alpha, args.beta), 3, 1)
        c = api.sd_eval_counters(scene, Qd[idx_d], alpha, args.beta, flags=api.SD_COUNTERS_BY_CLASS).cpu().numpy()
        work, flops_q, _ = _work(np, c)
        row = {"queries_per_s": nq / (ms * 1e-3), "ms_per_step": ms, "traversal_ms": trav,
               "roofline_frac": nq * flops_q / (trav * 1e-3) / 1e12 / ALU_PEAK_TFLOPS,
               "work_per_query_on_sample": {k2: work[k2] for k2 in ("nodes", "far_terms", "point_leaves",
                                                                    "edge_leaves", "triangle_leaves")}}
        if O is not None:
            row["parity_sample"], _ = _parity(np, O, osc, trees, Qs, d[idx_d].cpu().numpy(), g[idx_d].cpu().numpy(),
                                              alpha, args.beta, floor)
        res["alphas"][f"{alpha:g}"] = row
    return res


def point_sphere_leg(args, np, torch, api, scenes):
    """The 2,000-point sphere (radial noise 0.005) with 10,000 uniform queries,
    alpha = 100: Barnes-Hut (beta 0.5) against brute force (beta 0, the
    traversal opening every node, and the all-pairs kernel); each against the
    oracle on every query."""
    _progress("point sphere")
    sc, Q = scenes.point_sphere(2000, 10000)
    scene = api.upload_scene(sc)
    Qd = torch.as_tensor(Q, device="cuda")
    alpha = 100.0
    n = len(Q)

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            r = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps, r

    ms_bh, (d_bh, g_bh) = timed(lambda: api.sd_eval_grad(scene, Qd, alpha, args.beta))
    ms_b0, (d_b0, g_b0) = timed(lambda: api.sd_eval_grad(scene, Qd, alpha, 0.0))
    ms_all, (d_all, g_all) = timed(lambda: api.sd_eval_brute(scene, Qd, alpha))
    res = {"workload": f"{len(sc.P)} points on the unit sphere (radial N(0, 0.005^2)), {n} queries uniform in "
                       f"[-1.5, 1.5]^3, alpha={alpha:g}, value+gradient",
           "barnes_hut": {"beta": args.beta, "queries_per_s": n / (ms_bh * 1e-3), "ms": ms_bh},
           "brute_force_traversal": {"beta": 0.0, "queries_per_s": n / (ms_b0 * 1e-3), "ms": ms_b0},
           "brute_force_all_pairs": {"queries_per_s": n / (ms_all * 1e-3), "ms": ms_all}}
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        osc = O.OracleScene(sc.V, P=sc.P)
        trees = [O.OracleTree(*api.sd_export_bvh(scene, 0)), None, None]
        lo, hi = scenes.scene_aabb(sc)
        floor = 1e-3 * float(np.linalg.norm(hi - lo))
        Q64 = Q.astype(np.float64)
        res["barnes_hut"]["parity"], _ = _parity(np, O, osc, trees, Q64, d_bh.cpu().numpy(), g_bh.cpu().numpy(),
                                                 alpha, args.beta, floor)
        dr, gr, dm = O.brute(osc, Q64, alpha)
        for key, (dd, gg) in (("brute_force_traversal", (d_b0, g_b0)), ("brute_force_all_pairs", (d_all, g_all))):
            dd, gg = dd.cpu().numpy(), gg.cpu().numpy()
            res[key]["parity"] = {"n": n, "max_err_vs_oracle": float(O.value_error(dd, dr, floor).max()),
                                  "max_grad_err_vs_oracle": float(O.grad_error(gg, gr).max()),
                                  "conservative_violations": int(np.sum(dd.astype(np.float64) > dm))}
        # Barnes-Hut against the exact smooth distance: the price of the far field
        eb = np.abs(d_bh.cpu().numpy() - dr)
        res["barnes_hut"]["vs_exact_smooth_distance"] = {"max_abs": float(eb.max()), "mean_abs": float(eb.mean())}
    scene.free()
    return res


def icosphere_leg(args, np, torch, api, scenes, alphas=ICO_ALPHAS):
    """The bumpy level-7 icosphere (327,680 triangles) with 1M queries (half
    uniform in [-1.5, 1.5]^3, half within 0.02 of the surface) at alpha 50
    and 500: throughput, work, roofline fraction, and a 200,000-query sample
    of the default output against the oracle with d <= d_min."""
    _progress("icosphere")
    sc = scenes.bumpy_icosphere(level=7, seed=2)
    n = 1_000_000
    Q = scenes.icosphere_queries(sc, n, seed_box=3, seed_surf=4)
    t0 = time.perf_counter()
    scene = api.upload_scene(sc)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    Qd = torch.as_tensor(Q, device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.empty(n, device="cuda")
    g = torch.empty((n, 3), device="cuda")
    res = {"workload": f"bumpy icosphere level 7 ({len(sc.T)} triangles), {n} queries (half uniform in "
                       f"[-1.5,1.5]^3, half within 0.02 of the surface), beta={args.beta:g}, value+gradient",
           "build_ms": build_ms, "alphas": {}}
    O = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        osc = O.OracleScene(sc.V, T=sc.T)
        trees = [None, None, O.OracleTree(*api.sd_export_bvh(scene, 2))]
        lo, hi = scenes.scene_aabb(sc)
        floor = 1e-3 * float(np.linalg.norm(hi - lo))
        idx = np.sort(np.random.default_rng(789).choice(n, size=200_000, replace=False))
        idx_d = torch.as_tensor(idx, device="cuda")
    for alpha in alphas:
        ms, order_ms, trav = _timed_steps(torch, _ordered_step(api, scene, Qd, perm, d, g, alpha, args.beta), 20, 3)
        c = api.sd_eval_counters(scene, Qd, alpha, args.beta, flags=api.SD_COUNTERS_BY_CLASS).cpu().numpy()
        work, flops_q, bytes_q = _work(np, c)
        row = {"queries_per_s": n / (ms * 1e-3), "ms_per_step": ms, "query_order_ms": order_ms,
               "traversal_ms": trav, "work_per_query": work,
               "roofline": _roofline("k_eval (triangles)", n, trav, flops_q, bytes_q,
                                     _traffic(os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "eval.hip"),
                                              f"traffic_k_eval_icosphere_l7_1M_a{alpha:g}.json", n))}
        if O is not None:
            row["parity_sample"], _ = _parity(np, O, osc, trees, Q[idx].astype(np.float64), d[idx_d].cpu().numpy(),
                                              g[idx_d].cpu().numpy(), alpha, args.beta, floor)
        par_fn = None
        if O is not None:
            par_fn = lambda: _parity(np, O, osc, trees, Q[idx].astype(np.float64), d[idx_d].cpu().numpy(),
                                     g[idx_d].cpu().numpy(), alpha, args.beta, floor)[0]
        row["compensated_f32_sums"] = _compensated_row(np, torch, api, scene, Qd, perm, d, g, alpha, args.beta,
                                                       20, par_fn)
        res["alphas"][f"{alpha:g}"] = row
    return res, sc, scene


def _camera_rays(np, res, eye, fov_deg=40.0):
    """Pinhole camera at eye looking at the origin: res x res unit rays."""
    eye = np.asarray(eye, np.float64)
    f = -eye / np.linalg.norm(eye)
    r = np.cross(f, [0.0, 0.0, 1.0])
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    s = np.tan(np.radians(fov_deg) / 2)
    g = (np.arange(res) + 0.5) / res * 2 - 1
    px, py = np.meshgrid(g * s, -g * s)
    D = f[None] + px.reshape(-1, 1) * r[None] + py.reshape(-1, 1) * u[None]
    D /= np.linalg.norm(D, axis=1, keepdims=True)
    return np.tile(eye, (len(D), 1)).astype(np.float32), D.astype(np.float32)


def prims_leg(args, np, torch, api, scenes, sc, scene):
    """Edges and triangles as query primitives (Sec. 3.4) on the icosphere
    scene: 1M small random segments / triangles placed like the point queries
    (half uniform in the box, half near the surface), alpha 50, beta 0.5;
    throughput and an oracle sample."""
    rng = np.random.default_rng(31)
    n = 1_000_000
    alpha, beta = ICO_ALPHAS[0], args.beta
    C = scenes.icosphere_queries(sc, n, seed_box=32, seed_surf=33)
    out = {"workload": f"bumpy icosphere level 7 ({len(sc.T)} triangles), {n} query primitives "
                       f"(random segments / triangles of size ~0.02 at the point-query positions), "
                       f"alpha={alpha:g}, beta={beta:g}, value+gradient"}
    for nv, name in ((2, "edges"), (3, "triangles")):
        G = (C[:, None, :] + rng.normal(size=(n, nv, 3)) * 0.01).astype(np.float32)
        Gd = torch.as_tensor(G, device="cuda")
        api.sd_eval_grad_prims(scene, Gd, alpha, beta)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            d, g = api.sd_eval_grad_prims(scene, Gd, alpha, beta)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 3
        row = {"ms": ms, "value": n / (ms * 1e-3), "unit": "query primitives/s"}
        if not args.no_cpu_baseline:
            from oracle import oracle as O
            idx = np.sort(rng.choice(n, 2000, replace=False))
            osc = O.OracleScene(sc.V, T=sc.T)
            trees = [None, None, O.OracleTree(*api.sd_export_bvh(scene, 2))]
            dn, _ = api.sd_eval_grad_prims(scene, Gd[torch.as_tensor(idx, device="cuda")], alpha, beta)
            dr, _, _ = O.barnes_hut_prims(osc, trees, G[idx].astype(np.float64), alpha, beta, cut_f32=True)
            _, _, dm = O.brute_prims(osc, G[idx[:200]].astype(np.float64), alpha)
            floor = 1e-3 * float(np.linalg.norm(sc.V.max(0) - sc.V.min(0)))
            e = O.value_error(dn.cpu().numpy(), dr, floor)
            row["parity_sample"] = {"n": len(idx), "max_err_vs_oracle": float(e.max()),
                                    "median_err_vs_oracle": float(np.median(e)),
                                    "conservative_violations_of_200": int(np.sum(d[torch.as_tensor(idx[:200],
                                                                           device="cuda")].cpu().numpy() > dm))}
        out[name] = row
    return out


def contact_leg(args, np, torch, api, scenes):
    """Frictionless rigid-body contact (Sec. 4.5): the street body (a torus)
    dropped onto the street scene at scale 0.1;
    implicit steps of 10 ms, each a sequential-quadratic-programming solve of
    one smooth-distance constraint (value and gradient on the GPU)."""
    from paper_2108_10480_amd import contact as C
    sc, body_v = scenes.street_scene(0.1)
    scene = api.upload_scene(sc)
    lo, hi = scenes.scene_aabb(sc)
    # start 0.3 m above the highest scene vertex under the body's footprint
    x0, y0 = 0.5 * (lo[0] + hi[0]), 0.0
    ext = float(np.abs(body_v - body_v.mean(0)).max())
    near = (np.abs(sc.V[:, 0] - x0) < ext) & (np.abs(sc.V[:, 1] - y0) < ext)
    ground = float(sc.V[near, 2].max()) if near.any() else float(lo[2])
    start = (x0, y0, ground + ext + 0.3)
    body = C.RigidBody(body_v, mass=10.0, p=start, omega=(0.0, 0.5, 0.2))
    step = C.ContactStep(scene, alpha=50.0, alpha_q=50.0, d_safe=0.05, h=0.01)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, evals0 = [], step.evals
    nsteps = 80
    for _ in range(nsteps):
        it, c = step.step(body)
        iters.append(it)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    evals = step.evals - evals0
    return {"workload": f"street scene at scale 0.1 ({sc.counts()[0]} points, {sc.counts()[1]} wire segments, "
                        f"{sc.counts()[2]} triangles); body of {len(body_v)} vertices dropped, "
                        f"alpha=alpha_q=50, d_safe=0.05, h=0.01, {nsteps} steps from 0.3 m above the scene under it",
            "ms_per_step": dt / nsteps * 1e3, "sqp_iterations_mean": float(np.mean(iters)),
            "sqp_iterations_max": int(np.max(iters)), "solves_not_converged": step.stalls,
            "solves_ended_infeasible": step.infeasible, "constraint_target_c_res": step.c_res,
            "constraint_evaluations": evals, "exact_evaluations_near_contact": step.exact_evals,
            "exact_band": step.exact_band, "ms_per_evaluation": dt / evals * 1e3,
            "start_height_above_ground": float(start[2] - ground), "final_height_above_ground": float(body.p[2] - ground),
            "final_speed": float(np.linalg.norm(body.v))}


def beta_ablation_leg(args, np, torch, api, scenes):
    """Synthetic analogue of the beta ablation (Sec. 4.3): sphere-trace the zero
    isosurface of the vertices, the edges and the triangles of a bumpy
    icosphere (level 5: 10,242 vertices, 30,720 edges, 20,480 triangles) with
    alpha 200, alpha_U 1200; render time per beta and the distance along each
    ray between the beta isosurface and the exact one (beta = 0), relative to
    the bounding-box diagonal."""
    mesh = scenes.bumpy_icosphere(level=5, seed=2)
    V, T = mesh.V, mesh.T
    E = np.unique(np.sort(np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]]), axis=1), axis=0).astype(np.int32)
    lo, hi = V.min(0), V.max(0)
    diag = float(np.linalg.norm(hi - lo))
    res = args.ablation_res
    Oo, U = _camera_rays(np, res, (0.0, -3.2, 1.2))
    Od, Ud = torch.as_tensor(Oo, device="cuda"), torch.as_tensor(U, device="cuda")
    betas = [0.0, 0.1, 0.2, 0.3, 0.5, 0.75, 1.0]
    alpha, alpha_u = 200.0, 1200.0
    kw = dict(level=0.0, eps=1e-4 * diag, t_max=8.0, max_steps=1000)
    out = {"workload": f"bumpy icosphere level 5 ({len(V)} vertices, {len(E)} edges, {len(T)} triangles), "
                       f"{res}x{res} rays, alpha={alpha:g}, alpha_U={alpha_u:g}, eps={kw['eps']:.2g}",
           "bbox_diagonal": diag, "scenes": {}}
    for name, sc in (("vertices", scenes.Scene(V=V, P=np.arange(len(V), dtype=np.int32))),
                     ("edges", scenes.Scene(V=V, E=E)), ("triangles", scenes.Scene(V=V, T=T))):
        scene = api.upload_scene(sc)
        rows, t0 = {}, None
        for beta in betas:
            api.sd_sphere_trace(scene, Od, Ud, alpha, beta, alpha_u, **kw)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            t, st = api.sd_sphere_trace(scene, Od, Ud, alpha, beta, alpha_u, **kw)
            b.record()
            torch.cuda.synchronize()
            t = t.cpu().numpy().astype(np.float64)
            row = {"ms": a.elapsed_time(b), "hits": int(np.isfinite(t).sum()),
                   "mean_steps": float(st.double().mean())}
            if t0 is None:
                t0 = t
            else:
                both = np.isfinite(t) & np.isfinite(t0)
                e = np.abs(t[both] - t0[both]) / diag
                row.update({"speedup_vs_exact": rows["0"]["ms"] / row["ms"],
                            "err_mean_rel_diag": float(e.mean()), "err_p99_rel_diag": float(np.quantile(e, 0.99)),
                            "err_max_rel_diag": float(e.max()),
                            "hit_mismatch": int(np.sum(np.isfinite(t) != np.isfinite(t0)))})
            rows[f"{beta:g}"] = row
        out["scenes"][name] = rows
        scene.free()
    return out


def switch_study_leg(args, np, torch, api, scenes):
    """Synthetic analogue of the near/far switch study (Sec. 4.3): on the street
    scene's lidar-like points, trace vertical rays from the top of the box to
    the 0.1 isosurface (beta 0.5), step on downwards, and wherever beta 0.5001
    takes a different cut than beta 0.5 (fewer nodes visited) compare the two
    values and gradients."""
    sc, _ = scenes.street_scene(0.1)
    pts = scenes.Scene(V=sc.V, P=sc.P)
    scene = api.upload_scene(pts)
    lo, hi = scenes.scene_aabb(pts)
    diag = float(np.linalg.norm(hi - lo))
    alpha, b0, b1 = 50.0, 0.5, 0.5001
    rng = np.random.default_rng(11)
    n = 65536
    Oo = np.column_stack([rng.uniform(lo[0], hi[0], n), rng.uniform(lo[1], hi[1], n),
                          np.full(n, hi[2] + 1.0)]).astype(np.float32)
    U = np.tile(np.array([0.0, 0.0, -1.0], np.float32), (n, 1))
    t, _ = api.sd_sphere_trace(scene, torch.as_tensor(Oo, device="cuda"), torch.as_tensor(U, device="cuda"),
                               alpha, b0, level=0.1, eps=1e-4, t_max=float(hi[2] - lo[2] + 2.0), max_steps=2000)
    t = t.cpu().numpy()
    ok = np.isfinite(t)
    P0 = Oo[ok] + t[ok, None] * U[ok]
    h = 1e-3
    Ps = np.concatenate([P0 + k * h * U[ok] for k in range(16)]).astype(np.float32)
    Pd = torch.as_tensor(Ps, device="cuda")
    c0 = api.sd_eval_counters(scene, Pd, alpha, b0).cpu().numpy()
    c1 = api.sd_eval_counters(scene, Pd, alpha, b1).cpu().numpy()
    d0, g0 = api.sd_eval_grad(scene, Pd, alpha, b0)
    d1, g1 = api.sd_eval_grad(scene, Pd, alpha, b1)
    d0, g0, d1, g1 = (x.cpu().numpy().astype(np.float64) for x in (d0, g0, d1, g1))
    sw = c1[:, 0] < c0[:, 0]
    dd = np.abs(d1[sw] - d0[sw])
    cos = np.sum(g0[sw] * g1[sw], 1) / np.maximum(np.linalg.norm(g0[sw], axis=1) * np.linalg.norm(g1[sw], axis=1),
                                                   1e-30)
    scene.free()
    return {"workload": f"street points ({len(sc.P)}), alpha={alpha:g}, vertical rays from the top of the box to "
                        f"the 0.1 isosurface ({int(ok.sum())} of {n} hit), 16 points each at spacing {h:g}",
            "bbox_diagonal": diag, "points": int(len(Ps)), "switch_points": int(sw.sum()),
            "value_discrepancy_mean": float(dd.mean()) if dd.size else None,
            "value_discrepancy_max": float(dd.max()) if dd.size else None,
            "gradient_cosine_mean": float(cos.mean()) if cos.size else None,
            "gradient_cosine_min": float(cos.min()) if cos.size else None}


def rigid_leg(args, np, torch, api, scenes):
    """Differentiable rigid-body step on the mixed street scene: 256 rigid
    transforms of a 25,000-vertex torus (6.4M queries) against 2M points,
    20,000 wire segments and the 50,000-triangle torus at rest; forward
    (transform, order, Barnes-Hut value+gradient, the query-mesh distance
    D_k of each placement, Eq. 6) and the hand-written adjoint of sum_k D_k
    in (R, t, X)."""
    alpha, beta, alpha_q = 50.0, 0.5, 50.0
    ev = lambda: torch.cuda.Event(enable_timing=True)
    sc, body = scenes.street_scene(1.0)
    t0 = time.perf_counter()
    scene = api.upload_scene(sc)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    R, t = scenes.rigid_transforms(256, seed=5)
    X = torch.as_tensor(body, device="cuda")
    Rd = torch.as_tensor(R, device="cuda")
    td = torch.as_tensor(t, device="cuda")
    K, m = R.shape[0], body.shape[0]
    n = K * m
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.empty(n, device="cuda")
    g = torch.empty((n, 3), device="cuda")
    L = api.lib()

    def step(evs=None):
        if evs: evs[0].record()
        Q = api.sd_rigid_transform(X, Rd, td)
        if evs: evs[1].record()
        api.sd_query_order(scene, Q, out=perm)
        api.sd_eval_grad_ordered(scene, Q, perm, alpha, beta, out=d, grad_out=g)
        if evs: evs[2].record()
        # D_k and dD_k/dd_kj; dL/dD_k = 1 for L = sum_k D_k
        D, w, _ = api.sd_query_mesh_lse(d.reshape(K, m), None, alpha_q, want_vgrad=False)
        if evs: evs[3].record()
        out = api.sd_rigid_adjoint(X, Rd, w, g)
        if evs: evs[4].record()
        return Q, D, out

    step()
    torch.cuda.synchronize()
    evs = [[ev() for _ in range(5)] for _ in range(args.rigid_steps)]
    a, b = ev(), ev()
    a.record()
    for k in range(args.rigid_steps):
        Q, Dk, _ = step(evs[k])
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.rigid_steps
    st = lambda i, j: float(np.mean([e[i].elapsed_time(e[j]) for e in evs]))
    ms_adj = st(3, 4)
    ms_qm = st(2, 3)
    # query-mesh pass: d read three times (minimum, sum, weights), w written
    qm_bytes = n * 16
    cnt = api.sd_eval_counters(scene, Q[:200000].contiguous(), alpha, beta).double().mean(0).cpu().numpy()
    adj_bytes = n * (4 + 12) + m * 12 + K * (9 + 3) * 4 * 2
    res = {
        "workload": f"street scene: {sc.counts()[0]} points, {sc.counts()[1]} wire segments, "
                    f"{sc.counts()[2]} torus triangles; {K} rigid transforms x {m} body vertices = {n} "
                    f"queries, alpha={alpha:g}, beta={beta:g}, value+gradient and adjoint in (R, t, X)",
        "value": n / (ms * 1e-3), "unit": "queries/s (forward + adjoint)", "ms_per_step": ms,
        "stages_ms": {"transform": st(0, 1), "order_and_traversal": st(1, 2), "query_mesh_lse": ms_qm,
                      "adjoint": ms_adj, "build": build_ms},
        "query_mesh": {"alpha_q": alpha_q, "instances": K, "D_min": float(Dk.min()), "D_max": float(Dk.max()),
                       "roofline": {"bound": "hbm", "achieved": qm_bytes / (ms_qm * 1e-3) / 1e9,
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": qm_bytes / (ms_qm * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                    "bytes_per_query": 16, "traffic": None}},
        "work_per_query": {"nodes": float(cnt[0]), "far_terms": float(cnt[1]), "leaves": float(cnt[2])},
        "adjoint_roofline": {"bound": "hbm", "achieved": adj_bytes / (ms_adj * 1e-3) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": adj_bytes / (ms_adj * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "bytes_per_query": adj_bytes / n, "traffic": None},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        rng = np.random.default_rng(77)
        idx = np.sort(rng.choice(n, size=2000, replace=False))
        Qs = Q[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.float64)
        osc = O.OracleScene(sc.V, P=sc.P, E=sc.E, T=sc.T)
        trees = [O.OracleTree(*api.sd_export_bvh(scene, c)) for c in range(3)]
        t0 = time.perf_counter()
        dr, gr, stt = O.barnes_hut(osc, trees, Qs, alpha, beta, cut_f32=True)
        dt = time.perf_counter() - t0
        lo, hi = scenes.scene_aabb(sc)
        floor = 1e-3 * float(np.linalg.norm(hi - lo))
        dg = d[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        gg = g[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        err = O.value_error(dg, dr, floor)
        dm = O.dmin_tree(osc, trees, Qs)
        res["parity_sample"] = {"n": len(dg), "max_err_vs_oracle": float(err.max()),
                                "max_grad_err_vs_oracle": float(O.grad_error(gg, gr).max()),
                                "conservative_violations": int(np.sum(dg.astype(np.float64) > dm)),
                                "oracle_queries_per_s": len(idx) / dt}
        # query-mesh distance of two whole placements against the oracle composite
        from oracle import qmesh as QM
        Qk = Q[: 2 * m].cpu().numpy().astype(np.float64)
        dk, gk, _ = O.barnes_hut(osc, trees, Qk, alpha, beta, cut_f32=True)
        Dr = QM.query_mesh_lse(dk.reshape(2, m), gk.reshape(2, m, 3), alpha_q)[0]
        Dg = Dk[:2].cpu().numpy().astype(np.float64)
        res["query_mesh"]["parity_sample"] = {
            "instances": 2, "max_err_vs_oracle": float(np.max(np.abs(Dg - Dr) / np.maximum(np.abs(Dr), floor))),
            "metric": "|D - D_oracle| / max(|D_oracle|, 1e-3 scene diagonal); d with the default conservative rounding"}
    return res


MFMA_BF16_PEAK_TFLOPS = 2500.0
# matrix-product FLOPs per query of the surrogate: forward 128x256 + 3 x 256x256
# + 256 multiply-adds, input gradient the same minus the output layer
SUR_FWD_MACS = 128 * 256 + 3 * 256 * 256 + 256
SUR_BWD_MACS = 128 * 256 + 3 * 256 * 256


def surrogate_leg(args, sc, scene, np, torch, api, scenes, terrain=False, Xin=None):
    """Learned surrogate on one scene: train on labels from the exact
    evaluation, certify on held-out queries, then answer the scene's queries
    with routing of the certified band to Barnes-Hut, compared with
    Barnes-Hut alone on the same queries.  The frontier of the fixed network:
    validation error along training, and fallback fraction / speed / error
    outside the band against the cap on a cell's certified margin."""
    from paper_2108_10480_amd import surrogate as S
    beta, band = args.beta, 0.05
    if terrain:
        alpha, epochs = args.alpha, args.sur_c5_epochs
        lo, hi = scenes.scene_aabb(sc)
        lo, hi = lo - 0.1 * (hi - lo), hi + 0.1 * (hi - lo)
        Xtr_h = scenes.terrain_surrogate_samples(sc, args.sur_train, seed=6)
        Xva_h = scenes.terrain_queries(sc, 2_000_000, seed=7)
        what = f"terrain scene, {len(Xin)} headline queries (uniform in the scene box enlarged by 10 %)"
    else:
        alpha, epochs = ICO_ALPHAS[0], args.sur_epochs
        lo, hi = np.full(3, -1.5), np.full(3, 1.5)
        Xtr_h = scenes.surrogate_samples(sc, args.sur_train, seed=6)
        Xva_h = scenes.uniform_queries(2_000_000, 7, -1.5, 1.5)
        Xin = torch.as_tensor(scenes.uniform_queries(args.sur_nq, 8, -1.5, 1.5), device="cuda")
        what = f"same scene, {args.sur_nq} queries uniform in [-1.5,1.5]^3"
    lo, hi = tuple(float(x) for x in lo), tuple(float(x) for x in hi)
    ev = lambda: torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    Xtr = torch.as_tensor(Xtr_h, device="cuda")
    del Xtr_h
    ytr = api.sd_eval(scene, Xtr, alpha, beta)
    Xva = torch.as_tensor(Xva_h, device="cuda")
    yva = api.sd_eval(scene, Xva, alpha, beta)
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    sur = S.Surrogate(scenes.fourier_matrix(11, sigma=[0.5, 1.0, 2.0, 4.0]), scenes.surrogate_init(12),
                      max_batch=65536)
    curve = []

    def on_epoch(e, k):
        if e in (1, 2, 5, 10, 20, 40, 80, epochs):
            err = (sur.forward(Xva, grad=False) - yva).abs()
            curve.append({"epoch": e, "steps": k, "max_abs_err": float(err.max()),
                          "p99_abs_err": float(torch.quantile(err[:1_000_000], 0.99)),
                          "rmse": float((err ** 2).mean().sqrt())})
    t0 = time.perf_counter()
    losses = S.train(sur, Xtr, ytr, epochs, batch=65536, lr0=3e-3, lr_min=1e-5, seed=13, on_epoch=on_epoch)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = len(losses)
    del Xtr, ytr
    eps = sur.certify(Xva, yva, safety=1.5)
    yv = sur.forward(Xva, grad=False)
    verr = (yv - yva).abs()

    n = len(Xin)
    d = torch.empty(n, device="cuda")
    g = torch.empty((n, 3), device="cuda")
    routed = torch.empty(n, dtype=torch.uint8, device="cuda")
    de = torch.empty(n, device="cuda")
    ge = torch.empty((n, 3), device="cuda")
    perm = torch.empty(n, dtype=torch.int32, device="cuda")

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    def sur_path():
        S.sd_eval_surrogate(scene, sur, Xin, alpha, beta, band=band, out=d, grad_out=g, routed=routed)

    def bh_path():
        api.sd_query_order(scene, Xin, out=perm)
        api.sd_eval_grad_ordered(scene, Xin, perm, alpha, beta, out=de, grad_out=ge)

    ms_bh = timed(bh_path)
    ms_mlp = timed(lambda: sur.forward(Xin, grad=True))

    def routed_run():
        ms = timed(sur_path)
        _, _, _, nfb = S.sd_eval_surrogate(scene, sur, Xin, alpha, beta, band=band, out=d, grad_out=g,
                                           routed=routed)
        nfb = int(nfb)
        torch.cuda.synchronize()
        keep = routed == 0
        e_out = (d - de).abs()[keep]
        e_routed = (d - de).abs()[~keep]
        return ms, nfb, keep, {
            "fallback_fraction": nfb / n,
            "value_surrogate_path": n / (ms * 1e-3),
            "speedup_vs_barnes_hut": ms_bh / ms,
            "ms_surrogate_path": ms,
            "vs_exact_outside_band": ({"max_abs_err": float(e_out.max()),
                                       "p99_abs_err": float(torch.quantile(e_out[:1_000_000], 0.99)),
                                       "gate_1e-3_met": bool(float(e_out.max()) <= 1e-3)}
                                      if e_out.numel() else {"max_abs_err": None, "note": "every query routed"}),
            "routed_vs_exact_max_abs_diff": float(e_routed.max()) if e_routed.numel() else 0.0,
        }

    # global certificate (one margin everywhere), then a local one (cells),
    # then the local one with the cells' margins capped (cells above the cap
    # route every query): the speed / error frontier of this network
    ms_sur, nfb, keep, glob = routed_run()
    sur.certify_cells(Xva, yva, lo=lo, hi=hi, grid=args.sur_grid, safety=1.5)
    _, _, keep_local, loc = routed_run()
    frontier = []
    for cap in (1e-3, 3e-3, 1e-2, 3e-2):
        sur.certify_cells(Xva, yva, lo=lo, hi=hi, grid=args.sur_grid, safety=1.5, max_margin=cap)
        _, _, _, row = routed_run()
        frontier.append(dict(row, max_margin=cap))
    gate = frontier[0]
    sur.certify_cells(Xva, yva, lo=lo, hi=hi, grid=args.sur_grid, safety=1.5)
    routed_run()
    flops = n * 2.0 * (SUR_FWD_MACS + SUR_BWD_MACS)
    res = {
        "workload": f"{what}, alpha={alpha:g}, beta={beta:g}, band={band} + certified margin",
        "network": "3 -> 64 Fourier frequencies (sigma 0.5/1/2/4) -> 4 x 256 SiLU -> 1, BF16 weights, "
                   "FP32 accumulation",
        "train": {"samples": args.sur_train, "epochs": epochs, "steps": steps, "seconds": t_train,
                  "label_seconds": t_label, "loss_last": float(np.mean(losses[-50:])),
                  "ms_per_step": 1e3 * t_train / steps},
        "training_curve": curve,
        "eps_cert": eps,
        "validation": {"n": int(Xva.shape[0]), "max_abs_err": float(verr.max()),
                       "rmse": float((verr ** 2).mean().sqrt()),
                       "p99_abs_err": float(torch.quantile(verr[:1_000_000], 0.99))},
        "unit": "queries/s",
        "value_barnes_hut": n / (ms_bh * 1e-3),
        "ms": {"barnes_hut": ms_bh, "mlp_value_grad": ms_mlp},
        "global_certificate": glob,
        "local_certificate": dict(loc, grid=args.sur_grid),
        "local_certificate_1e-3_target": dict(gate, grid=args.sur_grid),
        "frontier_by_margin_cap": frontier,
        "roofline": {"bound": "mfma", "kernel": "k_mlp_grad (value + input gradient)",
                     "achieved": flops / (ms_mlp * 1e-3) / 1e12, "peak": MFMA_BF16_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": flops / (ms_mlp * 1e-3) / 1e12 / MFMA_BF16_PEAK_TFLOPS,
                     "hbm_bytes_per_query": 12 + 16,
                     "traffic": (None if terrain else
                                 _traffic(os.path.join(ROOT, "paper_2108_10480_amd", "csrc", "mlp.hip"),
                                          "traffic_k_mlp_grad_4M.json", n)),
                     "kernel_ms": ms_mlp},
    }
    tr = res["roofline"]["traffic"]
    if tr is not None:
        gbs = tr / (ms_mlp * 1e-3) / 1e9
        res["roofline"]["hbm_measured"] = {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                           "frac": gbs / HBM_PEAK_GBS}
    keep = keep_local
    if args.sur_oracle and not args.no_cpu_baseline and not terrain:
        from oracle import oracle as O
        rng = np.random.default_rng(321)
        idx = torch.as_tensor(np.sort(rng.choice(n, size=min(args.sur_oracle, n), replace=False)), device="cuda")
        keep_s = keep[idx].cpu().numpy()
        Qs = Xin[idx].cpu().numpy().astype(np.float64)
        trees = [None, None, O.OracleTree(*api.sd_export_bvh(scene, 2))]
        osc = O.OracleScene(sc.V, T=sc.T)
        dr, _, _ = O.barnes_hut(osc, trees, Qs, alpha, beta, cut_f32=True)
        eo = np.abs(d[idx].cpu().numpy() - dr)[keep_s]
        res["vs_oracle_outside_band"] = {"n": int(keep_s.sum()),
                                         "max_abs_err": float(eo.max()) if eo.size else None,
                                         "p99_abs_err": float(np.quantile(eo, 0.99)) if eo.size else None}
    sur.free()
    return res


if __name__ == "__main__":
    main()
