"""Benchmark of the relational retrieval hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload precision]
                    [--form bf16|f32|fp8] [--method proposal|bounded|exhaustive]
                    [--no-cpu-baseline] [--serving] [--latency] [--preds five|all]

One step = one farm_query_topk call over the 4,096-query batch of the
N = 20,000 scene, inputs resident in HBM: query normalisation, similarity GEMM,
TopK candidates, relation terms, composite scores, TopK and the
ScoredCandidate breakdown of the winners.  Default form: BF16 similarity GEMM
with the exact bound-pruned TopK whose candidates are scored over the learned
anchor lists (certified, full-scan fallback).  The scene is built once
(farm_build_memory), and the proposal network is trained on training scenes of
the same generator and its lists built (farm_build_proposals), all outside the
timed region.

Prints ONE JSON line with the throughput (queries/s), batch latency
percentiles, the roofline of the dominant kernel (timed live with the
library's HIP-event phase timer on the launch stream) and the CPU oracle
timed on a bounded sample of the same workload.  --serving instead runs the
request loop over 16 resident scenes and prints p50/p99 latency per rate;
--latency the closed-loop batch-1 latency per scene size.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
# VALU issue peak from the unit counts and clock: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz (one wave64 instruction per SIMD every 4 cycles), in tera lane
# operations per second.  The published FP32 vector figure (157.3 TFLOP/s)
# counts packed FP32 FMAs, which this library's kernels do not use.
PEAK_VALU_TLANE_OPS = 39.3216  # = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic floating-point operations of one (target, anchor) evaluation,
# counted on the definition (offsets, squares/products, scaling by 1/tau or
# 1/(2 sigma^2), exp, 1 + e, reciprocal, times the anchor similarity, max);
# a transcendental counts as one operation.
FLOP_PER_PAIR = {0: 12, 1: 7, 2: 7, 3: 11, 4: 11, 5: 12, 6: 11, 7: 11, 8: 12}
# Closest/Farthest (9, 10) have no fixed cost per pair (a count over the query's
# candidate set): their relations are left out of the ALU counts below.


def pred_pool(args):
    """Predicate ids the benchmark's queries draw from (None: the generator's default five)."""
    from synth import ALL_PREDS, EVERY_PRED
    return {"five": None, "all": ALL_PREDS, "every": EVERY_PRED}[args.preds]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter record, or
    None when there is none for this workload or the kernel's source file has
    changed since the counters were taken (sha256 prefix mismatch)."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("workload") != workload:
        return None
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["sha256_prefix"]:
        return None
    return float(rec["bytes_per_launch"])


def recorded_valu(kernel: str, workload: str):
    """VALU instruction counts of `kernel` from the committed counter record
    (profiles/valu.json), or None when there is none for this workload or the
    kernel's source file has changed since the counters were taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "valu.json")))["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("workload") != workload:
        return None
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec["sha256_prefix"]:
        return None
    return rec


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="precision")
    p.add_argument("--form", default="bf16", choices=["f32", "bf16", "fp8"])
    p.add_argument("--rescore-mult", type=int, default=4)
    p.add_argument("--method", default="proposal", choices=["exhaustive", "bounded", "proposal"])
    p.add_argument("--train-scenes", type=int, default=32,
                   help="training scenes of the proposal network (seeds 1000.., held out from the benchmark scene)")
    p.add_argument("--train-steps", type=int, default=600)
    p.add_argument("--list-m", type=int, default=256, help="anchors per (object, predicate) list")
    p.add_argument("--k", type=int, default=10)
    p.add_argument("--preds", default="five", choices=["five", "all", "every"],
                   help="predicates the queries draw from: the workload's five (Near..RightOf), all nine pairwise "
                        "ones (+ NextTo, InFrontOf, Behind, On) or every one (+ Closest, Farthest, Inside)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-value-lists", dest="value_lists", action="store_false",
                   help="skip the non-learned baseline (lists ranked by exact predicate value)")
    p.add_argument("--latency-queries", type=int, default=256, help="batch-1 requests timed for latency_ms")
    p.add_argument("--cpu-sample", type=int, default=0, help="queries in the CPU-oracle sample (0 = auto)")
    p.add_argument("--serving", action="store_true",
                   help="run the request loop over 16 resident scenes instead (p50/p99 latency per arrival rate)")
    p.add_argument("--rates", default="500,2000,5000", help="Poisson arrival rates (requests/s) of --serving")
    p.add_argument("--requests", type=int, default=3000, help="requests per rate of --serving")
    p.add_argument("--latency", action="store_true",
                   help="closed-loop batch-1 latency per scene size instead (one query at a time, p50/p99)")
    p.add_argument("--unary", default="cosine", choices=["cosine", "rrf"],
                   help="unary scores: the clamped cosine (default) or reciprocal-rank fusion over four query "
                        "channels in three embedding spaces (FP32 cosines; its own JSON line)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                   help="only run one plain device copy of BYTES (reference for the HBM byte counters) and exit")
    return p.parse_args(argv)


def copy_calibration(nbytes):
    """One device-to-device copy kernel of a known size: the byte counters of a
    profiler pass over it give the factor between counter units and bytes."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": n * 4, "bytes_written": n * 4}}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the layout over several GPUs is "
              "described, not implemented.", file=sys.stderr)
        sys.exit(2)
    if args.serving:
        serving(args)
        return
    if args.latency:
        latency(args)
        return
    if args.unary == "rrf":
        rrf_bench(args)
        return
    import torch

    import paper_2606_15476_amd as farm
    from synth import ALL_PREDS, CONFIGS, make_queries, make_scene

    cfg = CONFIGS[args.workload]
    t0 = time.time()
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene, preds=pred_pool(args))
    log(f"[bench] generated {cfg.name}: n={scene.n} d={scene.d} q={qb.q} R={qb.r_tot} in {time.time() - t0:.1f}s")

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mem = farm.Memory(t(scene.desc), t(scene.center), t(scene.extent), t(scene.ids.view(np.int32)), t(scene.cls),
                      scene.view_right, flags=farm.FARM_BUILD_BF16 | farm.FARM_BUILD_FP8)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    target, anchors = t(qb.target), t(qb.rel_anchor)
    k = args.k
    oid = torch.empty((qb.q, k), dtype=torch.int32, device=dev)
    osc = torch.empty((qb.q, k), dtype=torch.float32, device=dev)
    ot = torch.empty((qb.q, k, 8), dtype=torch.float32, device=dev)
    ob = torch.empty((qb.q, k, 8), dtype=torch.int32, device=dev)
    dtype = {"f32": farm.F32, "bf16": farm.BF16, "fp8": farm.FP8_E4M3}[args.form]
    method = {"exhaustive": farm.EXHAUSTIVE, "bounded": farm.BOUNDED, "proposal": farm.PROPOSAL}[args.method]
    cert = torch.zeros((qb.q,), dtype=torch.int32, device=dev)
    proposal_info = None
    if method == farm.PROPOSAL:
        proposal_info = prepare_proposals(farm, cfg, mem, args)

    def step():
        farm.query_topk(mem, ws, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors, k, oid, osc, ot, ob,
                        dtype=dtype, rescore_mult=args.rescore_mult, certified=cert, method=method)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    ws.status()
    ws.set_timing(True)
    ws.timings(reset=True)
    ws.proposal_stats(reset=True)
    torch.cuda.synchronize()
    times = []
    t_start = time.perf_counter()
    for s in range(args.steps):
        a = time.perf_counter()
        step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
        log(f"[bench] step {s + 1}/{args.steps}: {times[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    phases = ws.timings(reset=True)
    ws.set_timing(False)
    ws.status()
    if method == farm.BOUNDED:
        # full anchor scans of every candidate term: their count and FP32 dot products
        checked, _, _, fb_dots = ws.proposal_stats(reset=True)
        proposal_info = {"full_scan_terms_per_step": checked // max(args.steps, 1),
                         "full_scan_fp32_dots_per_step": fb_dots // max(args.steps, 1)}
    if method == farm.PROPOSAL:
        checked, fell, dots, fb_dots = ws.proposal_stats(reset=True)
        proposal_info["terms_per_step"] = checked // max(args.steps, 1)
        proposal_info["fallback_rate"] = round(fell / max(checked, 1), 5)
        proposal_info["fp32_dots_per_step"] = dots // max(args.steps, 1)
        proposal_info["fallback_fp32_dots_per_step"] = fb_dots // max(args.steps, 1)
        log(f"[bench] proposal terms {checked}, fell back {fell}")

    certified = int((cert.cpu().numpy() == 1).sum())
    recall_exact = None
    if dtype != farm.F32 or method != farm.EXHAUSTIVE:
        # Recall@K of this form against the exact FP32 path over the whole batch
        xid = torch.empty_like(oid)
        xsc = torch.empty_like(osc)
        farm.query_topk(mem, ws, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors, k, xid, xsc)
        torch.cuda.synchronize()
        a, b = oid.cpu().numpy(), xid.cpu().numpy()
        recall_exact = float(np.mean([len(set(a[i]) & set(b[i])) / k for i in range(qb.q)]))
        log(f"[bench] recall@{k} vs exact FP32 path: {recall_exact:.5f}; certified {certified}/{qb.q}")

    qps = qb.q * args.steps / elapsed
    ms_step = elapsed / args.steps * 1e3
    roofline = dominant_roofline(phases, scene, qb, args, cfg, proposal_info)
    phase_ms = {p: round(v[0] / max(v[1], 1), 3) for p, v in phases.items() if v[1]}

    # per-request latency: closed-loop batch-1 calls of the same form on the same scene
    req_lat = request_latency(farm, mem, qb, target, anchors, k, dtype, method, args) if args.latency_queries else None

    cpu = None
    recall = None
    errors = None
    if not args.no_cpu_baseline:
        cpu, recall, sample_rows, s64 = cpu_baseline(scene, qb, oid, osc, k, args.cpu_sample)
        errors = dtype_errors(farm, mem, ws, scene, qb, sample_rows, s64, k, method)

    baseline_lists = None
    if method == farm.PROPOSAL and args.value_lists:
        baseline_lists = value_list_baseline(farm, mem, ws, step, args)

    lat = np.asarray(times) * 1e3
    out = {
        "metric": "queries/s at N=20k objects, K=10",
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16 GEMM, f32 relational pass and rescoring",
                  "fp8": "fp8-e4m3 GEMM, f32 relational pass and rescoring"}[args.form],
        "data": "synthetic (seeded scene generator; the paper's datasets are not used)",
        "config": {"workload": f"{cfg.name}: N={scene.n} objects, D={scene.d}, Q={qb.q} queries, "
                               f"R~U{{{cfg.r_min}..{cfg.r_max}}} (R_tot={qb.r_tot}), K={k}",
                   "form": args.form, "method": args.method, "global_batch": qb.q, "parallelism": "none (1 GPU)",
                   "predicates": {"five": "Near, Above, Below, LeftOf, RightOf", "all": "all nine pairwise",
                                  "every": "all twelve (pairwise + Closest, Farthest, Inside)"}[args.preds]},
        "latency_ms": req_lat,
        "batch_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                             "p99": round(float(np.percentile(lat, 99)), 3), "what": "one step (the whole batch)"},
        "phase_ms": phase_ms,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "recall_at_10_vs_oracle": recall,
        "score_error_vs_oracle": errors,
        "recall_at_10_vs_exact_f32": recall_exact,
        "certified_queries": certified,
        "form": form_name(args),
        ("bounded" if method == farm.BOUNDED else "proposal"): proposal_info,
        "value_lists_baseline": baseline_lists,
    }
    print(json.dumps(out), flush=True)


def serving(args):
    """Poisson arrivals over 16 resident scenes (N log-uniform in [500, 20000],
    the precision generator, seeds 3000-3015; arrivals seed 3100), uniform scene
    choice, R ~ U{1..4}; each rate is served by the plain FP32 exhaustive form,
    the BF16 bound-pruned form and (with a trained network) the BF16
    learned-proposal form, each server warmed up untimed first (one request per
    scene, served to completion: first launches and workspace set-up).  Latency =
    completion seen by the host minus the scheduled arrival time."""
    import torch

    import paper_2606_15476_amd as farm
    from synth import ALL_PREDS, CONFIGS, make_queries, make_scene
    cfg = CONFIGS["precision"]
    rng = np.random.default_rng(3100)
    sizes = np.exp(rng.uniform(np.log(500), np.log(20000), 16)).astype(int)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    scenes, pools = [], []
    for i, n in enumerate(sizes):
        sc = make_scene(cfg, seed=3000 + i, n=int(n))
        qb = make_queries(cfg, sc, seed=3000 + i, q=64)
        mem = farm.Memory(t(sc.desc), t(sc.center), t(sc.extent), t(sc.ids.view(np.int32)), t(sc.cls), sc.view_right,
                          flags=farm.FARM_BUILD_BF16)
        scenes.append(mem)
        d = sc.d
        pools.append([(qb.target[q], int(qb.target_cls[q]), qb.rel_pred[qb.rel_off[q]:qb.rel_off[q + 1]],
                       qb.rel_anchor.reshape(-1, d)[qb.rel_off[q]:qb.rel_off[q + 1]]) for q in range(qb.q)])
    log(f"[serve] 16 scenes, N = {sorted(int(x) for x in sizes)}")
    forms = {"f32-exhaustive": (farm.F32, farm.EXHAUSTIVE), "bf16-bounded": (farm.BF16, farm.BOUNDED)}
    if args.train_scenes > 0:
        # the learned-proposal form: one network trained on training scenes of the generator, lists per scene
        net = train_network(farm, cfg, args)
        for m in scenes:
            farm.build_proposals(m, net, args.list_m)
        torch.cuda.synchronize()
        forms["bf16-proposal"] = (farm.BF16, farm.PROPOSAL)
    results = []
    for rate in [float(x) for x in args.rates.split(",")]:
        gaps = rng.exponential(1.0 / rate, args.requests)
        arrivals = np.cumsum(gaps)
        picks = [(int(rng.integers(16)), int(rng.integers(64))) for _ in range(args.requests)]
        for name, (dt, me) in forms.items():
            sv = farm.Server(slots=4, max_batch_q=64, max_batch_rel=256, k=10, dtype=dt, method=me,
                             hbm_budget=16 << 30)
            for m in scenes:
                sv.add_scene(m)
            # untimed warm-up: one request per scene, served to completion
            pending = {sv.submit(si, *pools[si][0]) for si in range(len(scenes))}
            while pending:
                sv.progress()
                for rid, *_ in sv.poll():
                    pending.discard(rid)
            lat = {}
            late = {}
            t0 = time.perf_counter()
            i = 0
            while len(lat) < args.requests:
                now = time.perf_counter() - t0
                while i < args.requests and arrivals[i] <= now:
                    s, q = picks[i]
                    rid = sv.submit(s, *pools[s][q])
                    late[rid] = (time.perf_counter() - t0) - arrivals[i]
                    i += 1
                sv.progress()
                for rid, st, ce, ns, _, _ in sv.poll():
                    lat[rid] = ns / 1e9 + late[rid]
            wall = time.perf_counter() - t0
            v = np.asarray(list(lat.values())) * 1e3
            st = sv.stats()
            sv.close()
            row = {"rate": rate, "form": name, "p50_ms": round(float(np.percentile(v, 50)), 3),
                   "p99_ms": round(float(np.percentile(v, 99)), 3), "served_per_s": round(args.requests / wall, 1),
                   "batches": int(st["batches"]), "deferrals": int(st["deferrals"])}
            log(f"[serve] {row}")
            results.append(row)
    print(json.dumps({"metric": "serving latency over 16 resident scenes", "unit": "ms", "n_gpus": 1,
                      "config": {"workload": "16 scenes, N log-uniform [500, 20000], D=1152, R~U{1..4}, K=10, "
                                             "Poisson arrivals", "slots": 4, "max_batch_q": 64,
                                 "requests_per_rate": args.requests, "scene_sizes": sorted(int(x) for x in sizes)},
                      "results": results}), flush=True)


def latency(args):
    """Closed-loop batch-1 latency: one query at a time (submit, wait for the
    result, next) on precision-generator scenes of N = 1k, 5k and 20k objects,
    for the plain FP32 exhaustive form and the BF16 learned-proposal form;
    latency = host wall time of one farm_query_topk call plus its
    synchronisation.  256 queries per scene after 16 untimed ones."""
    import torch

    import paper_2606_15476_amd as farm
    from synth import ALL_PREDS, CONFIGS, make_queries, make_scene
    cfg = CONFIGS["precision"]
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    net = train_network(farm, cfg, args) if args.train_scenes > 0 else None
    results = []
    for n in (1000, 5000, 20000):
        sc = make_scene(cfg, seed=4000 + n, n=n)
        qb = make_queries(cfg, sc, seed=4100 + n, q=272)
        mem = farm.Memory(t(sc.desc), t(sc.center), t(sc.extent), t(sc.ids.view(np.int32)), t(sc.cls), sc.view_right,
                          flags=farm.FARM_BUILD_BF16)
        forms = {"f32-exhaustive": (farm.F32, farm.EXHAUSTIVE)}
        if net is not None:
            farm.build_proposals(mem, net, args.list_m)
            forms["bf16-proposal"] = (farm.BF16, farm.PROPOSAL)
        ws = farm.Workspace(mem, 1, farm.FARM_MAX_REL, 64)
        d = sc.d
        queries = []
        for q in range(qb.q):
            r0, r1 = int(qb.rel_off[q]), int(qb.rel_off[q + 1])
            queries.append((t(qb.target[q:q + 1]), qb.target_cls[q:q + 1], np.array([0, r1 - r0], np.int32),
                            qb.rel_pred[r0:r1], t(qb.rel_anchor.reshape(-1, d)[r0:r1])))
        oid = torch.empty((1, args.k), dtype=torch.int32, device=dev)
        osc = torch.empty((1, args.k), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        for name, (dt, me) in forms.items():
            lat = []
            for i, (tg, tc, ro, rp, an) in enumerate(queries):
                a = time.perf_counter()
                farm.query_topk(mem, ws, tg, tc, ro, rp, an, args.k, oid, osc, dtype=dt, method=me)
                torch.cuda.synchronize()
                if i >= 16:
                    lat.append(time.perf_counter() - a)
            v = np.asarray(lat) * 1e3
            row = {"n": n, "form": name, "p50_ms": round(float(np.percentile(v, 50)), 3),
                   "p99_ms": round(float(np.percentile(v, 99)), 3), "queries": len(lat)}
            log(f"[latency] {row}")
            results.append(row)
    print(json.dumps({"metric": "closed-loop batch-1 query latency", "unit": "ms", "n_gpus": 1,
                      "config": {"workload": "precision generator, N in {1000, 5000, 20000}, D=1152, R~U{1..4}, "
                                             "K=10, one query per call"},
                      "results": results}), flush=True)


def train_network(farm, cfg, args):
    """The proposal network trained on exhaustive bindings of training scenes of
    the generator (seeds 1000, 1001, ...)."""
    import torch
    from paper_2606_15476_amd import proposal
    from synth import ALL_PREDS, make_queries, make_scene
    t0 = time.time()
    data, keep = [], []
    for i in range(args.train_scenes):
        seed = 1000 + i
        sc = make_scene(cfg, seed=seed)
        qt = make_queries(cfg, sc, seed=seed, q=256, preds=pred_pool(args))
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
        m = farm.Memory(t(sc.desc), t(sc.center), t(sc.extent), t(sc.ids.view(np.int32)), t(sc.cls), sc.view_right)
        w = farm.Workspace(m, qt.q, qt.r_tot, 16)
        bind = proposal.exhaustive_bindings(m, w, t(qt.target), qt.target_cls, qt.rel_off, qt.rel_pred,
                                            t(qt.rel_anchor))
        o, a, p, y = proposal.sample_pairs(bind, sc.ids, qt.rel_pred, np.random.default_rng(seed), per_relation=96)
        data.append((m, o, a, p, y))
        keep.append(w)
        log(f"[bench] training scene {seed}: {o.size} examples")
    t_data = time.time() - t0
    net = farm.ProposalNet(cfg.d, max_batch=4096, seed=7)
    t1 = time.time()
    hist = proposal.train(net, data, steps=args.train_steps, batch=4096, lr=2e-3, weight_decay=1e-4)
    t_train = time.time() - t1
    log(f"[bench] trained {args.train_steps} steps in {t_train:.1f}s: loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
    net.history, net.label_s, net.train_s = hist, t_data, t_train
    return net


def prepare_proposals(farm, cfg, mem, args):
    """Train the proposal network, then build the lists of the benchmark scene.
    Outside the timed region, like farm_build_memory."""
    import torch
    net = train_network(farm, cfg, args)
    hist = net.history
    t2 = time.time()
    farm.build_proposals(mem, net, args.list_m)
    torch.cuda.synchronize()
    t_build = time.time() - t2
    log(f"[bench] proposal lists (M={args.list_m}) built in {t_build:.2f}s")
    dtype = {"f32": farm.F32, "bf16": farm.BF16, "fp8": farm.FP8_E4M3}[args.form]
    return {"pass_in_lds": mem.proposal_pass_in_lds(dtype),
            "train_scenes": args.train_scenes, "train_steps": args.train_steps, "loss_first": round(hist[0][1], 5),
            "loss_last": round(hist[-1][1], 5), "label_s": round(net.label_s, 2), "train_s": round(net.train_s, 2),
            "table_build_s": round(t_build, 3), "list_m": args.list_m}


def dominant_roofline(phases, scene, qb, args, cfg, proposal_info):
    """Roofline of the kernel behind the phase with the largest time."""
    n, q, R = scene.n, qb.q, qb.r_tot
    timed = {p: v for p, v in phases.items() if v[1]}
    dominant = max(timed, key=lambda p: timed[p][0])
    ms, launches = timed[dominant]
    avg_s = ms / launches / 1e3
    if dominant == "pair":
        # ALU: the FP32 arithmetic VALU instructions (add, mul, FMA, transcendental) per
        # (relation, target, anchor) pair from the committed counter record, times the
        # launch's pairs, against the VALU issue peak; the fraction of all VALU
        # instructions (moves, selects, compares included) is reported beside it
        pairs = float(R) * n * (n - 1)
        rec = recorded_valu("k_pair_exhaustive", cfg.name)
        # beside it, the pass's algorithmic HBM bytes: every similarity row once (4 B per object
        # and query or relation row) and the boxes (24 B per object) per query
        nbytes = 4.0 * (q + R) * n + 24.0 * q * n
        out = {"bound": "alu", "kernel": "k_pair_exhaustive", "achieved": None, "peak": PEAK_VALU_TLANE_OPS,
               "unit": "T FP32 VALU lane-ops/s", "frac": None, "traffic": recorded_traffic("k_pair_exhaustive", cfg.name),
               "pair_evals_per_launch": pairs, "avg_launch_ms": round(avg_s * 1e3, 3),
               "algorithmic_gbs": round(nbytes / avg_s / 1e9, 2),
               "hbm_frac": round(nbytes / avg_s / 1e9 / PEAK_HBM_GBS, 6)}
        if rec:
            arith = rec["fp32_arith_insts"] * 64.0 / rec["pair_evals"]
            every = rec["sq_insts_valu"] * 64.0 / rec["pair_evals"]
            achieved = arith * pairs / avg_s / 1e12
            out.update(achieved=round(achieved, 3), frac=round(achieved / PEAK_VALU_TLANE_OPS, 4),
                       fp32_arith_lane_ops_per_pair=round(arith, 3), valu_lane_instr_per_pair=round(every, 3),
                       valu_issue_frac=round(every * pairs / avg_s / 1e12 / PEAK_VALU_TLANE_OPS, 4),
                       counts_from="profiles/valu.json (rocprofv3 SQ_INSTS_VALU and its classes)")
        return out
    if dominant == "gemm":
        flop = 2.0 * (q + R) * n * scene.d
        achieved = flop / avg_s / 1e12
        peak = PEAK_MFMA_TFLOPS[args.form]
        return {"bound": "mfma", "kernel": "k_sim_gemm<" + args.form + ">", "achieved": round(achieved, 2),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "traffic": recorded_traffic("k_sim_gemm_" + args.form, cfg.name), "avg_launch_ms": round(avg_s * 1e3, 3)}
    if dominant == "topk":
        # the candidate scan reads each target similarity row once (4 B per object and query)
        kernel = "k_bound_candidates" if args.method in ("bounded", "proposal") else "k_topk_rows"
        nbytes = 4.0 * q * n
        achieved = nbytes / avg_s / 1e9
        return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": recorded_traffic(kernel, cfg.name), "avg_launch_ms": round(avg_s * 1e3, 3)}
    if dominant == "propose":
        # semantic sets: each relation similarity row read once (4 B per anchor)
        nbytes = 4.0 * R * n
        achieved = nbytes / avg_s / 1e9
        return {"bound": "hbm", "kernel": "k_semantic_sets", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": recorded_traffic("k_semantic_sets", cfg.name), "avg_launch_ms": round(avg_s * 1e3, 3)}
    info = proposal_info or {}
    terms, m, dots = info.get("terms_per_step", 0), info.get("list_m", 0), info.get("fp32_dots_per_step", 0)
    if dominant == "rescore" and args.method == "proposal" and info:
        in_lds = bool(info.get("pass_in_lds"))
        kernel = "k_rescore_subset_lds" if in_lds else "k_rescore_terms<subset>"
        # proposal pass, algorithmic bytes: each relation's similarity row once (4 B per
        # object) and, per evaluated term, its list (4 B anchor index + 4 B cached predicate
        # value per entry; + a 4 B similarity gather when the row is not staged in LDS).
        # The FP32 dot products of unresolved anchors read descriptor rows (4 B x D each)
        # that are re-read across terms from the caches: reported beside, not counted.
        nbytes = 4.0 * R * n + float(terms) * m * (8.0 if in_lds else 12.0)
        dot_bytes = float(dots) * 4.0 * scene.d
        achieved = nbytes / avg_s / 1e9
        return {"bound": "hbm", "kernel": kernel, "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": recorded_traffic(kernel, cfg.name), "avg_launch_ms": round(avg_s * 1e3, 3),
                "algorithmic_bytes_per_launch": nbytes,
                "bytes_detail": {"relation_rows": 4.0 * R * n, "list_entries": float(terms) * m * 8.0,
                                 "terms": int(terms), "list_m": int(m),
                                 "fp32_dot_descriptor_bytes_not_counted": dot_bytes, "fp32_dots": int(dots)}}
    # full anchor scans of candidate terms (the fallback of the proposal method, or every
    # candidate term of the bound-pruned method): pair evaluations on the ALU
    pairwise = [FLOP_PER_PAIR[int(p)] for p in qb.rel_pred if int(p) in FLOP_PER_PAIR]
    per_pair = float(np.mean(pairwise)) if pairwise else 0.0
    if dominant == "fallback":
        n_terms, kernel = float(info.get("fallback_rate", 0.0) * terms), "k_rescore_fallback"
    else:
        n_terms, kernel = float(info.get("full_scan_terms_per_step", 0)), "k_rescore_terms<full>"
    ops = n_terms * n * per_pair
    achieved = ops / avg_s / 1e12
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3),
            "peak": PEAK_VALU_TLANE_OPS, "unit": "T lane-ops/s (operations counted on the definition)",
            "frac": round(achieved / PEAK_VALU_TLANE_OPS, 4), "traffic": None, "avg_launch_ms": round(avg_s * 1e3, 3),
            "pair_evals_per_launch": n_terms * n}


def request_latency(farm, mem, qb, target, anchors, k, dtype, method, args):
    """Per-request latency: one query per farm_query_topk call, the next after
    the previous result (host wall time of the call plus its synchronisation),
    on the benchmark's scene and form; p50/p99 over args.latency_queries
    requests after 16 untimed ones."""
    import torch
    ws1 = farm.Workspace(mem, 1, farm.FARM_MAX_REL, 64)
    oid = torch.empty((1, k), dtype=torch.int32, device=target.device)
    osc = torch.empty((1, k), dtype=torch.float32, device=target.device)
    lat = []
    nq = min(qb.q, args.latency_queries + 16)
    for i in range(nq):
        r0, r1 = int(qb.rel_off[i]), int(qb.rel_off[i + 1])
        ro = np.array([0, r1 - r0], np.int32)
        a = time.perf_counter()
        farm.query_topk(mem, ws1, target[i:i + 1], qb.target_cls[i:i + 1], ro, qb.rel_pred[r0:r1], anchors[r0:r1], k,
                        oid, osc, dtype=dtype, method=method)
        torch.cuda.synchronize()
        if i >= 16:
            lat.append(time.perf_counter() - a)
    v = np.asarray(lat) * 1e3
    del ws1
    return {"p50": round(float(np.percentile(v, 50)), 4), "p99": round(float(np.percentile(v, 99)), 4),
            "requests": len(lat), "what": "per request: closed-loop batch-1 farm_query_topk calls on the benchmark "
                                          "scene (host wall time incl. synchronisation)"}


def dtype_errors(farm, mem, ws, scene, qb, rows, s64, k, method):
    """Per similarity dtype, on the CPU sample's queries against the FP64
    oracle: the similarity GEMM's own s_sem (before any FP32 rescoring: max and
    RMS absolute error over all sample rows x N objects), and the returned TopK
    scores (max and median relative error, Recall@K of the ids)."""
    import oracle
    import torch
    from synth import QueryBatch
    sub = qb.subset(rows)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    target, anchors = t(sub.target), t(sub.rel_anchor)
    idx_of = {int(v): i for i, v in enumerate(scene.ids)}
    sem = QueryBatch(sub.target, sub.target_cls, np.zeros(sub.q + 1, np.int32), np.zeros(0, np.int32),
                     np.zeros((0, sub.target.shape[1]), np.float32), sub.planted)
    sem64 = oracle.score(scene, sem)  # no relations: the score is s_sem
    sim = torch.empty((sub.q, scene.n), dtype=torch.float32, device=dev)
    out = {}
    for name, dt in (("f32", farm.F32), ("bf16", farm.BF16), ("fp8", farm.FP8_E4M3)):
        oid = torch.empty((sub.q, k), dtype=torch.int32, device=dev)
        osc = torch.empty((sub.q, k), dtype=torch.float32, device=dev)
        farm.query_topk(mem, ws, target, sub.target_cls, sub.rel_off, sub.rel_pred, anchors, k, oid, osc, dtype=dt,
                        method=method)
        torch.cuda.synchronize()
        ids, sc = oid.cpu().numpy().view(np.uint32), osc.cpu().numpy().astype(np.float64)
        rel, hits = [], []
        for i in range(sub.q):
            want = set(int(x) for x in scene.ids[oracle.topk(s64[i], scene.ids, k)])
            hits.append(len(want & set(int(x) for x in ids[i])) / k)
            for g, v in zip(ids[i], sc[i]):
                ref = s64[i, idx_of[int(g)]]
                rel.append(abs(v - ref) / max(abs(ref), 1e-30))
        farm.similarity(mem, ws, target, sub.target_cls, sim, dtype=dt)
        torch.cuda.synchronize()
        e = sim.cpu().numpy().astype(np.float64) - sem64
        out[name] = {"gemm_sim_max_abs_err": float(np.max(np.abs(e))),
                     "gemm_sim_rms_err": float(np.sqrt(np.mean(e * e))),
                     "max_rel_err": float(np.max(rel)), "median_rel_err": float(np.median(rel)),
                     "recall_at_k_vs_oracle": float(np.mean(hits)), "queries": int(sub.q)}
        log(f"[bench] {name}: GEMM s_sem vs FP64 oracle max abs err {out[name]['gemm_sim_max_abs_err']:.2e}; "
            f"returned scores max rel err {out[name]['max_rel_err']:.2e}, "
            f"recall {out[name]['recall_at_k_vs_oracle']:.4f}")
    return out


def value_list_baseline(farm, mem, ws, step, args):
    """The same form with non-learned lists: per (object, predicate) the M
    anchors of largest exact predicate value (farm_build_proposals_by_value).
    Replaces the memory's lists; measured after every other leg."""
    import torch
    t0 = time.time()
    farm.build_proposals_by_value(mem, args.list_m)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    for _ in range(2):
        step()
    torch.cuda.synchronize()
    ws.proposal_stats(reset=True)
    a = time.perf_counter()
    steps = max(3, args.steps // 2)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - a) / steps * 1e3
    checked, fell, dots, fb_dots = ws.proposal_stats(reset=True)
    res = {"ms_per_step": round(ms, 3), "queries_per_s": None, "fallback_rate": round(fell / max(checked, 1), 5),
           "fp32_dots_per_step": dots // steps, "list_build_s": round(build_s, 3), "steps": steps,
           "what": "lists of the M anchors of largest exact predicate value (no network), same certificate"}
    log(f"[bench] value-ranked lists: {ms:.3f} ms/step, fallback rate {res['fallback_rate']}")
    return res


def form_name(args):
    gemm = {"f32": "FP32", "bf16": "BF16", "fp8": "FP8-e4m3"}[args.form] + " similarity GEMM"
    if args.method == "bounded":
        return (gemm + " + exact bound-pruned TopK (objects whose s_sem bound can reach the K-th lower bound "
                "scored in FP32 over every anchor)")
    if args.method == "proposal":
        return (gemm + f" + exact bound-pruned TopK whose candidates are scored over learned anchor lists "
                f"(M={args.list_m}) and semantic anchor sets, certified, with full-scan fallback")
    if args.form == "f32":
        return "exhaustive FP32 (plain method: every object over every anchor)"
    return gemm + f" + exhaustive estimate/upper-bound pass + FP32 rescoring of the top {args.rescore_mult}K"


def rrf_bench(args):
    """The method with reciprocal-rank-fusion unary scores on the workload's scene and queries: four
    query channels over three embedding spaces with the weights 1.0 / 0.5 / 0.75 / 1.0 (a 1,024-wide
    text space queried with the target description and with a noisier stand-in for the raw
    utterance, the descriptor table, a 2,048-wide image space), FP32 cosines, exact ranks."""
    import torch

    import paper_2606_15476_amd as farm
    import synth
    from synth import CONFIGS, make_queries, make_scene

    cfg = CONFIGS[args.workload]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene, preds=pred_pool(args))
    spaces, tv, av = synth.add_embedding_spaces(cfg, scene, qb, dims=(1024, 2048), seed=7)
    rng = np.random.default_rng(8)
    utt_t = tv[0] + rng.standard_normal(tv[0].shape).astype(np.float32) * 0.01
    utt_a = av[0] + rng.standard_normal(av[0].shape).astype(np.float32) * 0.01
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    mem = farm.Memory(t(scene.desc), t(scene.center), t(scene.extent), t(scene.ids.view(np.int32)), t(scene.cls),
                      scene.view_right)
    s_text = mem.add_embedding_space(t(spaces[0]))
    s_img = mem.add_embedding_space(t(spaces[1]))
    host_ch = [(s_text, 1.0, tv[0], av[0]), (s_text, 0.5, utt_t, utt_a), (0, 0.75, qb.target, qb.rel_anchor),
               (s_img, 1.0, tv[1], av[1])]
    ch = [(sp, w, t(a), t(b)) for sp, w, a, b in host_ch]
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    k = args.k
    method = {"exhaustive": farm.EXHAUSTIVE, "bounded": farm.BOUNDED, "proposal": farm.PROPOSAL}[args.method]
    if method == farm.PROPOSAL:
        prepare_proposals(farm, cfg, mem, args)
    oid = torch.empty((qb.q, k), dtype=torch.int32, device=dev)
    osc = torch.empty((qb.q, k), dtype=torch.float32, device=dev)
    cert = torch.zeros((qb.q,), dtype=torch.int32, device=dev)

    def step():
        farm.query_topk_rrf(mem, ws, ch, qb.target_cls, qb.rel_off, qb.rel_pred, k, oid, osc, certified=cert,
                            method=method)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ws.set_timing(True)
    ws.timings(reset=True)
    a = time.perf_counter()
    for sidx in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"[bench] rrf step {sidx + 1}/{args.steps}")
    elapsed = time.perf_counter() - a
    phases = ws.timings(reset=True)
    ws.set_timing(False)
    ws.status()
    phase_ms = {p: round(v[0] / max(v[1], 1), 3) for p, v in phases.items() if v[1]}
    rows = qb.q + qb.r_tot
    dims = [spaces[0].shape[1], spaces[0].shape[1], scene.d, spaces[1].shape[1]]
    flops = sum(2.0 * rows * scene.n * d for d in dims)
    fuse_s = phases["gemm"][0] / max(phases["gemm"][1], 1) / 1e3
    roof = {"bound": "mfma", "kernel": "k_sim_gemm<f32> per channel + k_rrf_rank (the fusion phase)",
            "achieved": round(flops / fuse_s / 1e12, 1), "peak": 157.3, "unit": "TFLOP/s",
            "frac": round(flops / fuse_s / 1e12 / 157.3, 4), "traffic": None,
            "avg_launch_ms": round(fuse_s * 1e3, 3),
            "what": "FP32 cosine FLOPs of the four channels over the whole fusion phase (GEMMs and ranking)"}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import rrf
        m = args.cpu_sample or 8
        sub = qb.subset(range(m))
        r1 = int(qb.rel_off[m])
        a = time.perf_counter()
        sem, asim = rrf.similarities(scene, [scene.desc] + spaces,
                                     [(sp, w, x[:m]) for sp, w, x, _ in host_ch],
                                     [(sp, w, y[:r1]) for sp, w, _, y in host_ch], sub.target_cls)
        # the oracle's spaces list is [descriptors, text, image]: the space indices match the memory's
        with oracle.similarities(sem, asim):
            s64 = oracle.score(scene, sub)
        order = [oracle.topk(s64[i], scene.ids, k) for i in range(m)]
        secs = time.perf_counter() - a
        got = oid[:m].cpu().numpy().view(np.uint32)
        hits = np.mean([len(set(map(int, got[i])) & set(map(int, scene.ids[order[i]]))) / k for i in range(m)])
        cpu = {"value": round(m / secs, 4), "unit": "queries/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": f"first {m} queries: exact FP64 ranks of the four channels over all {scene.n} objects, "
                         "fused rows, exhaustive scoring + TopK", "seconds": round(secs, 2),
               "recall_at_k_vs_oracle": float(hits)}
        log(f"[bench] rrf cpu baseline {secs:.1f}s, recall@{k} on the sample {hits:.4f}")
    qps = qb.q * args.steps / elapsed
    print(json.dumps({
        "metric": "queries/s at N=20k objects, K=10 (reciprocal-rank-fusion unary scores)", "value": round(qps, 2),
        "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 cosines, exact ranks, f32 relational pass",
        "data": "synthetic (seeded scene generator and embedding spaces)",
        "config": {"workload": f"{cfg.name}: N={scene.n}, Q={qb.q}, R_tot={qb.r_tot}, K={k}; four channels "
                               f"(weights 1.0/0.5/0.75/1.0) over spaces of width 1024, {scene.d}, 2048",
                   "method": args.method, "parallelism": "none (1 GPU)"},
        "phase_ms": phase_ms, "certified_queries": int((cert.cpu().numpy() == 1).sum()), "roofline": roof,
        "cpu_baseline": cpu}), flush=True)


def cpu_baseline(scene, qb, oid, osc, k, sample):
    """Time the FP64 oracle (plain exhaustive scoring + TopK) on a sample of
    the batch, with every host thread (the oracle parallelises over the objects
    of a query), and one query with a single thread."""
    import oracle
    oracle._load()
    threads = oracle.threads()
    m = sample or 16
    rows = list(range(m))
    sub = qb.subset(rows)
    log(f"[bench] cpu baseline: oracle on {m} queries, {threads} threads")
    a = time.perf_counter()
    s64 = oracle.score(scene, sub)
    order = [oracle.topk(s64[i], scene.ids, k) for i in range(m)]
    secs = time.perf_counter() - a
    ids = oid[:m].cpu().numpy().view(np.uint32)
    hits = [len(set(int(x) for x in ids[i]) & set(int(x) for x in scene.ids[order[i]])) / k for i in range(m)]
    log(f"[bench] cpu baseline: {secs:.1f}s, recall@{k} on the sample {np.mean(hits):.4f}")
    oracle.set_threads(1)
    a = time.perf_counter()
    oracle.score(scene, qb.subset(range(1)))
    secs1 = time.perf_counter() - a
    oracle.set_threads(threads)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    log(f"[bench] cpu baseline, one thread: {secs1:.1f}s for one query")
    return ({"value": round(m / secs, 4), "unit": "queries/s", "cores": threads, "kind": "oracle",
             "sample": f"first {m} queries of the batch, full exhaustive FP64 scoring of all {scene.n} objects + TopK",
             "seconds": round(secs, 2), "one_thread_seconds_per_query": round(secs1, 2), "cpu": model,
             "nproc": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0))},
            {"value": float(np.mean(hits)), "queries": m, "what": "|TopK_gpu & TopK_oracle| / K on the CPU sample"},
            rows, s64)


if __name__ == "__main__":
    main()
