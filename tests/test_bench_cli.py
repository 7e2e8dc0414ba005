"""bench.py's command-line contract that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_of_each_phase_kind():
    """The roofline block names the kernel, its bound and a fraction of the published peak."""
    sys.path.insert(0, ROOT)
    import bench
    from synth import CONFIGS, make_queries, make_scene

    class Args:
        form, method = "bf16", "proposal"

    cfg = CONFIGS["tiny"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)
    info = {"terms_per_step": 100, "list_m": 16, "fp32_dots_per_step": 10, "fallback_rate": 0.1, "pass_in_lds": True}
    cases = {"gemm": ("mfma", "k_sim_gemm<bf16>"), "pair": ("alu", "k_pair_exhaustive"),
             "topk": ("hbm", "k_bound_candidates"), "rescore": ("hbm", "k_rescore_subset_lds"),
             "propose": ("hbm", "k_semantic_sets")}

    class Bounded:
        form, method = "bf16", "bounded"

    runs = [(Args, info, phase, want) for phase, want in cases.items()]
    # full anchor scans: the proposal method's fallback and the bound-pruned method's candidate terms
    runs.append((Args, dict(info, terms_per_step=10**7, fallback_rate=0.5), "fallback",
                 ("alu", "k_rescore_fallback")))
    runs.append((Bounded, {"full_scan_terms_per_step": 10**7}, "rescore", ("alu", "k_rescore_terms<full>")))
    for a, inf, phase, (bound, kernel) in runs:
        phases = {p: (1e-4, 1) for p in ("normalize", "gemm", "pair", "topk", "rescore", "propose", "fallback")}
        phases[phase] = (1e-3, 1)
        r = bench.dominant_roofline(phases, scene, qb, a, cfg, inf)
        assert r["bound"] == bound and r["kernel"].startswith(kernel), (phase, r)
        assert 0.0 < r["frac"] == round(r["achieved"] / r["peak"], 4)
        json.dumps(r, allow_nan=False)
