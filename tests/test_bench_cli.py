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
        if phase == "pair":
            # instruction counts come from the committed counter record of the precision
            # workload only: none for this scene
            assert r["frac"] is None and r["achieved"] is None
        else:
            assert 0.0 < r["frac"] == round(r["achieved"] / r["peak"], 4)
        json.dumps(r, allow_nan=False)


def test_exhaustive_roofline_from_the_counter_record():
    """The exhaustive pass's ALU fraction: FP32 arithmetic VALU instructions per pair from
    profiles/valu.json times the launch's pairs, over the VALU issue peak (256 CU x 4 SIMD x 16
    lanes x 2.4 GHz); skipped when the record no longer matches the kernel source."""
    import pytest
    sys.path.insert(0, ROOT)
    import bench
    from synth import CONFIGS, make_queries, make_scene

    rec = bench.recorded_valu("k_pair_exhaustive", "precision")
    if rec is None:
        pytest.skip("no VALU record for the current kernel source")

    class Args:
        form, method = "f32", "exhaustive"

    cfg = CONFIGS["tiny"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)

    class Precision:
        name = "precision"

    phases = {"pair": (2.0, 2), "gemm": (0.1, 2)}
    r = bench.dominant_roofline(phases, scene, qb, Args, Precision, None)
    pairs = float(qb.r_tot) * scene.n * (scene.n - 1)
    want = rec["fp32_arith_insts"] * 64.0 / rec["pair_evals"] * pairs / 1e-3 / 1e12
    assert abs(r["achieved"] - want) <= 1e-3 * want + 1e-3
    assert r["peak"] == 39.3216
    assert r["frac"] == round(r["achieved"] / r["peak"], 4)
    assert r["valu_issue_frac"] >= r["frac"]
