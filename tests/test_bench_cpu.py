"""The benchmark's stdout line stays short enough for a log tail to hold it whole."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

X = 0.123456789012345  # a float with every digit, as measured values have


def full_record() -> dict:
    """A record with every arm present and long numbers everywhere."""
    eps3 = {f"eps={e:g}": None for e in (0.0, 1e-3, 1e-2)}
    return {
        "metric": "time-to-residual-1e-6 at 2049^2 2D HJB (patchy method, warm start from u_hat)",
        "value": X, "unit": "s", "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": X, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded instance generator)",
        "config": {"workload": "w" * 200, "n": 2049, "h": X, "dx": X, "eps": 0.0, "tol": 1e-6, "free_nodes": 3800000,
                   "seed": 0, "n_controls": 64, "patches": 64},
        "stages_s": {k: X for k in ("t_coarse", "t_upsample", "t_synthesize", "t_label", "t_solve")},
        "passes": 300, "node_updates_per_s": X, "node_updates_per_free_node": X, "policy_updates_per_free_node": X,
        "check_sweeps": {"per_step": X, "node_update_share": X, "visit_time_share": X, "visit_ms_per_step": X},
        "accuracy_vs_oracle": {"nodes": 65536, "max_abs": X, "mean_abs": X, "oracle_residual": X, "oracle_sweeps": 2000},
        "speedup_vs_global_jacobi_cold": X,
        "roofline": {"kernel": "k" * 60, "bound": "alu", "achieved": X, "peak": 157.3, "unit": "TFLOP/s", "frac": X,
                     "traffic": X, "avg_launch_us": X, "visit_ms_per_step": X, "measured_over": "m" * 300,
                     "flops_per_node_update": 1474, "flops_per_policy_update": 25},
        "cpu_baseline": {"value": X, "unit": "s", "cores": 16, "kind": "oracle", "cpu_model": "c" * 60,
                         "sample": "s" * 250},
        "arms": {
            "global_jacobi_cold": {"time_s": X, "sweeps": 1672, "node_updates_per_s": X, "sweep_kernel_us": X,
                                   "sweep_kernel_frac": X, "max_abs_vs_oracle": X},
            "global_jacobi_uhat": {"time_s_after_uhat": X},
            "static_decomposition_cold": {"time_s": X},
            "c2_diffusion": {k: {"patchy_time_s": X, "global_jacobi_cold_s": X, "max_abs_diff": X}
                             for k in ("eps=0.001", "eps=0.01")},
            "independent_patches": {k: {"decomposition_error_max": X, "band_max": X, "interior_max": X,
                                        "interior_mean": X} for k in eps3},
            "h_equals_dx": {"patchy_time_s": X, "global_jacobi_cold_s": X, "halo": 3},
            "batch_256_instances": {"time_s_batched": X, "time_s_sequential": X, "bit_exact_vs_single": "256/256",
                                    "active_tiles": {"time_s_batched": X, "time_s_sequential": X,
                                                     "bit_exact_vs_single": "256/256"}},
            "rank1_bumps": {k: {"time_s": X} for k in ("full_sweeps", "active_tiles_cold", "active_tiles_uhat")},
            "balanced_patches": {"largest_over_mean": [2.0, 1.5], "kept_round": 1, "time_s": X},
            "learned_warm_start": {"train_problems": 192,
                                   "start_error_mean": {"uhat": X, "uhat_bicubic": X, "network": X},
                                   "jacobi_sweeps": {"cold": X, "uhat": X, "uhat_bicubic": X, "network": X},
                                   "active_tiles_time_s": {"uhat": X, "uhat_bicubic": X, "network": X},
                                   "active_tiles_stop_error_max": {"uhat": X, "uhat_bicubic": X, "network": X}},
            "exit_to_boundary": {"table0": [{"equation": e, "eps": eps, "jacobi_sweeps_sl2": 1000,
                                             "jacobi_sweeps_sl3": 1000, "lambda": 0.0}
                                            for e in ("A", "B", "B2", "C") for eps in (0.0, 1e-2)]},
        },
    }


def test_summary_line_is_short_and_complete():
    line = json.dumps(bench.summary_line(full_record()))
    assert len(line) <= 4096, len(line)
    d = json.loads(line)
    for k in ("metric", "value", "unit", "ms_per_step", "dtype", "config", "roofline", "cpu_baseline",
              "accuracy_vs_oracle", "arms"):
        assert k in d
    assert set(d["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert d["cpu_baseline"]["cores"] == 16 and d["cpu_baseline"]["kind"] == "oracle"
    assert "workload" in d["config"] and "h" in d["config"]


def test_summary_line_without_arms():
    rec = full_record()
    rec["arms"] = {}
    del rec["cpu_baseline"], rec["accuracy_vs_oracle"]
    d = json.loads(json.dumps(bench.summary_line(rec)))
    assert d["arms"] == {} and d["value"] == X
