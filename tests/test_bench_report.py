"""Host logic of the benchmark's report (no GPU): the choice of the fastest
reduced-run schedule that meets the 1e-2 stress bar at t_end."""
import bench


def _pod(start=(0.04, 0.026)):
    sweep = lambda pairs: {f"freeze_every_{n}": {"T_over_T_ref": t, "stress_rel_err_vs_plain": s}
                           for n, (t, s) in pairs.items()}
    return {"T_rom_over_T_ref": start[0], "stress_rel_err_vs_plain": start[1],
            "freeze_sweep": sweep({100: (0.10, 0.013), 50: (0.20, 0.0085)}),
            "midpoint_freeze_sweep": sweep({200: (0.102, 0.0052)}),
            "extrapolated_midpoint_freeze_sweep": sweep({200: (0.057, 0.023), 150: (0.077, 0.0032)}),
            "exact_windows": {"T_over_T_ref": 0.038, "stress_rel_err_vs_plain": 0.0257},
            "adaptive_windows": {"T_over_T_ref": 0.12, "stress_rel_err_vs_plain": 0.0198}}


def test_fastest_schedule_within_the_bar():
    best = bench.pod_best_within(_pod(), 1e-2)
    assert best == {"time_ratio": 0.077, "stress_err": 0.0032, "schedule": "extrapolated-midpoint freezes every 150"}


def test_default_schedule_wins_when_it_meets_the_bar():
    best = bench.pod_best_within(_pod(start=(0.04, 0.009)), 1e-2)
    assert best["schedule"] == "start freezes every 300" and best["time_ratio"] == 0.04


def test_none_within_the_bar():
    assert bench.pod_best_within(_pod(), 1e-3) is None
