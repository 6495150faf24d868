"""Launch tuning through the C ABI (fse_plan_get_tuning / fse_plan_set_tuning)
and the autotuner: defaults by precision, range checks, results unchanged by
the tuning (workgroup shape pinned), and the autotuner leaving the fastest
measured tuning set on the plan."""

import numpy as np
import pytest

import paper_2207_00233_amd as fse
from paper_2207_00233_amd import autotune, synth

pytestmark = pytest.mark.gpu


def _frames():
    rng = np.random.default_rng(43)
    out = []
    for (H, W) in [(96, 128), (64, 80), (130, 70), (80, 160)]:
        img = synth.polygon_image(rng, H, W, radius=(8, 40))
        out.append((img, synth.slice_loss(rng, H, W, 16, (0.2, 0.5))))
    return [f[0] for f in out], [f[1] for f in out]


def test_defaults_and_range_checks():
    with fse.Plan(fse.Params(precision=fse.FSE_FP32_RERANK)) as plan:
        t = plan.get_tuning()
        assert (t["wave_threshold_16"], t["wave_threshold_8"], t["frame_groups"],
                t["crit_depth"], t["crit_prio"], t["crit_waves"]) == (0, 128, 3, 0.9, 1, 4)
        for bad in ({"frame_groups": 17}, {"frame_groups": -1}, {"crit_depth": 1.5},
                    {"wave_threshold_16": -1}, {"crit_prio": 2}, {"crit_waves": 2},
                    {"crit_waves": 32}):
            with pytest.raises(fse.FseError):
                plan.set_tuning(**bad)
        assert plan.get_tuning() == t  # a rejected tuning changes nothing
        plan.set_tuning(frame_groups=0, crit_depth=-1.0, crit_waves=-1)  # back to "by precision"
        assert plan.get_tuning() == t
    with fse.Plan(fse.Params(precision=fse.FSE_FP32)) as plan:
        t = plan.get_tuning()
        assert (t["wave_threshold_16"], t["wave_threshold_8"], t["frame_groups"],
                t["crit_depth"], t["crit_waves"]) == (128, 0, 3, 0.9, 4)
    with fse.Plan(fse.Params(precision=fse.FSE_FP64)) as plan:
        t = plan.get_tuning()
        assert (t["frame_groups"], t["crit_depth"], t["crit_waves"]) == (3, 0.9, 4)


@pytest.mark.parametrize("precision", [fse.FSE_FP32_RERANK, fse.FSE_FP32])
def test_tuning_does_not_change_results(precision):
    imgs, losts = _frames()
    p = fse.Params(border_d=14, iterations=50, precision=precision)
    res = []
    with fse.Plan(p) as plan:
        for groups, crit in ((1, 0.0), (4, 0.5), (2, 0.0)):
            plan.set_tuning(wave_threshold_16=0, wave_threshold_8=0, frame_groups=groups,
                            crit_depth=crit, crit_waves=4)
            res.append(plan.fse_conceal_image(imgs, losts, want_float=True))
            assert plan.last_call_stats()["groups"] == groups
    for other in res[1:]:
        for a, b in zip(res[0], other):
            np.testing.assert_array_equal(a.out_f, b.out_f)


def test_autotune_sets_the_fastest_tuning():
    imgs, losts = _frames()
    p = fse.Params(border_d=14, iterations=50, precision=fse.FSE_FP32)
    grid = {"frame_groups": (1, 2), "crit_depth": (0.0, 0.5)}
    with fse.Plan(p) as plan:
        best, results = autotune.autotune(
            plan, lambda: plan.fse_conceal_image(imgs, losts), grid=grid, reps=2)
        # (1, 0.5) coincides with (1, 0.0): three distinct tunings
        assert len(results) == 3
        assert best == min(results, key=lambda r: r[1])[0]
        assert plan.get_tuning() == best


def test_measured_peaks_are_plausible():
    # the microbenchmarks behind the benchmark's measured roofline peaks:
    # within a factor of the published MI355X figures (FP32 78.6 TFLOP/s
    # without packed instructions, FP64 78.6, HBM 8 TB/s)
    pk = fse.measure_peaks()
    print(f"[gpu] peaks {pk}", flush=True)
    assert pk["compute_units"] > 0
    assert 10.0 < pk["fp32_fma_tflops"] < 100.0
    assert 10.0 < pk["fp64_fma_tflops"] < 100.0
    assert 5.0 < pk["lds_read_tbps"] < 200.0
    assert 1.0 < pk["hbm_copy_tbps"] < 10.0
