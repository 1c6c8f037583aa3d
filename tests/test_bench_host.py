"""Host logic of bench.py (no GPU): the committed counter summaries of the
dominant kernel match its current source and the measured launch shape, so
the benchmark line carries measured HBM traffic and VALU issue; a different
launch shape or source is refused (null), never reported."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_counter_summaries_match_the_kernel_source():
    b = _bench()
    plan = (16, 2, 512)  # the launch shape the summaries were taken with
    traffic = b.measured_traffic(plan)
    assert traffic is not None, "k_tile2d.hip or em_slots.hpp changed since the counters were taken: profile again"
    # about 16 MB per packed launch of two sweeps, well below the 201.3 MB of
    # algorithmic int8 bytes
    assert 10e6 < traffic < 30e6
    v = b.measured_valu(plan, 34.8e-6)
    assert v is not None and 0.5 < v["frac"] < 1.0
    assert b.VALU_PEAK_WAVE_INSTS == 256 * 4 * 2.4e9 / 4


def test_default_plan_is_the_profiled_one():
    b = _bench()
    assert b.PROFILED_PLAN == "16,2,512"
    assert b.measured_traffic(tuple(int(x) for x in b.PROFILED_PLAN.split(","))) is not None


def test_other_launch_shapes_are_refused():
    b = _bench()
    assert b.measured_traffic((16, 4, 512)) is None
    assert b.measured_valu((8, 2, 512), 34.8e-6) is None


def test_cpu_baseline_leg_reports_all_cores_and_one_thread():
    """The oracle leg of the benchmark runs on the host only; a short sample."""
    b = _bench()
    out = b.cpu_baseline(1.5)
    assert out["kind"] == "oracle" and out["unit"] == "spin flips/ns" and out["value"] > 0 and out["cores"] >= 1
    st = out["single_thread"]
    assert st["cores"] == 1 and st["value"] > 0
    assert st["value"] <= out["value"] * 1.5 or out["cores"] == 1  # one thread is not faster than all


def test_run_env_fields():
    import torch

    env = _bench().run_env(torch)
    assert set(env) == {"gpu", "hip", "torch", "host_threads"} and env["host_threads"] >= 1
    assert env["torch"] == torch.__version__
