"""The benchmark's host-side arithmetic, on the CPU: the roofline object of
the dominant kernel, the per-phase rooflines, the clock/power summary and
the refusal of more than one GPU.  (The measured figures themselves come
from GPU runs; these check how they are turned into the JSON line.)"""
import os
import subprocess
import sys

import pytest

import bench
from paper_2512_23969_amd import accounting as acc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _res(param, phase_ms, msgs, launches=2, clock=None, dedup=None):
    phases = {p: (0.0, 0, 0) for p in ("prelude", "fors", "tree", "wots", "fused")}
    for p, ms in phase_ms.items():
        phases[p] = (ms * launches, launches, msgs * launches)
    gpu = {"gfx_clock_mhz": {"mean": clock} if clock else None, "socket_power_w": None}
    return {"phases": phases, "dedup": dedup, "gpu": gpu}


@pytest.mark.parametrize("param", [1, 2, 3, 7])
def test_roofline_of_the_fused_kernel(param):
    msgs, ms = 4096, 14.0
    r = bench.roofline(param, _res(param, {"fused": ms, "prelude": 0.05, "wots": 0.13}, msgs, clock=2300.0))
    assert r["kernel"] == "k_fused" and r["bound"] == "alu" and r["unit"].startswith("TOP/s")
    # achieved prices every unit at the textbook count; isa_frac at the compiled count
    ops = (acc.ops_per_signature(param, "fors", textbook=True) + acc.ops_per_signature(param, "tree", textbook=True)) * msgs
    assert r["achieved"] == pytest.approx(ops / (ms / 1e3) / 1e12, rel=1e-3)
    isa = (acc.ops_per_signature(param, "fors") + acc.ops_per_signature(param, "tree")) * msgs
    assert r["isa_frac"] == pytest.approx(isa / (ms / 1e3) / acc.VALU_PEAK_OPS, abs=1e-4)
    assert r["peak"] == pytest.approx(acc.VALU_PEAK_OPS / 1e12, rel=1e-4)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert r["avg_launch_ms"] == pytest.approx(ms)
    # units per launch: the per-signature hash counts of FORS + TREE times the batch
    c = acc.per_signature(param)
    for h, n in r["units_per_launch"].items():
        assert n == int((c[h]["fors"] + c[h]["tree"]) * msgs)
    # the same fraction against the peak at the sampled clock
    assert r["frac_at_measured_clock"] == pytest.approx(r["frac"] * 2400.0 / 2300.0, abs=1e-3)
    assert r["mix_ceiling_frac"] == pytest.approx(acc.mix_ceiling_seconds(r["units_per_launch"]) / (ms / 1e3),
                                                  abs=1e-3)


def test_roofline_of_the_plain_path_and_dedup_scaling():
    # plain mode: k_tree is the dominant kernel; with dedup only the distinct
    # trees count as work
    res = _res(1, {"tree": 10.0, "fors": 1.0}, 4096, dedup=(1000, 800))
    r = bench.roofline(1, res)
    assert r["kernel"] == "k_tree" and r["clock_mhz"] is None and r["frac_at_measured_clock"] is None
    full = bench.roofline(1, _res(1, {"tree": 10.0, "fors": 1.0}, 4096))
    assert r["achieved"] == pytest.approx(full["achieved"] * 0.8, rel=1e-3)


def test_roofline_of_a_graph_replay():
    # the whole step against its FORS + TREE work
    msgs, step = 4096, 25.0
    res = {"cfg": {"batch": msgs}, "ms_per_step": step, "dedup": None}
    r = bench.graph_roofline(2, res)
    ops = (acc.ops_per_signature(2, "fors", textbook=True) + acc.ops_per_signature(2, "tree", textbook=True)) * msgs
    assert r["achieved"] == pytest.approx(ops / (step / 1e3) / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    assert r["traffic"] is None and r["avg_launch_ms"] == pytest.approx(step)
    # with tree dedup only the distinct trees count
    d = bench.graph_roofline(2, dict(res, dedup=(1000, 800)))
    dops = (acc.ops_per_signature(2, "fors", textbook=True) + 0.8 * acc.ops_per_signature(2, "tree", textbook=True)) * msgs
    assert d["achieved"] == pytest.approx(dops / (step / 1e3) / 1e12, rel=1e-3)


def test_phase_rooflines():
    msgs = 4096
    pr = bench.phase_rooflines(1, _res(1, {"prelude": 0.05, "fors": 1.0, "tree": 12.0, "wots": 0.13}, msgs))
    assert set(pr) == {"prelude", "fors", "tree", "wots"}
    assert pr["wots"]["bound"] == "hbm"
    b = acc.wots_gather_bytes(1) * msgs
    assert pr["wots"]["achieved"] == pytest.approx(b / 0.13e-3 / 1e9, rel=1e-3)
    assert pr["wots"]["frac"] == pytest.approx(b / 0.13e-3 / 8e12, abs=1e-4)
    t = acc.ops_per_signature(1, "tree") * msgs
    assert pr["tree"]["frac"] == pytest.approx(t / 12e-3 / acc.VALU_PEAK_OPS, abs=1e-4)


def test_telemetry_summary_drops_the_settle_window():
    s = bench.GpuSampler.__new__(bench.GpuSampler)
    s.period, s.settle, s.err = 0.01, 1.0, None
    # (seconds since start, MHz, W): the first second still shows idle figures
    s.samples = [(0.1, 94.0, 240.0), (0.5, 94.0, 240.0), (1.0, 2390.0, 1000.0), (1.5, 2394.0, 1010.0)]
    out = s.summary()
    assert out["samples"] == 2
    assert out["gfx_clock_mhz"] == {"mean": 2392.0, "min": 2390.0, "max": 2394.0}
    assert out["socket_power_w"] == {"mean": 1005.0, "min": 1000.0, "max": 1010.0}
    s.samples = [(0.2, 94.0, 240.0)]
    assert s.summary()["gfx_clock_mhz"] is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_energy_summary_and_per_set_percentiles():
    e = bench.energy_summary(100.0, 112.0, 0.0, 2.0, 8192, "window")
    assert e["mean_power_w"] == 6.0 and e["joules_per_signature"] == pytest.approx(12.0 / 8192, abs=1e-7)
    # a counter that did not advance (or is missing) gives no figure
    assert bench.energy_summary(100.0, 100.0, 0.0, 2.0, 8192, "w") is None
    assert bench.energy_summary(None, 1.0, 0.0, 2.0, 8192, "w") is None

    class _Slh:
        NAMES = {1: "128f", 2: "192f"}
    params = [1, 2] * 50
    lat = [0.001 * (i + 1) for i in range(100)]
    out = bench.per_set_latency(_Slh, params, lat, skip=10)
    assert out["128f"]["requests"] == 45 and out["192f"]["requests"] == 45
    # 128f holds the odd ranks 11, 13, ..., 99 (ms): the median is the 23rd of 45
    assert out["128f"]["p50_ms"] == pytest.approx(55.0) and out["128f"]["p99_ms"] == pytest.approx(99.0)


def test_traffic_only_from_counters_on_the_current_kernels(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.profiled_traffic("c2_128f_4096", "fused", "k_fused") == (None, "no counter summary")
    import json
    f.write_text(json.dumps({"device_source_sha256": bench.device_source_hash(),
                             "entries": {"c2_128f_4096/fused/k_fused": {"bytes_per_launch": 123, "summary": "x.md"}}}))
    assert bench.profiled_traffic("c2_128f_4096", "fused", "k_fused") == (123, "x.md")
    # another mode runs other kernels (or the same kernel over other trees)
    assert bench.profiled_traffic("c2_128f_4096", "fused-dedup", "k_fused")[0] is None
    assert bench.profiled_traffic("c3_192f_4096", "plain", "k_tree")[0] is None
    f.write_text(json.dumps({"device_source_sha256": "0" * 64,
                             "entries": {"c2_128f_4096/fused/k_fused": {"bytes_per_launch": 123}}}))
    assert bench.profiled_traffic("c2_128f_4096", "fused", "k_fused")[0] is None