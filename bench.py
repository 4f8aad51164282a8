#!/usr/bin/env python3
"""Throughput benchmark of batched SPHINCS+ signing on one MI355X.

One step = one slh_sign_batch call over the whole batch (prelude, FORS,
TREE and WOTS kernels), inputs and outputs resident in HBM.  Prints one
JSON line.  Headline workload: SPHINCS+-SHA2-128f, one key, 4096 random
32-byte messages, in its autotuned mode.  The line also carries, under
"extra", the 192f (1 key) and 256f (64 keys) batch-4096 workloads and the
128f one again, each in its autotuned mode and in the plain per-phase path,
with a roofline object each; "serving" holds the continuous-batching
workload with p50/p99 per parameter set.  --all adds the small sets, the
SHAKE sets, the other modes and the small-batch latencies.
"""
from __future__ import annotations

import argparse
import contextlib
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2512_23969_amd import workloads as _workloads  # noqa: E402  (numpy only)

WORKLOADS = {
    "c2_128f_4096": "SPHINCS+-SHA2-128f, 1 key, 4096 x 32-byte messages, one fused persistent launch",
    "c3_192f_4096": "SPHINCS+-SHA2-192f, 1 key, 4096 x 32-byte messages, hipGraph-captured pipeline",
    "c4_256f_4096x64": "SPHINCS+-SHA2-256f, 64 keys, 4096 x 32-byte messages, one fused multi-key launch",
    "s1_128s_1024": "SPHINCS+-SHA2-128s, 1 key, 1024 x 32-byte messages",
    "s2_192s_1024": "SPHINCS+-SHA2-192s, 1 key, 1024 x 32-byte messages",
    "s3_256s_1024": "SPHINCS+-SHA2-256s, 1 key, 1024 x 32-byte messages",
    "k1_shake128f_4096": "SPHINCS+-SHAKE-128f, 1 key, 4096 x 32-byte messages",
    "k2_shake192f_4096": "SPHINCS+-SHAKE-192f, 1 key, 4096 x 32-byte messages",
    "k3_shake256f_4096x64": "SPHINCS+-SHAKE-256f, 64 keys, 4096 x 32-byte messages",
    "k4_shake128s_1024": "SPHINCS+-SHAKE-128s, 1 key, 1024 x 32-byte messages",
}


# the metric as the benchmark specification names it; the value is the 128f
# workload's, and "extra" holds the 192f and 256f ones
METRIC = "signatures/s (128f/192f/256f, batch 4096) + p50/p99 latency; % VALU peak"
# the batch-4096 workloads of the default line, each in the execution mode
# its configuration names and in the plain per-phase path
DEFAULT_WORKLOADS = ("c2_128f_4096", "c3_192f_4096", "c4_256f_4096x64")
# the mode each batch-4096 configuration is timed in ("graph-any": the
# hipGraph-captured pipeline over the per-phase kernels or over the fused
# kernel, whichever the autotuner found faster)
CONFIG_MODE = {name: c["mode"] for name, c in _workloads.CONFIGS.items() if "mode" in c}


# HBM bytes per launch measured with rocprofv3 counters, valid while the
# device sources hash to the value recorded with them
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_b4096.json")
DEVICE_SOURCES = ("kernels.hpp", "slh_dev.hpp", "sha2_dev.hpp", "keccak_dev.hpp", "set_impl.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def device_source_hash() -> str:
    """SHA-256 of the device code and launch sources (kernels and their grids)."""
    h = hashlib.sha256()
    for f in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_23969_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload: str, mode: str, kernel: str):
    """(bytes per launch, source) of `kernel` in `workload` signed in `mode`,
    from the committed counter summary when it was taken on the current
    device sources, else (None, reason)."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None, "no counter summary"
    e = t.get("entries", {}).get("%s/%s/%s" % (workload, mode, kernel))
    if e is None:
        return None, "not profiled"
    if t.get("device_source_sha256") != device_source_hash():
        return None, "kernels changed since the counters were taken"
    return int(e["bytes_per_launch"]), e.get("summary", os.path.relpath(TRAFFIC_FILE, ROOT))


def setup(slh, workloads, name):
    import numpy as np
    import torch
    cfg = workloads.CONFIGS[name]
    param, batch = cfg["param"], cfg["batch"]
    ctx = slh.Context(0)
    slots = []
    ctx.pks = []
    for i in range(cfg["keys"]):
        pk, sk = slh.keygen(param, workloads.key_seed(param, i))
        slots.append(ctx.add_keys(param, sk))
        ctx.pks.append(pk)
    if cfg["keys"] > 1:
        kidx = workloads.key_assignment(cfg["cfg"], batch, cfg["keys"])
    else:
        kidx = [0] * batch
    msgs = workloads.messages(cfg["cfg"], batch, cfg["length"])
    items, blob, total = slh.pack_batch([param] * batch, [slots[k] for k in kidx], msgs)
    d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
    d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
    return ctx, items, d_m, d_s, cfg, msgs, kidx


def verify_inputs(slh, ctx, items, d_m, d_s, cfg, kidx):
    """(items, msgs, sigs, pks, results) verifying the batch's signatures."""
    import numpy as np
    import torch
    param, batch = cfg["param"], cfg["batch"]
    npk = 2 * slh.sizes(param)["n"]
    d_pk = torch.frombuffer(bytearray(b"".join(ctx.pks)), dtype=torch.uint8).cuda()
    vit = np.zeros(batch, dtype=slh.VERIFY_DTYPE)
    vit["param"] = param
    vit["msg_off"] = items["msg_off"]
    vit["msg_len"] = items["msg_len"]
    vit["sig_off"] = items["sig_off"]
    vit["pk_off"] = np.asarray(kidx, dtype=np.uint64) * npk
    res = torch.zeros(batch, dtype=torch.int32, device="cuda")
    return vit, d_m, d_s, d_pk, res


def verify_leg(slh, ctx, items, d_m, d_s, cfg, kidx, steps):
    """Batched GPU verification of the batch just signed: every signature
    must verify; throughput over `steps` launches."""
    import torch
    batch = cfg["batch"]
    vit, d_m, d_s, d_pk, res = verify_inputs(slh, ctx, items, d_m, d_s, cfg, kidx)
    ctx.verify_batch(vit, d_m, d_s, d_pk, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.verify_batch(vit, d_m, d_s, d_pk, res)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"value": round(batch * steps / el, 1), "unit": "verifications/s",
            "ms_per_batch": round(1e3 * el / steps, 3), "all_valid": int(res.sum()) == batch}


class GpuSampler:
    """Samples the graphics clock (MHz) and socket power (W) of the GPU that
    torch calls device 0, through amdsmi on a host thread.  The amdsmi device
    is the one at the same PCI address; if none matches or amdsmi is missing,
    the summary says why and holds no figures.  The firmware's metrics lag
    the load by a fraction of a second, so the summary drops the samples of
    the first `settle_s` seconds."""

    def __init__(self, period_s=0.01, settle_s=1.0):
        import threading
        self.period, self.settle, self.h, self.err = period_s, settle_s, None, None
        self.energy_err = None
        self.samples = []  # (seconds since start, clock MHz, power W)
        self.stop = threading.Event()
        self.th = None
        try:
            import amdsmi
            import torch
            amdsmi.amdsmi_init()
            pr = torch.cuda.get_device_properties(0)
            want = "%04x:%02x:%02x." % (int(pr.pci_domain_id), int(pr.pci_bus_id), int(pr.pci_device_id))
            for h in amdsmi.amdsmi_get_processor_handles():
                if amdsmi.amdsmi_get_gpu_device_bdf(h).lower().startswith(want):
                    self.h = h
            if self.h is None:
                self.err = "no amdsmi device at PCI address " + want
            self.amdsmi = amdsmi
        except Exception as e:  # telemetry is optional; the benchmark is not
            self.err = repr(e)

    def _loop(self):
        a = self.amdsmi
        t0 = time.perf_counter()
        while not self.stop.is_set():
            try:
                c = a.amdsmi_get_clock_info(self.h, a.AmdSmiClkType.GFX)
                w = a.amdsmi_get_power_info(self.h)
                c = c.get("clk", c.get("cur_clk"))
                w = w.get("current_socket_power", w.get("socket_power"))
                if isinstance(c, (int, float)) and isinstance(w, (int, float)):
                    self.samples.append((time.perf_counter() - t0, float(c), float(w)))
            except Exception as e:
                self.err = repr(e)
                return
            self.stop.wait(self.period)

    def __enter__(self):
        import threading
        if self.h is not None:
            self.th = threading.Thread(target=self._loop, daemon=True)
            self.th.start()
        return self

    def __exit__(self, *exc):
        self.stop.set()
        if self.th:
            self.th.join()

    def energy_j(self):
        """The GPU's accumulated energy in joules (amdsmi's energy counter:
        accumulator x resolution in microjoules), or None."""
        if self.h is None:
            return None
        try:
            e = self.amdsmi.amdsmi_get_energy_count(self.h)
            count = e.get("energy_accumulator", e.get("power"))
            res = e.get("counter_resolution")
            if isinstance(count, (int, float)) and isinstance(res, (int, float)) and res > 0:
                return float(count) * float(res) * 1e-6
            self.energy_err = "energy counter fields: %s" % sorted(e)
        except Exception as ex:  # telemetry is optional
            self.energy_err = repr(ex)
        return None

    def summary(self):
        def st(v):
            return {"mean": round(sum(v) / len(v), 1), "min": min(v), "max": max(v)} if v else None
        kept = [x for x in self.samples if x[0] >= self.settle]
        out = {"source": "amdsmi every %d ms over further untimed steps of the same workload, first %.1f s "
                         "dropped" % (round(1e3 * self.period), self.settle),
               "samples": len(kept), "gfx_clock_mhz": st([x[1] for x in kept]),
               "socket_power_w": st([x[2] for x in kept])}
        if self.err:
            out["error"] = self.err
        if getattr(self, "energy_err", None):
            out["energy_error"] = self.energy_err
        return out


def energy_summary(e0, e1, t0, t1, signatures, what):
    """Energy over a window from two counter readings (None if the counter
    is unavailable or did not advance)."""
    if e0 is None or e1 is None or e1 <= e0 or t1 <= t0 or not signatures:
        return None
    return {"window": what, "joules": round(e1 - e0, 3), "seconds": round(t1 - t0, 4), "signatures": signatures,
            "mean_power_w": round((e1 - e0) / (t1 - t0), 1),
            "joules_per_signature": round((e1 - e0) / signatures, 7)}


def run(slh, workloads, name, steps, warmup, mode="plain", tune=False, tune_out=None, verify=False,
        telemetry_s=2.0, knobs=None):
    import torch
    from paper_2512_23969_amd import autotune
    ctx, items, d_m, d_s, cfg, msgs, kidx = setup(slh, workloads, name)
    path = tune_out or autotune.DEFAULT_CACHE
    if tune:
        # the verification stage needs this batch signed first
        ctx.sign_batch(items, d_m, d_s)
        torch.cuda.synchronize()
        best, _ = autotune.tune_and_store(slh, ctx, cfg["param"], items, d_m, d_s, cfg["batch"], path, log=log,
                                          verify=verify_inputs(slh, ctx, items, d_m, d_s, cfg, kidx))
    mode, best = autotune.resolve_mode(cfg["param"], cfg["batch"], mode, path or autotune.DEFAULT_CACHE)
    if knobs:
        # explicit knobs over the tuned ones (profiling one kernel variant)
        best = dict(best or autotune.KNOB_DEFAULTS, **knobs)
    if best:
        autotune.apply(ctx, cfg["param"], best)
        best = {k: v for k, v in best.items() if k != "by_mode"}
    m = slh.MODES[mode]
    ctx.dedup_stats(reset=True)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        ctx.sign_batch(items, d_m, d_s, mode=m, stream=stream)
    torch.cuda.synchronize()
    ctx.phase_times(reset=True)
    ctx.profile(True)
    sampler = GpuSampler() if telemetry_s > 0 else None
    # per-step GPU time from events on the stream the steps run on
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    e_a = sampler.energy_j() if sampler else None
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        ctx.sign_batch(items, d_m, d_s, mode=m, stream=stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    e_b = sampler.energy_j() if sampler else None
    ctx.profile(False)
    step_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    phases = ctx.phase_times(reset=True)
    trees, distinct = ctx.dedup_stats(reset=True)
    energy = {"timed_steps": energy_summary(e_a, e_b, t0, t1, steps * cfg["batch"], "the timed steps")}
    # clock, power and energy under this load: further steps outside the
    # timed region, after a settling second (the firmware's figures lag)
    with sampler or contextlib.nullcontext():
        if sampler is not None and sampler.h is not None:
            t2 = time.perf_counter()
            while time.perf_counter() - t2 < sampler.settle:
                for _ in range(4):
                    ctx.sign_batch(items, d_m, d_s, mode=m, stream=stream)
                torch.cuda.synchronize()
            e_c, t3, n = sampler.energy_j(), time.perf_counter(), 0
            while time.perf_counter() - t3 < telemetry_s:
                for _ in range(4):
                    ctx.sign_batch(items, d_m, d_s, mode=m, stream=stream)
                n += 4
                torch.cuda.synchronize()
            e_d, t4 = sampler.energy_j(), time.perf_counter()
            energy["window"] = energy_summary(e_c, e_d, t3, t4, n * cfg["batch"],
                                              "%.1f s of further steps after a 1 s settle" % telemetry_s)
    ver = verify_leg(slh, ctx, items, d_m, d_s, cfg, kidx, steps) if verify else None
    ctx.close()
    elapsed = t1 - t0
    return {
        "elapsed": elapsed,
        "ms_per_step": 1000.0 * elapsed / steps,
        "sig_per_s": cfg["batch"] * steps / elapsed,
        "phases": phases,
        "cfg": cfg,
        "name": name,
        "steps": steps,
        "mode": mode,
        "tuning": best,
        # (trees needed, distinct trees computed) per step, dedup modes only
        "dedup": (trees // (warmup + steps), distinct // (warmup + steps)) if trees else None,
        "verify": ver,
        "step_ms": {"median": round(step_ms[len(step_ms) // 2], 4), "min": round(step_ms[0], 4),
                    "max": round(step_ms[-1], 4)},
        "gpu": sampler.summary() if sampler is not None else {"source": "off", "gfx_clock_mhz": None,
                                                               "socket_power_w": None},
        "energy": energy,
    }


def host_cpu():
    """The host's CPU model and core counts."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"model": model or platform.processor() or None, "os_cpu_count": os.cpu_count(),
            "affinity_cores": affinity}


def cpu_baseline(name, workloads, seconds=15.0):
    """The oracle, as it stands, on the host cores: sign messages of the same
    workload with one thread per core this process may run on, for about
    `seconds`; then on one thread for about a tenth of that."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    cfg = workloads.CONFIGS[name]
    param = cfg["param"]
    p = oracle.params(workloads.NAME_OF[param])
    pk, sk = oracle.keygen(p, workloads.key_seed(param, 0))
    msgs = workloads.messages(cfg["cfg"], cfg["batch"], cfg["length"])
    host = host_cpu()
    threads = host["affinity_cores"]
    done = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds and done < len(msgs):
            chunk = msgs[done:done + threads]
            list(ex.map(lambda m: oracle.sign(p, m, sk), chunk))
            done += len(chunk)
    el = time.perf_counter() - t0
    one, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < seconds / 10 and one < 64:
        oracle.sign(p, msgs[(done + one) % len(msgs)], sk)
        one += 1
    el1 = time.perf_counter() - t1
    return {"value": done / el, "unit": "signatures/s", "cores": threads, "kind": "oracle",
            "sample": "first %d messages of the %s workload, key 0, %d host threads (one per core of the "
                      "process's affinity), %.1f s" % (done, name, threads, el),
            "host": host,
            "single_thread": {"value": one / el1, "sample": "%d messages, 1 thread, %.1f s" % (one, el1)}}


def latency_bench(slh, workloads, reps=20):
    """Small-batch latency: key generation, and one slh_sign_batch call plus
    synchronisation for batches of 1, 16 and 64 messages of 256 bytes of one
    set (fused mode; such batches take the split per-phase path), median of
    `reps` calls after warm-up."""
    import torch
    out = {"keygen_ms": {}, "sign_ms": {}}
    ctx = slh.Context(0)
    for p in (1, 2, 3, 7):
        ts = []
        for i in range(5):
            t0 = time.perf_counter()
            slh.keygen(p, workloads.key_seed(p, 2000 + i))
            ts.append(time.perf_counter() - t0)
        out["keygen_ms"][slh.NAMES[p]] = round(1e3 * sorted(ts)[2], 3)
        slot = ctx.add_keys(p, slh.keygen(p, workloads.key_seed(p, 2000))[1])
        for batch in (1, 16, 64):
            msgs = workloads.messages(90 + p, batch, 256)
            items, blob, total = slh.pack_batch([p] * batch, [slot] * batch, msgs)
            d_m = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
            d_s = torch.zeros(total, dtype=torch.uint8, device="cuda")
            for _ in range(3):
                ctx.sign_batch(items, d_m, d_s, mode=slh.MODES["fused"])
            torch.cuda.synchronize()
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                ctx.sign_batch(items, d_m, d_s, mode=slh.MODES["fused"])
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            out["sign_ms"]["%s/%d" % (slh.NAMES[p], batch)] = round(1e3 * sorted(ts)[reps // 2], 3)
    ctx.close()
    return out


def percentile(v, q):
    """The library's percentile: the element at rank round(q (len - 1)) of the sorted values."""
    return v[min(len(v) - 1, int(q * (len(v) - 1) + 0.5))]


def per_set_latency(slh, params, lat, skip):
    """p50 / p99 latency (ms) of each parameter set's requests after the first `skip`."""
    import numpy as np
    p = np.asarray(params[skip:])
    lat = np.asarray(lat[skip:])
    out = {}
    for prm in sorted(set(params)):
        v = np.sort(lat[p == prm])
        if len(v):
            out[slh.NAMES[prm]] = {"requests": int(len(v)), "p50_ms": round(float(percentile(v, 0.5)) * 1e3, 3),
                                   "p99_ms": round(float(percentile(v, 0.99)) * 1e3, 3)}
    return out


def serve_bench(slh, workloads, n, rates, log, mode="fused", cache_layers=0, lanes=4, schedule="items"):
    """Serving workload: n requests, parameter set 50/30/20 % 128f/192f/256f,
    256 device-resident keys (128/77/51), log-normal message lengths (median
    256 B, 32 B - 16 KiB), random bytes.  First all requests at time 0 (the
    saturated rate), then Poisson arrivals at fractions of that rate.
    Latency = completion - arrival, PCIe transfers included (messages in from
    host memory, signatures out to host memory)."""
    import numpy as np
    import torch
    keys_per_set = (128, 77, 51)
    t0 = time.perf_counter()
    reqs = workloads.serving_requests(n, keys_per_set=keys_per_set)
    params = [p for p, _, _ in reqs]
    kidx = [k for _, k, _ in reqs]
    msgs = [m for _, _, m in reqs]
    log("serve: %d requests generated in %.1f s" % (n, time.perf_counter() - t0))
    srv = slh.Server(0, lanes=lanes, max_batch=4096, max_wait_us=2000, mode=slh.MODES[mode],
                     cache_layers=cache_layers)
    slots = {}
    sks = {}
    for p, cnt in zip((1, 2, 3), keys_per_set):
        sks[p] = [slh.keygen(p, workloads.key_seed(p, 1000 + i))[1] for i in range(cnt)]
        slots[p] = srv.add_keys(p, sks[p])
        if schedule == "chunks":
            srv.set_tuning(p, fused_schedule=slh.FUSED_CHUNKS)
    ks = [slots[p] + k for p, k in zip(params, kidx)]
    out = {"requests": n, "mix": "50/30/20 % 128f/192f/256f", "keys": 256,
           "msg_len": "log-normal, median 256 B, clipped to [32, 16384]", "lanes": lanes, "max_batch": 4096,
           "max_wait_us": 2000, "mode": mode, "cache_layers": cache_layers, "fused_schedule": schedule,
           "latency": "arrival to completion, host buffers (PCIe included)",
           "points": []}
    reqs0, blob = slh.trace(params, ks, msgs, [0.0] * n)
    sigs, lat, st = srv.replay(reqs0, blob)
    sat = st["sig_per_s"]
    out["saturated_sig_per_s"] = round(sat, 1)
    log("serve: saturated %.0f sig/s, %d launches" % (sat, st["launches"]))
    # bit-exactness of the served signatures: every request against the same
    # requests signed in plain batches of 8192 (alone vs in the mix)
    bad = 0
    with slh.Context(0) as ctx:
        for p in (1, 2, 3):
            ctx.add_keys(p, sks[p])
        for c0 in range(0, n, 8192):
            chk = range(c0, min(n, c0 + 8192))
            ref = slh.sign_messages(ctx, [params[i] for i in chk], [ks[i] for i in chk], [msgs[i] for i in chk])
            for j, i in enumerate(chk):
                sb = slh.sizes(params[i])["sig_bytes"]
                o = int(reqs0[i]["sig_off"])
                bad += sigs[o:o + sb].tobytes() != ref[j]
    out["checked_against_plain_batch"] = n
    out["mismatches"] = int(bad)
    for f in rates:
        arr = workloads.poisson_arrivals(n, f * sat)
        r, blob = slh.trace(params, ks, msgs, arr)
        skip = min(1000, n // 10)
        _, lat, st = srv.replay(r, blob, skip=skip)
        pt = {"load": f, "offered_sig_per_s": round(f * sat, 1), "sig_per_s": round(st["sig_per_s"], 1),
              "p50_ms": round(st["p50_s"] * 1e3, 3), "p99_ms": round(st["p99_s"] * 1e3, 3),
              "mean_batch": round(st["mean_batch"], 1),
              "per_set": per_set_latency(slh, params, lat, skip)}
        out["points"].append(pt)
        log("serve: %s" % pt)
    srv.close()
    return out


def roofline(param, res):
    """Roofline of the dominant kernel: k_fused (FORS + TREE) in the fused
    modes, k_tree in the plain mode.  Kernel time from the library's HIP
    events around that kernel on the benchmark's stream.  `achieved` prices
    each compression at the textbook instruction count (one VALU operation
    per FIPS 180-4 primitive: 1384 per SHA-256, 4144 per SHA-512 block on
    32-bit lanes; 4320 per Keccak-f permutation); `isa_frac` prices it at
    the instructions the compiled kernels issue per compression."""
    from paper_2512_23969_amd import accounting as acc
    phase, kernel, parts = ("fused", "k_fused", ("fors", "tree")) if res["phases"]["fused"][1] else \
        ("tree", "k_tree", ("tree",))
    ms, launches, msgs = res["phases"][phase]
    if launches == 0:
        return None
    per_launch_msgs = msgs / launches
    # with tree dedup only the distinct trees are computed
    scale = {"tree": res["dedup"][1] / res["dedup"][0] if res.get("dedup") else 1.0}
    ops = sum(acc.ops_per_signature(param, p, textbook=True) * scale.get(p, 1.0) for p in parts) * per_launch_msgs
    isa = sum(acc.ops_per_signature(param, p) * scale.get(p, 1.0) for p in parts) * per_launch_msgs
    avg_s = ms / launches / 1000.0
    achieved = ops / avg_s / 1e12
    peak = acc.VALU_PEAK_OPS / 1e12
    c = acc.per_signature(param)
    clk = (res["gpu"]["gfx_clock_mhz"] or {}).get("mean")
    units = {h: int(sum(c[h][p] * scale.get(p, 1.0) for p in parts) * per_launch_msgs)
             for h in ("sha256", "sha512", "keccak") if sum(c[h].values())}
    traffic, source = profiled_traffic(res.get("name", ""), res.get("mode", ""), kernel)
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": round(peak, 3),
            "unit": "TOP/s (32-bit VALU lane-ops)", "frac": round(achieved / peak, 4),
            "traffic": traffic, "traffic_source": source,
            "avg_launch_ms": round(ms / launches, 4),
            "units_per_launch": units,
            "ops_per_unit": {"sha256": acc.TEXTBOOK_SHA256, "sha512": acc.TEXTBOOK_SHA512,
                             "keccak": acc.TEXTBOOK_KECCAK},
            "isa_ops_per_unit": {"sha256": acc.OPS_SHA256, "sha512": acc.OPS_SHA512, "keccak": acc.OPS_KECCAK},
            "isa_frac": round(isa / avg_s / acc.VALU_PEAK_OPS, 4),
            # the same work at the rate each hash's instruction mix reaches in
            # isolation (calibration probe): 1.0 = as fast as that mix runs
            "mix_ceiling_frac": round(acc.mix_ceiling_seconds(units) / avg_s, 4),
            "single_rate_frac": round(isa / avg_s / acc.VALU_SINGLE_RATE_OPS, 4),
            # the same fractions against the peak at the graphics clock sampled
            # during the steps (the published peak assumes 2.4 GHz)
            "clock_mhz": clk,
            "frac_at_measured_clock": round(achieved / peak * 2400.0 / clk, 4) if clk else None,
            "mix_ceiling_frac_at_measured_clock":
                round(acc.mix_ceiling_seconds(units) / avg_s * 2400.0 / clk, 4) if clk else None}


def graph_roofline(param, res):
    """Roofline of a hipGraph replay.  The kernels inside a replayed graph
    are not timed one by one, so the whole step (prelude, FORS, TREE and
    WOTS+ kernels) is priced against its FORS and TREE work: a lower bound
    of the dominant kernel's fraction.  The same kernels timed one by one
    are in the eager row of the mode the graph replays."""
    from paper_2512_23969_amd import accounting as acc
    parts = ("fors", "tree")
    scale = {"tree": res["dedup"][1] / res["dedup"][0] if res.get("dedup") else 1.0}
    n = res["cfg"]["batch"]
    s = res["ms_per_step"] / 1e3
    ops = sum(acc.ops_per_signature(param, p, textbook=True) * scale.get(p, 1.0) for p in parts) * n
    isa = sum(acc.ops_per_signature(param, p) * scale.get(p, 1.0) for p in parts) * n
    c = acc.per_signature(param)
    units = {h: int(sum(c[h][p] * scale.get(p, 1.0) for p in parts) * n)
             for h in ("sha256", "sha512", "keccak") if sum(c[h].values())}
    peak = acc.VALU_PEAK_OPS / 1e12
    return {"bound": "alu", "kernel": "graph replay (whole step)", "achieved": round(ops / s / 1e12, 3),
            "peak": round(peak, 3), "unit": "TOP/s (32-bit VALU lane-ops)", "frac": round(ops / s / 1e12 / peak, 4),
            "traffic": None, "traffic_source": "a graph replay is not profiled kernel by kernel",
            "avg_launch_ms": round(res["ms_per_step"], 4), "units_per_launch": units,
            "isa_frac": round(isa / s / acc.VALU_PEAK_OPS, 4),
            "mix_ceiling_frac": round(acc.mix_ceiling_seconds(units) / s, 4),
            "single_rate_frac": round(isa / s / acc.VALU_SINGLE_RATE_OPS, 4)}


def phase_rooflines(param, res, msg_bytes=32):
    """Each timed phase against its bound: the hashing phases against the
    VALU issue rate (units x per-unit instructions), the WOTS+ gather against
    HBM bandwidth (bytes it must move).  The prelude runs one lane per
    message (latency-bound at batch 4096); its fraction shows that."""
    from paper_2512_23969_amd import accounting as acc
    c = acc.per_signature(param)
    peak_ops = acc.VALU_PEAK_OPS
    out = {}
    scale = {"tree": res["dedup"][1] / res["dedup"][0] if res.get("dedup") else 1.0}
    for ph, (ms, launches, msgs) in res["phases"].items():
        if not launches or ms <= 0:
            continue
        s = ms / 1e3
        if ph in ("fors", "tree", "fused"):
            parts = ("fors", "tree") if ph == "fused" else (ph,)
            ops = sum(acc.ops_per_signature(param, p) * scale.get(p, 1.0) for p in parts) * msgs
            units = {h: sum(c[h][p] * scale.get(p, 1.0) for p in parts) * msgs
                     for h in ("sha256", "sha512", "keccak")}
            out[ph] = {"bound": "alu", "achieved": round(ops / s / 1e12, 3), "unit": "TOP/s",
                       "frac": round(ops / s / peak_ops, 4),
                       "mix_ceiling_frac": round(acc.mix_ceiling_seconds(units) / s, 4)}
        elif ph == "prelude":
            ops = acc.prelude_ops(param, msg_bytes) * msgs
            out[ph] = {"bound": "alu (one lane per message)", "achieved": round(ops / s / 1e12, 4),
                       "unit": "TOP/s", "frac": round(ops / s / peak_ops, 5)}
        elif ph == "wots":
            b = acc.wots_gather_bytes(param) * msgs
            out[ph] = {"bound": "hbm", "achieved": round(b / s / 1e9, 1), "unit": "GB/s",
                       "frac": round(b / s / 8e12, 4)}
    return out


def summary(acc, r, mode):
    """The figures of one workload and mode for the line's "extra" object."""
    prm = r["cfg"]["param"]
    out = {"workload": r["name"], "value": round(r["sig_per_s"], 1), "unit": "signatures/s",
           "ms_per_step": round(r["ms_per_step"], 3), "steps": r["steps"], "mode": mode, "tuning": r["tuning"],
           "compressions_per_s": compressions_per_s(acc, prm, r["sig_per_s"]),
           "useful_valu_frac": round(r["sig_per_s"] * acc.ops_per_signature(prm, textbook=True)
                                     / acc.VALU_PEAK_OPS, 4),
           "roofline": roofline(prm, r) if "graph" not in mode else graph_roofline(prm, r),
           "phase_ms_per_step": {k: round(v[0] / r["steps"], 3) for k, v in r["phases"].items() if v[1]},
           "phase_roofline": phase_rooflines(prm, r), "step_ms": r["step_ms"],
           "gfx_clock_mhz": (r["gpu"]["gfx_clock_mhz"] or {}).get("mean"),
           "socket_power_w": (r["gpu"]["socket_power_w"] or {}).get("mean"),
           "energy": r["energy"]}
    if r["verify"]:
        out["verify"] = r["verify"]
    if r["dedup"]:
        trees, distinct = r["dedup"]
        out["dedup"] = {"trees_per_step": trees, "distinct_trees_per_step": distinct,
                        "tree_work_saved": round(1.0 - distinct / trees, 4),
                        "note": "identical signatures; work per signature below the paper's, "
                                "so not the headline value"}
    return out


def compressions_per_s(acc, param, sig_per_s):
    c256, c512 = acc.compressions_per_signature(param)
    return {"sha256": round(sig_per_s * c256, 0), "sha512": round(sig_per_s * c512, 0),
            "keccak_f": round(sig_per_s * acc.permutations_per_signature(param), 0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2_128f_4096", choices=sorted(WORKLOADS))
    ap.add_argument("--mode", default="config",
                    choices=["config", "auto", "plain", "fused", "graph", "graph-plain", "graph-any", "dedup",
                             "fused-dedup", "graph-dedup"],
                    help="execution mode; config = the mode the workload's configuration names (fused launch, "
                         "hipGraph pipeline), else the autotuned one; auto = the autotuner's fastest mode; "
                         "graph-any = the faster hipGraph pipeline (dedup modes: within-batch tree dedup)")
    ap.add_argument("--tune", action="store_true", help="run the autotuner first and store its result")
    ap.add_argument("--tune-out", default=None, help="tuning cache file (default: the package's tuning.json)")
    ap.add_argument("--only", action="store_true",
                    help="time the --workload alone (no 192f/256f/plain legs; profiler runs)")
    ap.add_argument("--all", action="store_true",
                    help="also time the small and SHAKE sets, the other modes and small-batch latency")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-n", type=int, default=100000, help="requests of the serving workload (0 = skip)")
    ap.add_argument("--serve-rates", default="0.25,0.5,0.75,0.9,1.0,1.2")
    ap.add_argument("--serve-mode", default="fused", choices=["plain", "fused", "dedup", "fused-dedup"])
    ap.add_argument("--serve-cache-layers", type=int, default=0,
                    help="upper hypertree layers cached per key on the server's lanes (dedup modes)")
    ap.add_argument("--serve-lanes", type=int, default=4, help="in-flight batches of the signing server")
    ap.add_argument("--serve-schedule", default="items", choices=["items", "chunks"],
                    help="fused kernel schedule of the server's batches (fused_schedule of the SHA2 fast sets)")
    ap.add_argument("--telemetry-s", type=float, default=2.0,
                    help="seconds of further untimed steps (after a 1 s settle) over which amdsmi reads the "
                         "clock, power and energy counter; 0 = none (profiler runs)")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="GPU_MAX_HW_QUEUES for this process (0 = keep the environment's). The serving leg "
                         "keeps 4 lanes x 4 streams busy; with 16 hardware queues none of them share one")
    ap.add_argument("--no-serve-dedup", action="store_true",
                    help="skip the second serving run (fused-dedup with 4 cached layers per key)")
    ap.add_argument("--knob", action="append", default=[], metavar="NAME=VALUE",
                    help="set one slh_tuning knob of the --workload over its tuned value (repeatable); "
                         "for profiling a kernel shape or instruction variant")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (calibrates HBM counters)")
    args = ap.parse_args()
    if args.hw_queues:
        # read by the HIP runtime when it initialises, which nothing has done yet
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, max(1, args.hw_queues)))
    if args.copy_calib:
        import torch
        src = torch.ones(args.copy_calib, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_calib, "launches": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: signing shards by message with no exchange, "
              "and the benchmark measures the single-GPU kernel (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    from paper_2512_23969_amd import accounting as acc
    from paper_2512_23969_amd import slh, workloads
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    mode0 = CONFIG_MODE.get(args.workload, "auto") if args.mode == "config" else args.mode
    log("bench: workload", args.workload, mode0)
    knobs = {}
    for kv in args.knob:
        k, _, v = kv.partition("=")
        if k not in slh.TUNING_FIELDS:
            ap.error("unknown knob %r (one of %s)" % (k, ", ".join(slh.TUNING_FIELDS)))
        knobs[k] = int(v)
    res = run(slh, workloads, args.workload, args.steps, args.warmup, mode0, args.tune, args.tune_out,
              verify=True, telemetry_s=args.telemetry_s, knobs=knobs)
    param = res["cfg"]["param"]
    line = {
        "metric": METRIC,
        "value": round(res["sig_per_s"], 1),
        "unit": "signatures/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "step_ms": res["step_ms"],
        "gpu_telemetry": res["gpu"],
        "energy": res["energy"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded random keys and 32-byte messages)",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload],
                   "parameter_set": "SPHINCS+-" + acc.full_name(param),
                   "batch": res["cfg"]["batch"], "keys": res["cfg"]["keys"], "msg_bytes": 32,
                   "mode": res["mode"], "tuning": res["tuning"],
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
        "compressions_per_s": compressions_per_s(acc, param, res["sig_per_s"]),
        "useful_valu_frac": round(res["sig_per_s"] * acc.ops_per_signature(param, textbook=True)
                                  / acc.VALU_PEAK_OPS, 4),
        "phase_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in res["phases"].items() if v[1]},
        "roofline": roofline(param, res) if "graph" not in res["mode"] else graph_roofline(param, res),
        "phase_roofline": phase_rooflines(param, res),
        "verify": res["verify"],
    }
    if res["dedup"]:
        line["dedup"] = {"trees_per_step": res["dedup"][0], "distinct_trees_per_step": res["dedup"][1]}
    extra = {}
    steps_c = max(3, args.steps // 2)
    if not args.only:
        # every batch-4096 SHA2 fast-set workload in the execution mode its
        # configuration names (with that mode's tuned knobs) and in the plain
        # per-phase path, the reference the batched modes are measured against
        from paper_2512_23969_amd import autotune
        for name in DEFAULT_WORKLOADS:
            cfg = workloads.CONFIGS[name]
            cmode, _ = autotune.resolve_mode(cfg["param"], cfg["batch"], CONFIG_MODE[name])
            got = {}
            # a fused graph's kernels are timed in an eager fused run beside it
            for mode in dict.fromkeys((cmode, "plain") + (("fused",) if cmode == "graph" else ())):
                if name == args.workload and mode == res["mode"]:
                    got[mode] = summary(acc, res, mode)
                    continue
                log("bench: workload", name, mode)
                r = run(slh, workloads, name, steps_c, args.warmup, mode, verify=True, telemetry_s=args.telemetry_s)
                got[mode] = summary(acc, r, mode)
            for mode, v in got.items():
                extra["%s/%s" % (name, mode)] = v
            if cmode != "plain":
                extra["%s/config_vs_plain" % name] = {
                    "config_mode": cmode, "ratio": round(got[cmode]["value"] / got["plain"]["value"], 4)}
                if "graph" in cmode:
                    # a graph replays the same kernels; their per-kernel figures
                    # are those of the eager run of the same knobs
                    base = "plain" if cmode == "graph-plain" else "fused"
                    extra["%s/%s" % (name, cmode)]["roofline_of_kernels"] = "%s/%s" % (name, base)
    if args.all:
        log("bench: small-batch latency")
        line["latency"] = latency_bench(slh, workloads)
        # the other modes of the batch-4096 workloads (hipGraph-captured
        # pipeline, tree dedup), the small sets at batch 1024 and the SHAKE sets
        for name in ("c2_128f_4096", "c3_192f_4096", "c4_256f_4096x64", "s1_128s_1024", "s2_192s_1024",
                     "s3_256s_1024", "k1_shake128f_4096", "k2_shake192f_4096", "k3_shake256f_4096x64",
                     "k4_shake128s_1024"):
            if name.startswith("s") or name.startswith("k4"):
                modes = ("plain",)  # the small sets take the per-phase path in every mode
            elif name.startswith("k"):
                modes = ("plain", "fused", "dedup")
            else:
                modes = ("fused", "graph", "dedup", "fused-dedup")
            for mode in modes:
                key = "%s/%s" % (name, mode)
                if key in extra or (name == args.workload and mode == res["mode"]):
                    continue
                log("bench: workload", name, mode)
                r = run(slh, workloads, name, steps_c, args.warmup, mode,
                        args.tune and mode == "plain" and name != args.workload, args.tune_out,
                        verify=mode == "plain", telemetry_s=args.telemetry_s)
                extra[key] = summary(acc, r, mode)
    if extra:
        line["extra"] = extra
    if args.serve_n:
        log("bench: serving")
        rates = [float(x) for x in args.serve_rates.split(",")]
        line["serving"] = serve_bench(slh, workloads, args.serve_n, rates, log, args.serve_mode,
                                      args.serve_cache_layers, args.serve_lanes, args.serve_schedule)
        if not args.no_serve_dedup:
            # tree sharing across the requests of a key (within-batch dedup and
            # a per-key cache of the top layers): same bytes, less work
            log("bench: serving with dedup and key cache")
            line["serving_dedup_cache"] = serve_bench(slh, workloads, args.serve_n, rates, log, "fused-dedup", 4,
                                                      args.serve_lanes, args.serve_schedule)
    if not args.no_cpu:
        log("bench: cpu baseline")
        line["cpu_baseline"] = cpu_baseline(args.workload, workloads, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
