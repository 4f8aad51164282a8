"""Autotuner of the signing kernels.

Two stages, as in the paper's Section III-B ("Fusion Trade-offs in FORS"):
an analytic search proposes candidate FORS groupings, then the candidates
are timed on the GPU and the fastest is kept.

* ``fors_fusion_search(...)`` states the paper's FORS-fusion trade-off
  (Section III-B, its Algorithm 1) as a search over block layouts: trees
  per block and sets fused through shared memory, constrained by the
  block's threads and shared memory, ranked by barrier count and then
  resource use.  With the RTX 4090's 48 KiB static shared memory it gives
  the paper's Table 4.
* ``gfx950_groups(param)`` re-expresses the same trade-off for this
  library's FORS kernels, whose unit is a group of trees reduced by one
  256-lane workgroup with two leaves per lane: the LDS per group must fit the
  160 KiB of a CU, and the groups are ranked by barrier count per message.
* ``tune(...)`` times the compiled variants on a real batch, kernel by
  kernel (the FORS shape and instruction variant from the FORS kernel's own
  HIP events; TREE block size, layer order, kept or recomputed chains and
  the TREE instruction variant from whole steps; then the per-phase path
  against the fused persistent kernel in both of its schedules (fixed chunk
  shares per work item, or chunks taken one at a time); then the
  verification kernel's variant) and keeps the fastest; results are cached
  in a JSON file keyed by GPU architecture, parameter set and batch size.
"""
from __future__ import annotations

import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning.json")

# (n, a = log t, k) of the parameter sets (the paper's Table 1)
FORS_SHAPE = {1: (16, 6, 33), 2: (24, 8, 33), 3: (32, 9, 35), 4: (16, 12, 14), 5: (24, 14, 17), 6: (32, 14, 22)}
FORS_SHAPE.update({p + 6: s for p, s in list(FORS_SHAPE.items())})  # SHAKE sets: same shapes


def fors_fusion_search(k: int, log_t: int, n: int, smem_bytes: int, max_threads: int = 1024,
                       alpha: float = 0.6):
    """The FORS-fusion trade-off of the paper's Section III-B for a GPU with
    `smem_bytes` of shared memory and `max_threads` threads per block.

    A block gives one thread to every leaf of `trees` whole FORS trees (2^a
    leaves each) and fuses `fusion` such sets through its shared memory (one
    n-byte node per leaf and set).  The k trees of a signature then take
    ceil(k / trees) / fusion rounds of a level barriers each.  A layout is
    feasible when its threads and fused node buffers fit the block, it
    keeps at least `alpha` of the threads busy, and it does not fill both
    resources exactly.  The best layout has the fewest barriers, then the
    highest thread use, then the highest shared-memory use.  The paper
    leaves alpha unstated; any alpha in (0.5, 0.6875] gives its Table 4 for
    the RTX 4090's 48 KiB of static shared memory.

    Returns (best, feasible); each layout is a dict with trees, fusion,
    threads, smem, thread_use, smem_use and barriers (None, [] if nothing
    is feasible)."""
    leaves = 1 << log_t

    def layout(trees, fusion):
        threads, smem = trees * leaves, fusion * trees * leaves * n
        return {"trees": trees, "fusion": fusion, "threads": threads, "smem": smem,
                "thread_use": threads / max_threads, "smem_use": smem / smem_bytes,
                "barriers": log_t * math.ceil(k / trees) / fusion}

    def feasible(c):
        full = c["thread_use"] == 1 and c["smem_use"] == 1
        return c["smem"] <= smem_bytes and c["thread_use"] >= alpha and not full

    # at most k trees per block, and no more fused sets than the k trees fill
    shapes = [(t, f) for t in range(1, min(k, max_threads // leaves) + 1) for f in range(1, k // t + 1)]
    options = [c for c in (layout(t, f) for t, f in shapes) if feasible(c)]
    if not options:
        return None, []
    best = min(options, key=lambda c: (c["barriers"], -c["thread_use"], -c["smem_use"]))
    return best, options


COMPILED_GROUPS = {1: (4, 8, 16), 2: (4, 8, 16), 3: (2, 4, 8), 4: (1, 2), 5: (1, 2), 6: (1, 2)}
COMPILED_GROUPS.update({p + 6: g for p, g in list(COMPILED_GROUPS.items())})


def gfx950_groups(param: int, lds_bytes: int = 160 * 1024, lanes: int = 256, compiled=None):
    """FORS groupings of this library ranked analytically for gfx950.

    A group of FG units (a unit is a FORS tree, or for trees above 2^12
    leaves a subtree of 2^12 leaves) keeps FG * 2^(au-1) level-1 nodes of n
    bytes in LDS and is reduced by one workgroup of `lanes` lanes.  Returns
    a list of dicts sorted by (barriers per message, idle lanes in the pair
    phase)."""
    n, a, k = FORS_SHAPE[param]
    au = min(a, 12)
    units = k << (a - au)  # units per message
    out = []
    for fg in compiled or COMPILED_GROUPS[param]:
        lds = fg * (1 << (au - 1)) * n
        if lds > lds_bytes:
            continue
        pairs = fg * (1 << (au - 1))
        rounds = math.ceil(pairs / lanes)
        idle = rounds * lanes - pairs
        groups_per_msg = units / fg
        barriers = groups_per_msg * au  # one per level of every group
        out.append({"fg": fg, "lds_bytes": lds, "pair_rounds": rounds, "idle_lanes": idle,
                    "barriers_per_msg": barriers, "wgs_per_cu_lds": lds_bytes // max(1, lds)})
    out.sort(key=lambda c: (c["barriers_per_msg"], c["idle_lanes"]))
    return out


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def cache_key(arch: str, param: int, batch: int) -> str:
    # batches are bucketed by powers of two
    b = 1 << max(0, int(math.ceil(math.log2(max(1, batch)))))
    return "%s/%d/%d" % (arch, param, b)


def lookup(param: int, batch: int, path: str = DEFAULT_CACHE):
    """Tuned setting for (this GPU, param, batch) or None."""
    c = load_cache(path)
    return c.get(cache_key(_arch(), param, batch))


def best_for(param: int, batch: int, mode: str | None = None, path: str = DEFAULT_CACHE):
    """The tuned knobs of the fastest mode (mode None) or of `mode` (plain,
    fused, graph-plain, graph) for (this GPU, param, batch), or None."""
    e = lookup(param, batch, path)
    if not e:
        return None
    b = e.get("best")
    if mode is None or (b and b.get("mode") == mode):
        return b
    return (b or {}).get("by_mode", {}).get(mode)


def resolve_mode(param: int, batch: int, mode: str, path: str = DEFAULT_CACHE):
    """(mode, tuned knobs) for a requested mode: "auto" = the fastest tuned
    mode, "graph-any" = the faster of the two hipGraph pipelines, else the
    mode itself with the knobs tuned for it (or the fastest mode's knobs)."""
    if mode == "auto":
        b = best_for(param, batch, None, path)
        return (b or {}).get("mode", "plain"), b
    if mode == "graph-any":
        g = [best_for(param, batch, m, path) for m in ("graph-plain", "graph")]
        g = [x for x in g if x]
        if not g:
            return "graph", best_for(param, batch, None, path)
        b = min(g, key=lambda x: x["ms"])
        return b["mode"], b
    return mode, best_for(param, batch, mode, path) or best_for(param, batch, None, path)


# Knobs the empirical stage searches, per parameter-set family (slh.h
# slh_tuning): fast sets have every FORS and TREE shape and both layer
# orders; the SHA2 fast sets also the instruction variants; the small sets
# only the FORS group size and keep_chains.
LPLS = (2, 4)
FORS_THREADS = (128, 256, 512)
TREE_WAVES = (2, 4, 8)
VARIANTS = (1, 2)  # SLH_VARIANT_NO_BITOP3, SLH_VARIANT_SPLIT_ADDS (0 is the default)
WGS_PER_CU = (0, 1, 2, 3)
KNOB_DEFAULTS = {"fors_trees_per_group": 0, "wgs_per_cu": 0, "keep_chains": 1, "split_max_blocks": 0,
                 "fors_leaves_per_lane": 2, "fors_threads": 256, "tree_waves": 4, "layer_order": 0,
                 "variant_tree": 0, "variant_fors": 0, "variant_verify": 0, "fused_wave0_chunks": 0,
                 "fused_waves": 4, "fused_blocks_per_item": 1, "fused_schedule": 1}
# default chains chunks of wave 0 in a fused TREE block, by waves per
# workgroup and len (35 / 51 / 67)
FUSED_W0 = {4: {35: 8, 51: 11, 67: 14}, 2: {35: 17, 51: 24, 67: 31}}
FUSED_WAVES = (4, 2)
FUSED_CHUNKS = 2  # fused_schedule: SLH_FUSED_CHUNKS


def _fast(param):
    return (param - 1) % 6 < 3


def _sha2_fast(param):
    return param <= 3


def _median(v):
    v = sorted(v)
    return v[len(v) // 2]


def _events_ms(torch, stream, run, reps):
    """Median and minimum over `reps` calls of run() of the GPU time between
    HIP events recorded on `stream` around each call (after one warm-up)."""
    run()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        run()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    t = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
    return _median(t), min(t)


def _phase_ms(slh, ctx, run, phases, reps):
    """Median over `reps` calls of the summed GPU time of `phases` (the
    library's per-kernel HIP events), after one warm-up."""
    import torch
    run()
    torch.cuda.synchronize()
    ctx.phase_times(reset=True)
    ctx.profile(True)
    per = []
    for _ in range(reps):
        run()
        pt = ctx.phase_times(reset=True)
        per.append(sum(pt[p][0] for p in phases))
    ctx.profile(False)
    return _median(per), min(per)


def tune(slh, ctx, param: int, items, d_msgs, d_sigs, reps: int = 7, log=None, verify=None):
    """Time the compiled variants on this batch, one kernel at a time as the
    paper does (its per-kernel choice of code, Section III-C), then the
    execution mode; returns (best, stages).

      1. FORS kernel (per-phase path, its own HIP events): trees per group x
         leaves per lane x workgroup lanes, and the instruction variants;
      2. TREE and WOTS+ (whole step, HIP events): block waves x layer order
         (parallel with kept or recomputed chains, or in order), and the
         instruction variants;
      3. mode: the per-phase path with the winners of 1-2 against the fused
         persistent kernel (trees per group x leaves per lane at 4 and 2
         waves per workgroup, then 1 or 2 TREE blocks per work item, then
         persistent workgroups per CU x
         keep_chains, then wave 0's share of a TREE block around the
         default), and each mode's winner captured in a hipGraph;
      4. verification (if `verify` = (items, msgs, sigs, pks, results) is
         given): the instruction variants of the verify kernel.
    Every point is the median of `reps` timed runs after a warm-up."""
    import torch
    stream = torch.cuda.current_stream()
    stages = {"fors": [], "tree": [], "mode": [], "verify": []}

    def knobs(**kw):
        k = dict(KNOB_DEFAULTS)
        k.update(kw)
        return k

    def setk(k):
        ctx.set_tuning(param, **{f: v for f, v in k.items() if f in KNOB_DEFAULTS})

    def say(stage, row):
        stages[stage].append(row)
        if log:
            log("tune %s %s %s" % (param, stage, row))

    def sign(mode):
        return lambda: ctx.sign_batch(items, d_msgs, d_sigs, mode=slh.MODES[mode], stream=stream)

    # 1. FORS
    fors = []
    for fg in slh.FORS_GROUPS[param]:
        shapes = [(l, t, 0) for l in LPLS for t in FORS_THREADS] if _fast(param) else [(2, 256, 0)]
        if _sha2_fast(param):
            shapes += [(2, 256, v) for v in VARIANTS]
        for lpl, ft, var in shapes:
            k = knobs(fors_trees_per_group=fg, fors_leaves_per_lane=lpl, fors_threads=ft, variant_fors=var)
            setk(k)
            med, mn = _phase_ms(slh, ctx, sign("plain"), ("fors",), reps)
            row = dict(k, ms=round(med, 4), min_ms=round(mn, 4))
            say("fors", row)
            fors.append(row)
    fb = min(fors, key=lambda r: r["ms"])
    base = knobs(**{f: fb[f] for f in ("fors_trees_per_group", "fors_leaves_per_lane", "fors_threads",
                                        "variant_fors")})
    # 2. TREE and WOTS+ (layer order, keep, block waves, variants)
    tree = []
    orders = [(0, 1), (0, 0), (1, 0)] if _fast(param) else [(0, 1), (0, 0)]
    for order, keep in orders:
        for waves in (TREE_WAVES if _fast(param) else (4,)):
            for var in (0,) + (VARIANTS if _sha2_fast(param) and waves == 4 else ()):
                k = dict(base, layer_order=order, keep_chains=keep, tree_waves=waves, variant_tree=var)
                setk(k)
                med, mn = _events_ms(torch, stream, sign("plain"), reps)
                row = dict(k, mode="plain", ms=round(med, 4), min_ms=round(mn, 4))
                say("tree", row)
                tree.append(row)
    best = min(tree, key=lambda r: r["ms"])
    say("mode", dict(best))
    # 3. the fused persistent kernel (parallel layers): its FORS shape at each
    # workgroup size, then persistent workgroups per CU and kept chains, then
    # wave 0's share of a TREE block around the default
    if _fast(param):
        fused = []

        def time_fused(k):
            setk(k)
            med, mn = _events_ms(torch, stream, sign("fused"), reps)
            row = dict(k, mode="fused", ms=round(med, 4), min_ms=round(mn, 4))
            say("mode", row)
            fused.append(row)
            return row

        for nw in FUSED_WAVES:
            for fg in slh.FORS_GROUPS[param]:
                for lpl in LPLS:
                    time_fused(knobs(fors_trees_per_group=fg, fors_leaves_per_lane=lpl, fused_waves=nw))
        fb = min(fused, key=lambda r: r["ms"])
        time_fused(dict(fb, fused_blocks_per_item=2))
        fb = min(fused, key=lambda r: r["ms"])
        per = 4 // fb["fused_waves"]  # workgroups of this size per four-wave workgroup
        for wpc in WGS_PER_CU:
            for keep in (1, 0):
                if (wpc, keep) != (0, 1):
                    time_fused(dict(fb, wgs_per_cu=wpc * per, keep_chains=keep))
        fb = min(fused, key=lambda r: r["ms"])
        w0d = FUSED_W0[fb["fused_waves"]][slh.sizes(param)["len"]] * fb["fused_blocks_per_item"]
        for w0 in (w0d - 2, w0d - 1, w0d + 1, w0d + 2):
            time_fused(dict(fb, fused_wave0_chunks=w0))
        # the kernel scheduled per chains chunk (no barrier per item): its
        # FORS shape, then persistent workgroups per CU and kept chains
        chunks = [time_fused(knobs(fors_trees_per_group=fg, fors_leaves_per_lane=lpl, fused_schedule=FUSED_CHUNKS))
                  for fg in slh.FORS_GROUPS[param] for lpl in LPLS]
        cb = min(chunks, key=lambda r: r["ms"])
        for wpc in WGS_PER_CU:
            for keep in (1, 0):
                if (wpc, keep) != (0, 1):
                    time_fused(dict(cb, wgs_per_cu=wpc, keep_chains=keep))
        fb = min(fused, key=lambda r: r["ms"])
        if fb["ms"] < best["ms"]:
            best = fb
    # the hipGraph-captured pipeline of each mode's best knobs
    by_mode = {}
    for r in stages["mode"]:
        if r["mode"] not in by_mode or r["ms"] < by_mode[r["mode"]]["ms"]:
            by_mode[r["mode"]] = dict(r)
    for base_mode, graph_mode in (("plain", "graph-plain"), ("fused", "graph")):
        if base_mode not in by_mode:
            continue
        k = dict(by_mode[base_mode])
        setk(k)
        med, mn = _events_ms(torch, stream, sign(graph_mode), reps)
        row = dict(k, mode=graph_mode, ms=round(med, 4), min_ms=round(mn, 4))
        say("mode", row)
        by_mode[graph_mode] = row
        if row["ms"] < best["ms"]:
            best = row
    # 4. verification
    best = dict(best)
    if verify is not None:
        vitems, vm, vs, vpk, vres = verify
        vbest = None
        for var in ((0,) + VARIANTS if _sha2_fast(param) else (0,)):
            setk(knobs(variant_verify=var))
            med, mn = _events_ms(torch, stream, lambda: ctx.verify_batch(vitems, vm, vs, vpk, vres, stream=stream),
                                 reps)
            row = {"variant_verify": var, "ms": round(med, 4), "min_ms": round(mn, 4)}
            say("verify", row)
            if vbest is None or row["ms"] < vbest["ms"]:
                vbest = row
        best["variant_verify"] = vbest["variant_verify"]
        for r in by_mode.values():
            r["variant_verify"] = vbest["variant_verify"]
    apply(ctx, param, best)
    best["by_mode"] = by_mode
    return best, stages


def tune_and_store(slh, ctx, param, items, d_msgs, d_sigs, batch, path: str = DEFAULT_CACHE, log=None,
                   verify=None, reps: int = 7):
    best, stages = tune(slh, ctx, param, items, d_msgs, d_sigs, reps=reps, log=log, verify=verify)
    c = load_cache(path)
    c[cache_key(_arch(), param, batch)] = {
        "best": best, "stages": stages, "analytic": gfx950_groups(param),
        "timing": "median of %d runs after a warm-up: HIP events around each call on the signing stream "
                  "(the FORS stage: the library's events around the FORS kernel)" % reps}
    with open(path, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    return best, stages


def apply(ctx, param: int, setting: dict):
    """Set the tuned knobs (a row of the tuner's tables) on a context;
    returns its mode name."""
    ctx.set_tuning(param, **{f: setting.get(f, v) for f, v in KNOB_DEFAULTS.items()})
    return setting.get("mode", "plain")
