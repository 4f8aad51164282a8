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
* ``tune(...)`` times every compiled variant (execution mode, FORS trees per
  group, persistent workgroups per CU) on a real batch and returns the
  fastest; results are cached in a JSON file keyed by GPU architecture,
  parameter set and batch size.
"""
from __future__ import annotations

import json
import math
import os
import time

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


def tune(slh, ctx, param: int, items, d_msgs, d_sigs, reps: int = 3, modes=("plain", "fused"),
         wgs=(0, 1, 2, 3), log=None):
    """Time every compiled variant on this batch; returns (best, table)."""
    import torch
    table = []
    for mode in modes:
        for fg in slh.FORS_GROUPS[param]:
            for wpc in (wgs if mode == "fused" else (0,)):
                ctx.set_tuning(param, fg, wpc, 1)
                m = slh.MODES[mode]
                ctx.sign_batch(items, d_msgs, d_sigs, mode=m)  # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    ctx.sign_batch(items, d_msgs, d_sigs, mode=m)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1000.0 / reps
                row = {"mode": mode, "fors_trees_per_group": fg, "wgs_per_cu": wpc, "keep_chains": 1,
                       "ms": round(ms, 4)}
                table.append(row)
                if log:
                    log("tune %s %s" % (param, row))
    best = min(table, key=lambda r: r["ms"])
    return best, table


def tune_and_store(slh, ctx, param, items, d_msgs, d_sigs, batch, path: str = DEFAULT_CACHE, log=None):
    best, table = tune(slh, ctx, param, items, d_msgs, d_sigs, log=log)
    c = load_cache(path)
    c[cache_key(_arch(), param, batch)] = {"best": best, "table": table,
                                            "analytic": gfx950_groups(param)}
    with open(path, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    return best, table


def apply(ctx, param: int, setting: dict):
    """Set the tuned knobs on a context; returns the tuned mode name."""
    ctx.set_tuning(param, setting["fors_trees_per_group"], setting["wgs_per_cu"], setting["keep_chains"])
    return setting["mode"]
