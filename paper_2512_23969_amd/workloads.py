"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds input generation only (random bytes, key seeds, request
mixes); none of the signature arithmetic.  Both the GPU path and the oracle
consume what it produces.

The paper signs random messages of a fixed length with one key per run; its
evaluation names no dataset (Section V: a batch of messages per launch,
input length 1K-4K bytes in the input-size study).  The recipes below follow
that shape: uniform random bytes, 32-byte messages for the throughput
configurations, log-normal lengths for the serving mix.
"""
from __future__ import annotations

import numpy as np

# parameter-set id -> security parameter n in bytes (the paper's Table 1)
N_OF = {1: 16, 2: 24, 3: 32, 4: 16, 5: 24, 6: 32, 7: 16, 8: 24, 9: 32, 10: 16, 11: 24, 12: 32}
NAME_OF = {1: "128f", 2: "192f", 3: "256f", 4: "128s", 5: "192s", 6: "256s",
           7: "shake-128f", 8: "shake-192f", 9: "shake-256f", 10: "shake-128s", 11: "shake-192s",
           12: "shake-256s"}
ID_OF = {v: k for k, v in NAME_OF.items()}


def key_seed(param: int, i: int) -> bytes:
    """3n-byte seed SK.seed | SK.prf | PK.seed of key i of a parameter set."""
    return np.random.default_rng([param, i, 0x5EED]).bytes(3 * N_OF[param])


def messages(cfg: int, count: int, length: int = 32) -> list[bytes]:
    """count uniform random messages of a fixed length for configuration cfg."""
    rng = np.random.default_rng([cfg, 1])
    return [rng.bytes(length) for _ in range(count)]


def sample_indices(cfg: int, count: int, nsample: int) -> list[int]:
    """Sorted distinct indices to check at full size (first and last included)."""
    rng = np.random.default_rng([cfg, 2])
    pick = set(int(x) for x in rng.choice(count, size=min(nsample, count), replace=False))
    pick.update({0, count - 1})
    return sorted(pick)


def key_assignment(cfg: int, count: int, nkeys: int) -> list[int]:
    """Key index per message, uniform over nkeys."""
    rng = np.random.default_rng([cfg, 3])
    return [int(x) for x in rng.integers(0, nkeys, size=count)]


# Workload configurations (name, parameter set, batch, keys, message length)
CONFIGS = {
    "c1_128f_16": dict(cfg=1, param=1, batch=16, keys=1, length=32),
    # `mode`: how the benchmark signs the batch ("graph-any" = the faster of
    # the two hipGraph pipelines; a workload without one runs the fastest
    # tuned mode)
    "c2_128f_4096": dict(cfg=2, param=1, batch=4096, keys=1, length=32, mode="fused"),
    "c3_192f_4096": dict(cfg=3, param=2, batch=4096, keys=1, length=32, mode="graph-any"),
    "c4_256f_4096x64": dict(cfg=4, param=3, batch=4096, keys=64, length=32, mode="fused"),
    # the small sets (not in the paper): one key, 1024 x 32-byte messages
    "s1_128s_1024": dict(cfg=11, param=4, batch=1024, keys=1, length=32),
    "s2_192s_1024": dict(cfg=12, param=5, batch=1024, keys=1, length=32),
    "s3_256s_1024": dict(cfg=13, param=6, batch=1024, keys=1, length=32),
    # the SHAKE256 instantiation of the same shapes (not in the paper)
    "k1_shake128f_4096": dict(cfg=21, param=7, batch=4096, keys=1, length=32),
    "k2_shake192f_4096": dict(cfg=22, param=8, batch=4096, keys=1, length=32),
    "k3_shake256f_4096x64": dict(cfg=23, param=9, batch=4096, keys=64, length=32),
    "k4_shake128s_1024": dict(cfg=24, param=10, batch=1024, keys=1, length=32),
}


def serving_requests(count: int, seed: int = 5, keys_per_set=(128, 77, 51)):
    """Request mix of the serving workload.

    Parameter set 128f/192f/256f with probability 0.5/0.3/0.2; key uniform
    among the set's resident keys; message length log-normal with median
    256 B, clipped to [32, 16384]; random bytes.
    Returns a list of (param, key_index_within_set, message bytes).
    """
    rng = np.random.default_rng([seed, 7])
    params = rng.choice([1, 2, 3], size=count, p=[0.5, 0.3, 0.2])
    lens = np.clip(np.rint(np.exp(rng.normal(np.log(256.0), 1.386, size=count))), 32, 16384)
    out = []
    for prm, ln in zip(params, lens):
        kidx = int(rng.integers(0, keys_per_set[int(prm) - 1]))
        out.append((int(prm), kidx, rng.bytes(int(ln))))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 11) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng([seed, 13])
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
