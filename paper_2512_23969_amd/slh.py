"""Python binding of the C ABI in ``include/slh.h`` (argument marshalling only).

Every hash of the signing path runs in the HIP kernels of ``libslh.so``.
PyTorch supplies device memory and streams.  If the shared library is not
built, importing this module raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslh.so")

SHA2_128F, SHA2_192F, SHA2_256F = 1, 2, 3
NAMES = {1: "128f", 2: "192f", 3: "256f", 4: "128s", 5: "192s", 6: "256s",
         7: "shake-128f", 8: "shake-192f", 9: "shake-256f", 10: "shake-128s", 11: "shake-192s",
         12: "shake-256s"}
IDS = {v: k for k, v in NAMES.items()}
MODE_PLAIN, MODE_FUSED, MODE_GRAPH, MODE_DEDUP = 0, 1, 2, 4
MODES = {"plain": MODE_PLAIN, "fused": MODE_FUSED, "graph": MODE_GRAPH | MODE_FUSED,
         "graph-plain": MODE_GRAPH, "dedup": MODE_DEDUP, "fused-dedup": MODE_FUSED | MODE_DEDUP,
         "graph-dedup": MODE_GRAPH | MODE_FUSED | MODE_DEDUP}

OK, EINVAL, ENOMEM, EDEVICE, EBUSY = 0, -1, -2, -3, -4
PHASES = ("prelude", "fors", "tree", "wots", "fused")
# compiled FORS group sizes per parameter set
FORS_GROUPS = {1: (4, 8, 16), 2: (4, 8, 16), 3: (2, 4, 8), 4: (1, 2), 5: (1, 2), 6: (1, 2)}
FORS_GROUPS.update({p + 6: g for p, g in list(FORS_GROUPS.items())})  # SHAKE: same shapes

ITEM_DTYPE = np.dtype([("param", "<u4"), ("key_slot", "<u4"), ("msg_off", "<u8"),
                       ("msg_len", "<u8"), ("sig_off", "<u8")])
assert ITEM_DTYPE.itemsize == 32


class SlhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("slh error %d: %s" % (code, msg))
        self.code = code


class slh_tuning(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in
                ("fors_trees_per_group", "wgs_per_cu", "keep_chains", "split_max_blocks", "fors_leaves_per_lane",
                 "fors_threads", "tree_waves", "layer_order", "variant_tree", "variant_fors", "variant_verify",
                 "fused_wave0_chunks", "fused_waves", "fused_blocks_per_item", "fused_schedule")]


TUNING_FIELDS = tuple(f for f, _ in slh_tuning._fields_)
LAYERS_PARALLEL, LAYERS_IN_ORDER = 0, 1
FUSED_ITEMS, FUSED_CHUNKS = 1, 2
VARIANT_DEFAULT, VARIANT_NO_BITOP3, VARIANT_SPLIT_ADDS = 0, 1, 2
VARIANTS = {VARIANT_DEFAULT: "default", VARIANT_NO_BITOP3: "no-bitop3", VARIANT_SPLIT_ADDS: "split-adds"}


def make_tuning(fors_trees_per_group=0, wgs_per_cu=0, keep_chains=1, split_max_blocks=0, **knobs):
    """An slh_tuning from keyword knobs (the fields of slh.h; 0 = default)."""
    t = slh_tuning(fors_trees_per_group, wgs_per_cu, keep_chains, split_max_blocks)
    for k, v in knobs.items():
        if k not in TUNING_FIELDS:
            raise TypeError("unknown tuning knob %r" % k)
        setattr(t, k, int(v))
    return t


class slh_serve_config(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("min_batch", ctypes.c_uint32),
                ("max_wait_us", ctypes.c_uint32), ("msg_bytes", ctypes.c_uint64), ("hbm_budget", ctypes.c_uint64),
                ("mode", ctypes.c_uint32), ("queue_limit", ctypes.c_uint32), ("cache_layers", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class slh_serve_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("launches", ctypes.c_uint64), ("wall_s", ctypes.c_double),
                ("sig_per_s", ctypes.c_double), ("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double),
                ("mean_s", ctypes.c_double), ("max_s", ctypes.c_double), ("mean_batch", ctypes.c_double)]


# slh_item_ext: the external interface (pure / pre-hash, context string, hedged)
ITEM_EXT_DTYPE = np.dtype([("param", "<u4"), ("key_slot", "<u4"), ("msg_off", "<u8"), ("msg_len", "<u8"),
                           ("sig_off", "<u8"), ("ctx_off", "<u8"), ("rnd_off", "<u8"), ("ctx_len", "<u4"),
                           ("prehash", "<u4")])
assert ITEM_EXT_DTYPE.itemsize == 56
RND_NONE = 0xFFFFFFFFFFFFFFFF
SPLIT_NEVER = 0xFFFFFFFF  # slh_tuning.split_max_blocks: never split small batches
PREHASH_NONE, PREHASH_SHA256, PREHASH_SHA512 = 0, 1, 2

VERIFY_DTYPE = np.dtype([("param", "<u4"), ("pad", "<u4"), ("msg_off", "<u8"), ("msg_len", "<u8"),
                         ("sig_off", "<u8"), ("pk_off", "<u8")])
assert VERIFY_DTYPE.itemsize == 40
VERIFY_EXT_DTYPE = np.dtype([("param", "<u4"), ("prehash", "<u4"), ("msg_off", "<u8"), ("msg_len", "<u8"),
                             ("sig_off", "<u8"), ("pk_off", "<u8"), ("ctx_off", "<u8"), ("ctx_len", "<u4"),
                             ("pad", "<u4")])
assert VERIFY_EXT_DTYPE.itemsize == 56

REQ_DTYPE = np.dtype([("param", "<u4"), ("key_slot", "<u4"), ("msg_off", "<u8"), ("msg_len", "<u8"),
                      ("sig_off", "<u8"), ("arrival_s", "<f8")])
assert REQ_DTYPE.itemsize == 40
MAX_SIG_BYTES = 49856
# slh_sign_batch_noalloc: requests per call and the per-GPU working array
NOALLOC_MAX_ITEMS = 4096
NOALLOC_SCRATCH_BYTES = 256 << 20


class slh_sizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint32) for f in
                ("n", "h", "d", "hp", "a", "k", "len", "m", "seed_bytes", "pk_bytes", "sk_bytes",
                 "sig_bytes")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libslh.so is not built; run python -m paper_2512_23969_amd.build")
    # torch carries its own copy of the HIP runtime (same soname).  Loading
    # torch first makes libslh.so bind to that copy, so the process has one
    # HIP runtime; the other order would load two and the second sees no GPU.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t
    L.slh_params.argtypes = [u32, ctypes.POINTER(slh_sizes)]
    L.slh_ctx_create.argtypes = [ctypes.c_int, u64, ctypes.POINTER(vp)]
    L.slh_ctx_destroy.argtypes = [vp]
    L.slh_last_error.argtypes = [vp]
    L.slh_last_error.restype = ctypes.c_char_p
    L.slh_keygen.argtypes = [u32, ctypes.c_char_p, vp, vp]
    L.slh_ctx_add_keys.argtypes = [vp, u32, ctypes.c_char_p, u32, ctypes.POINTER(u32)]
    L.slh_sign_batch.argtypes = [vp, vp, u32, vp, u64, vp, u64, u32, vp]
    L.slh_sign_batch_noalloc.argtypes = [vp, vp, u32, vp, u64, vp, u64, u32, vp]
    L.slh_verify.argtypes = [u32, ctypes.c_char_p, sz, ctypes.c_char_p, sz, ctypes.c_char_p]
    L.slh_ctx_profile.argtypes = [vp, ctypes.c_int]
    L.slh_ctx_set_tuning.argtypes = [vp, u32, ctypes.POINTER(slh_tuning)]
    L.slh_ctx_get_tuning.argtypes = [vp, u32, ctypes.POINTER(slh_tuning)]
    L.slh_ctx_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                      ctypes.POINTER(u64), ctypes.c_int]
    L.slh_verify_batch.argtypes = [vp, vp, u32, vp, u64, vp, u64, vp, u64, vp, vp]
    L.slh_ctx_dedup_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.c_int]
    L.slh_ctx_cache_keys.argtypes = [vp, u32, u32, u32]
    L.slh_ctx_reserve.argtypes = [vp, u32, u32]
    L.slh_sign_batch_ext.argtypes = [vp, vp, u32, vp, u64, vp, u64, u32, vp]
    L.slh_verify_batch_ext.argtypes = [vp, vp, u32, vp, u64, vp, u64, vp, u64, vp, vp]
    L.slh_serve_create.argtypes = [ctypes.c_int, ctypes.POINTER(slh_serve_config), ctypes.POINTER(vp)]
    L.slh_serve_destroy.argtypes = [vp]
    L.slh_serve_last_error.argtypes = [vp]
    L.slh_serve_last_error.restype = ctypes.c_char_p
    L.slh_serve_add_keys.argtypes = [vp, u32, ctypes.c_char_p, u32, ctypes.POINTER(u32)]
    L.slh_serve_set_tuning.argtypes = [vp, u32, ctypes.POINTER(slh_tuning)]
    L.slh_serve_replay.argtypes = [vp, vp, u64, vp, u64, vp, u64, vp, u64, ctypes.POINTER(slh_serve_stats)]
    L.slh_serve_start.argtypes = [vp]
    L.slh_serve_stop.argtypes = [vp]
    L.slh_serve_submit.argtypes = [vp, u32, u32, ctypes.c_char_p, u64, u64]
    L.slh_serve_poll.argtypes = [vp, vp, vp, u64, vp, u32, ctypes.POINTER(u32)]
    return L


lib = _load()


def _check(rc, ctx=None):
    if rc < 0:
        raise SlhError(rc, lib.slh_last_error(ctx).decode(errors="replace"))
    return rc


def sizes(param: int) -> dict:
    s = slh_sizes()
    _check(lib.slh_params(int(param), ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in s._fields_}


def keygen(param: int, seed: bytes):
    """(pk, sk) from seed = SK.seed | SK.prf | PK.seed, computed on the GPU."""
    s = sizes(param)
    if len(seed) != s["seed_bytes"]:
        raise ValueError("seed must be %d bytes" % s["seed_bytes"])
    pk = ctypes.create_string_buffer(s["pk_bytes"])
    sk = ctypes.create_string_buffer(s["sk_bytes"])
    _check(lib.slh_keygen(int(param), seed, pk, sk))
    return pk.raw, sk.raw


def verify(param: int, msg: bytes, sig: bytes, pk: bytes) -> bool:
    """Signature check on the GPU; True if valid."""
    if len(pk) != sizes(param)["pk_bytes"]:
        raise ValueError("wrong public key length")
    rc = _check(lib.slh_verify(int(param), msg, len(msg), sig, len(sig), pk))
    return rc == 1


class Context:
    """A signing context: a device key table and working memory on one GPU."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = ctypes.c_void_p()
        _check(lib.slh_ctx_create(int(device), int(hbm_budget), ctypes.byref(h)))
        self.h = h
        self.device = device
        self.key_params: list[int] = []

    def close(self):
        if self.h:
            lib.slh_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def error(self) -> str:
        return lib.slh_last_error(self.h).decode(errors="replace")

    def add_keys(self, param: int, sks) -> int:
        """Upload secret keys (bytes or list of bytes, 4n each); returns the first slot."""
        blob = b"".join(sks) if isinstance(sks, (list, tuple)) else bytes(sks)
        skb = sizes(param)["sk_bytes"]
        if len(blob) == 0 or len(blob) % skb:
            raise ValueError("keys must be a positive multiple of %d bytes" % skb)
        first = ctypes.c_uint32()
        _check(lib.slh_ctx_add_keys(self.h, int(param), blob, len(blob) // skb, ctypes.byref(first)),
               self.h)
        self.key_params += [param] * (len(blob) // skb)
        return first.value

    def reserve(self, count: int, mode: int = MODE_PLAIN):
        """Allocate the working memory for batches of up to `count` requests now."""
        _check(lib.slh_ctx_reserve(self.h, int(count), int(mode)), self.h)

    def cache_keys(self, first_slot: int, count: int, layers: int):
        """Cache the top `layers` hypertree layers of keys first_slot .. first_slot + count - 1
        (used by the dedup modes)."""
        _check(lib.slh_ctx_cache_keys(self.h, int(first_slot), int(count), int(layers)), self.h)

    def set_tuning(self, param: int, fors_trees_per_group: int = 0, wgs_per_cu: int = 0,
                   keep_chains: int = 1, split_max_blocks: int = 0, **knobs):
        """Set the kernel knobs of a parameter set (the other slh_tuning
        fields, TUNING_FIELDS, as keywords; 0 = default)."""
        t = make_tuning(fors_trees_per_group, wgs_per_cu, keep_chains, split_max_blocks, **knobs)
        _check(lib.slh_ctx_set_tuning(self.h, int(param), ctypes.byref(t)), self.h)

    def get_tuning(self, param: int) -> dict:
        t = slh_tuning()
        _check(lib.slh_ctx_get_tuning(self.h, int(param), ctypes.byref(t)), self.h)
        return {f: getattr(t, f) for f in TUNING_FIELDS}

    def profile(self, enable: bool = True):
        """Record HIP events around every kernel of later sign_batch calls."""
        _check(lib.slh_ctx_profile(self.h, 1 if enable else 0), self.h)

    def phase_times(self, reset: bool = True) -> dict:
        """{phase: (milliseconds, launches, messages)} accumulated so far."""
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        la = (ctypes.c_uint64 * n)()
        me = (ctypes.c_uint64 * n)()
        _check(lib.slh_ctx_phase_times(self.h, ms, la, me, 1 if reset else 0), self.h)
        return {p: (ms[i], la[i], me[i]) for i, p in enumerate(PHASES)}

    def dedup_stats(self, reset: bool = True) -> tuple:
        """(trees needed, distinct trees computed) of the dedup-mode calls."""
        t, d = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib.slh_ctx_dedup_stats(self.h, ctypes.byref(t), ctypes.byref(d), 1 if reset else 0), self.h)
        return t.value, d.value

    def verify_batch(self, items: np.ndarray, msgs, sigs, pks, results, stream=None):
        """Enqueue verification of `items` (VERIFY_DTYPE); results is an int32
        CUDA tensor receiving 1 (valid) / 0 per item."""
        items = np.ascontiguousarray(items, dtype=VERIFY_DTYPE)
        mp, mb = _ptr(msgs)
        sp, sb = _ptr(sigs)
        pp, pb = _ptr(pks)
        rp, _ = _ptr(results)
        _check(lib.slh_verify_batch(self.h, items.ctypes.data, len(items), mp, mb, sp, sb, pp, pb, rp,
                                    _stream_handle(stream)), self.h)

    def sign_batch(self, items: np.ndarray, msgs, sigs, mode: int = MODE_PLAIN, stream=None):
        """Enqueue signing of `items` (ITEM_DTYPE array) on `stream`.

        msgs / sigs are uint8 CUDA tensors (or (pointer, nbytes) pairs)."""
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        mp, mb = _ptr(msgs)
        sp, sb = _ptr(sigs)
        st = _stream_handle(stream)
        _check(lib.slh_sign_batch(self.h, items.ctypes.data, len(items), mp, mb, sp, sb, int(mode), st),
               self.h)

    def sign_batch_noalloc(self, items: np.ndarray, msgs, sigs, mode: int = MODE_PLAIN, stream=None):
        """As sign_batch, through the entry point that allocates nothing (working
        memory in the library's fixed per-GPU array; at most NOALLOC_MAX_ITEMS items)."""
        items = np.ascontiguousarray(items, dtype=ITEM_DTYPE)
        mp, mb = _ptr(msgs)
        sp, sb = _ptr(sigs)
        _check(lib.slh_sign_batch_noalloc(self.h, items.ctypes.data, len(items), mp, mb, sp, sb, int(mode),
                                          _stream_handle(stream)), self.h)

    def verify_batch_ext(self, items: np.ndarray, msgs, sigs, pks, results, stream=None):
        """Enqueue verification through the external interface (VERIFY_EXT_DTYPE items)."""
        items = np.ascontiguousarray(items, dtype=VERIFY_EXT_DTYPE)
        mp, mb = _ptr(msgs)
        sp, sb = _ptr(sigs)
        pp, pb = _ptr(pks)
        rp, _ = _ptr(results)
        _check(lib.slh_verify_batch_ext(self.h, items.ctypes.data, len(items), mp, mb, sp, sb, pp, pb, rp,
                                        _stream_handle(stream)), self.h)

    def sign_batch_ext(self, items: np.ndarray, msgs, sigs, mode: int = MODE_PLAIN, stream=None):
        """Enqueue signing through the external interface (ITEM_EXT_DTYPE items)."""
        items = np.ascontiguousarray(items, dtype=ITEM_EXT_DTYPE)
        mp, mb = _ptr(msgs)
        sp, sb = _ptr(sigs)
        _check(lib.slh_sign_batch_ext(self.h, items.ctypes.data, len(items), mp, mb, sp, sb, int(mode),
                                      _stream_handle(stream)), self.h)


def _ptr(t):
    if isinstance(t, tuple):
        return ctypes.c_void_p(int(t[0])), int(t[1])
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def pack_batch(params, slots, messages, align: int = 16, msg_align: int = 4):
    """Lay out messages (each at a msg_align-byte offset; 4-byte aligned
    messages are hashed from dword loads) and signature slots; returns
    (items, msg_blob, sig_bytes_total)."""
    items = np.zeros(len(messages), dtype=ITEM_DTYPE)
    parts = []
    moff = 0
    soff = 0
    for i, (p, s, m) in enumerate(zip(params, slots, messages)):
        items[i] = (p, s, moff, len(m), soff)
        pad = (-len(m)) % msg_align
        parts.append(m + bytes(pad))
        moff += len(m) + pad
        soff += (sizes(p)["sig_bytes"] + align - 1) // align * align
    return items, b"".join(parts), soff


def sign_messages_ext(ctx: Context, params, slots, messages, contexts=None, prehash=None, rnds=None,
                      mode: int = MODE_PLAIN):
    """Sign through the external interface; contexts / prehash / rnds are
    per-message lists (None: empty context, pure, deterministic)."""
    import torch
    n = len(messages)
    contexts = contexts or [b""] * n
    prehash = prehash or [PREHASH_NONE] * n
    rnds = rnds or [None] * n
    items = np.zeros(n, dtype=ITEM_EXT_DTYPE)
    blob = bytearray()
    soff = 0
    for i in range(n):
        mo = len(blob)
        blob += messages[i]
        co = len(blob)
        blob += contexts[i]
        ro = RND_NONE
        if rnds[i] is not None:
            ro = len(blob)
            blob += rnds[i]
        items[i] = (params[i], slots[i], mo, len(messages[i]), soff, co, ro, len(contexts[i]), prehash[i])
        soff += (sizes(params[i])["sig_bytes"] + 15) // 16 * 16
    dev = torch.device("cuda", ctx.device)
    msgs = torch.frombuffer(bytearray(blob or b"\0"), dtype=torch.uint8).to(dev)
    sigs = torch.zeros(max(soff, 16), dtype=torch.uint8, device=dev)
    ctx.sign_batch_ext(items, (msgs.data_ptr(), len(blob)), sigs, mode)
    torch.cuda.synchronize(dev)
    host = sigs.cpu().numpy().tobytes()
    return [host[int(it["sig_off"]):int(it["sig_off"]) + sizes(int(it["param"]))["sig_bytes"]] for it in items]


def sign_messages(ctx: Context, params, slots, messages, mode: int = MODE_PLAIN):
    """Sign a list of messages synchronously; returns a list of signatures (bytes)."""
    import torch
    items, blob, total = pack_batch(params, slots, messages)
    dev = torch.device("cuda", ctx.device)
    msgs = torch.frombuffer(bytearray(blob or b"\0"), dtype=torch.uint8).to(dev)
    sigs = torch.zeros(max(total, 16), dtype=torch.uint8, device=dev)
    ctx.sign_batch(items, (msgs.data_ptr(), len(blob)), sigs, mode)
    torch.cuda.synchronize(dev)
    host = sigs.cpu().numpy().tobytes()
    return [host[int(it["sig_off"]):int(it["sig_off"]) + sizes(int(it["param"]))["sig_bytes"]]
            for it in items]


class Server:
    """Continuous-batching signing server (lanes of in-flight batches)."""

    def __init__(self, device: int = 0, lanes: int = 0, max_batch: int = 0, min_batch: int = 0,
                 max_wait_us: int = 0, msg_bytes: int = 0, hbm_budget: int = 0, mode: int = MODE_PLAIN,
                 queue_limit: int = 0, cache_layers: int = 0):
        cfg = slh_serve_config(lanes, max_batch, min_batch, max_wait_us, msg_bytes, hbm_budget, mode,
                               queue_limit, cache_layers, 0)
        h = ctypes.c_void_p()
        rc = lib.slh_serve_create(int(device), ctypes.byref(cfg), ctypes.byref(h))
        if rc < 0:
            raise SlhError(rc, "slh_serve_create failed")
        self.h = h

    def _check(self, rc):
        if rc < 0:
            raise SlhError(rc, lib.slh_serve_last_error(self.h).decode(errors="replace"))
        return rc

    def close(self):
        if self.h:
            lib.slh_serve_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_keys(self, param: int, sks) -> int:
        blob = b"".join(sks) if isinstance(sks, (list, tuple)) else bytes(sks)
        skb = sizes(param)["sk_bytes"]
        first = ctypes.c_uint32()
        self._check(lib.slh_serve_add_keys(self.h, int(param), blob, len(blob) // skb, ctypes.byref(first)))
        return first.value

    def set_tuning(self, param: int, fors_trees_per_group: int = 0, wgs_per_cu: int = 0, keep_chains: int = 1,
                   split_max_blocks: int = 0, **knobs):
        t = make_tuning(fors_trees_per_group, wgs_per_cu, keep_chains, split_max_blocks, **knobs)
        self._check(lib.slh_serve_set_tuning(self.h, int(param), ctypes.byref(t)))

    def replay(self, reqs: np.ndarray, msgs: bytes, skip: int = 0):
        """Serve a trace (REQ_DTYPE array, msg offsets into `msgs`).
        Returns (signature blob, latencies array, stats dict); each request's
        signature sits at its sig_off."""
        reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
        n = len(reqs)
        total = int((reqs["sig_off"] + MAX_SIG_BYTES).max()) if n else 16
        sigs = np.zeros(total, dtype=np.uint8)
        lat = np.zeros(max(1, n), dtype=np.float64)
        mbuf = np.frombuffer(msgs or b"\0", dtype=np.uint8)
        st = slh_serve_stats()
        self._check(lib.slh_serve_replay(self.h, reqs.ctypes.data, n, mbuf.ctypes.data, len(msgs),
                                         sigs.ctypes.data, total, lat.ctypes.data, int(skip), ctypes.byref(st)))
        return sigs, lat[:n], {f: getattr(st, f) for f, _ in st._fields_}

    def start(self):
        self._check(lib.slh_serve_start(self.h))

    def stop(self):
        self._check(lib.slh_serve_stop(self.h))

    def submit(self, param: int, key_slot: int, msg: bytes, tag: int) -> int:
        """0 if accepted, EBUSY if the queue is full."""
        rc = lib.slh_serve_submit(self.h, int(param), int(key_slot), msg, len(msg), int(tag))
        if rc == EBUSY:
            return rc
        return self._check(rc)

    def poll(self, max_results: int = 256):
        """List of (tag, signature bytes with trailing space, latency s)."""
        tags = np.zeros(max_results, dtype=np.uint64)
        sigs = np.zeros(max_results * MAX_SIG_BYTES, dtype=np.uint8)
        lat = np.zeros(max_results, dtype=np.float64)
        n = ctypes.c_uint32()
        self._check(lib.slh_serve_poll(self.h, tags.ctypes.data, sigs.ctypes.data, MAX_SIG_BYTES,
                                       lat.ctypes.data, max_results, ctypes.byref(n)))
        return [(int(tags[i]), sigs[i * MAX_SIG_BYTES:(i + 1) * MAX_SIG_BYTES].tobytes(), float(lat[i]))
                for i in range(n.value)]


def trace(params, slots, messages, arrivals):
    """Build a replay trace: (REQ_DTYPE array, message blob)."""
    reqs = np.zeros(len(messages), dtype=REQ_DTYPE)
    moff = soff = 0
    for i, (p, k, m, a) in enumerate(zip(params, slots, messages, arrivals)):
        reqs[i] = (p, k, moff, len(m), soff, a)
        moff += len(m)
        soff += (sizes(p)["sig_bytes"] + 15) // 16 * 16
    return reqs, b"".join(messages)
