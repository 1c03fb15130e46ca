"""ctypes binding of libphmm.so (include/phmm.h).  Argument marshalling only:
every step of the computation runs in the library's gfx950 kernels."""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libphmm.so")

PHMM_OK = 0
PHMM_EINVAL = -1
PHMM_ERANGE = -2
PHMM_ENOMEM = -3
PHMM_EDEVICE = -4
PHMM_ETIMEOUT = -5
PHMM_PENDING = 1
PHMM_FP32_RERUN = 0
PHMM_FP64_PLAIN = 1
PHMM_FLAG_FP32 = 0x01
PHMM_FLAG_RERUN = 0x02
PHMM_FLAG_LONG = 0x04
PHMM_FLAG_RESCALED = 0x08
PHMM_FLAG_FP64 = 0x10

_ERRNAMES = {PHMM_EINVAL: "PHMM_EINVAL", PHMM_ERANGE: "PHMM_ERANGE", PHMM_ENOMEM: "PHMM_ENOMEM",
             PHMM_EDEVICE: "PHMM_EDEVICE", PHMM_ETIMEOUT: "PHMM_ETIMEOUT"}


class PhmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("accept_min_sum", ctypes.c_double),
                ("force_class", ctypes.c_int), ("one_pair_per_wave", ctypes.c_int),
                ("fp32_max_rows", ctypes.c_uint32), ("long_fp32_max_rows", ctypes.c_uint32),
                ("watchdog_spins", ctypes.c_uint32),
                ("timing", ctypes.c_int), ("route_diverse_fp64", ctypes.c_int)]


class _DeviceBatch(ctypes.Structure):
    _fields_ = [("reads", ctypes.c_void_p), ("base_quals", ctypes.c_void_p),
                ("ins_quals", ctypes.c_void_p), ("del_quals", ctypes.c_void_p),
                ("gcp", ctypes.c_void_p), ("read_offsets", ctypes.c_void_p),
                ("n_reads", ctypes.c_uint32), ("haplotypes", ctypes.c_void_p),
                ("hap_offsets", ctypes.c_void_p), ("n_haps", ctypes.c_uint32),
                ("pair_list", ctypes.c_void_p), ("n_pairs", ctypes.c_uint64),
                ("max_read_len", ctypes.c_uint32), ("max_hap_len", ctypes.c_uint32)]


class _Counts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("packs_fp32", "packs_fp64", "rerun_items",
                                                "rerun_pairs", "long_pairs", "long_tiles",
                                                "lane_columns", "long_pairs_fp32",
                                                "deferred_packs")]


class _ServerOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("lanes", ctypes.c_uint32),
                ("long_lanes", ctypes.c_uint32), ("hbm_budget_bytes", ctypes.c_uint64),
                ("max_batch_regions", ctypes.c_uint32), ("short_cu_percent", ctypes.c_uint32),
                ("long_read_min", ctypes.c_uint32), ("long_grid_percent", ctypes.c_uint32)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("lane", ctypes.c_uint32), ("is_long", ctypes.c_uint32),
                ("batch", ctypes.c_uint64), ("queue_s", ctypes.c_double),
                ("latency_s", ctypes.c_double)]


class _ServerCounters(ctypes.Structure):
    _fields_ = [("regions", ctypes.c_uint64), ("pairs", ctypes.c_uint64),
                ("cells", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("full_batches", ctypes.c_uint64), ("waiting_short", ctypes.c_uint64),
                ("waiting_long", ctypes.c_uint64), ("lane_busy_s", ctypes.c_double),
                ("span_s", ctypes.c_double), ("cu_mask_status", ctypes.c_int)]


class _Timing(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("pack_ms", "short_ms", "rerun_ms", "long_ms",
                                               "total_ms")]


_lock = threading.Lock()
_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libphmm.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                raise RuntimeError("libphmm.so is not built (python -m paper_2606_25738_amd.build)")
            # torch ships its own HIP runtime under the same soname
            # (libamdhip64.so.7) as the system one libphmm.so links: whichever
            # is loaded first serves the whole process, and torch does not
            # find the GPU on a runtime other than its own.  Load torch's
            # first so that the library and torch share it.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(_LIB_PATH)
            vp, u8p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8)
            u64p, u32p = ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint32)
            dp = ctypes.POINTER(ctypes.c_double)
            L.phmm_default_options.argtypes = [ctypes.POINTER(_Options)]
            L.phmm_default_options.restype = None
            L.phmm_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(_Options)]
            L.phmm_destroy.argtypes = [vp]
            L.phmm_destroy.restype = None
            L.phmm_last_error.restype = ctypes.c_char_p
            L.phmm_class_n.argtypes = [ctypes.c_int]
            L.phmm_validate_batch.argtypes = [u8p] * 5 + [u64p, ctypes.c_uint32, u8p, u64p,
                                                         ctypes.c_uint32, u32p, ctypes.c_uint64,
                                                         u32p, u32p]
            L.phmm_forward_batch.argtypes = [vp] + [u8p] * 5 + [u64p, ctypes.c_uint32, u8p, u64p,
                                                               ctypes.c_uint32, u32p,
                                                               ctypes.c_uint64, dp, u8p]
            L.phmm_forward_one.argtypes = [u8p] * 5 + [ctypes.c_uint32, u8p, ctypes.c_uint32, dp]
            L.phmm_workspace_bytes.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32,
                                               ctypes.c_uint32]
            L.phmm_workspace_bytes.restype = ctypes.c_size_t
            L.phmm_forward_batch_async.argtypes = [vp, ctypes.POINTER(_DeviceBatch), vp, vp, vp,
                                                   ctypes.c_size_t, vp]
            L.phmm_forward_batch_graph.argtypes = [vp, ctypes.POINTER(_DeviceBatch), vp, vp, vp,
                                                   ctypes.c_size_t, vp]
            L.phmm_forward_batch_noalloc.argtypes = [vp, ctypes.POINTER(_DeviceBatch), vp, vp, vp]
            L.phmm_device_status.argtypes = [vp, vp]
            L.phmm_last_counts.argtypes = [vp, vp, ctypes.POINTER(_Counts)]
            L.phmm_last_timing.argtypes = [vp, ctypes.POINTER(_Timing)]
            L.phmm_vector_peak.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]
            L.phmm_copy_calib.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                          ctypes.c_void_p]
            fp = ctypes.POINTER(ctypes.c_float)
            L.phmm_autotune.argtypes = [vp, ctypes.c_uint64, fp]
            L.phmm_set_class_costs.argtypes = [vp, fp]
            L.phmm_autotune_sample.argtypes = [vp, ctypes.POINTER(_DeviceBatch), vp, ctypes.c_size_t,
                                               vp, fp]
            L.phmm_get_class_costs.argtypes = [vp, fp]
            L.phmm_genotype_batch.argtypes = [vp, dp, ctypes.c_uint64, u64p, u32p, u32p, u64p,
                                              ctypes.c_uint32, dp, ctypes.c_uint64, u32p]
            L.phmm_genotype_batch_async.argtypes = [vp] + [ctypes.c_void_p, ctypes.c_uint64] + \
                [ctypes.c_void_p] * 4 + [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_void_p]
            L.phmm_server_default_options.argtypes = [ctypes.POINTER(_ServerOptions)]
            L.phmm_server_default_options.restype = None
            L.phmm_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int,
                                             ctypes.POINTER(_ServerOptions)]
            L.phmm_server_destroy.argtypes = [vp]
            L.phmm_server_destroy.restype = None
            L.phmm_server_submit.argtypes = [vp] + [u8p] * 5 + [u64p, ctypes.c_uint32, u8p, u64p,
                                                               ctypes.c_uint32,
                                                               ctypes.POINTER(ctypes.c_uint32),
                                                               ctypes.c_uint64,
                                                               ctypes.POINTER(ctypes.c_uint64)]
            for f in (L.phmm_server_wait, L.phmm_server_poll):
                f.argtypes = [vp, ctypes.c_uint64, dp, u8p, ctypes.POINTER(_RequestInfo)]
            L.phmm_server_stats.argtypes = [vp, ctypes.POINTER(_ServerCounters)]
            _lib = L
    return _lib


def _check(rc: int):
    if rc != PHMM_OK:
        raise PhmmError(rc, lib().phmm_last_error().decode(errors="replace"))


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u64(a):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def phmm_num_classes() -> int:
    return lib().phmm_num_classes()


def phmm_class_n(c: int) -> int:
    return lib().phmm_class_n(c)


class Context:
    """A phmm_ctx on one device (phmm_create / phmm_destroy)."""

    def __init__(self, device: int = 0, precision: int = PHMM_FP32_RERUN,
                 accept_min_sum: float | None = None, force_class: int = -1,
                 one_pair_per_wave: bool = False, fp32_max_rows: int | None = None,
                 long_fp32_max_rows: int | None = None,
                 watchdog_spins: int = 0, timing: bool = False,
                 route_diverse_fp64: bool = True):
        L = lib()
        o = _Options()
        L.phmm_default_options(ctypes.byref(o))
        o.precision = precision
        if accept_min_sum is not None:
            o.accept_min_sum = accept_min_sum
        o.force_class = force_class
        o.one_pair_per_wave = int(bool(one_pair_per_wave))
        if fp32_max_rows is not None:
            o.fp32_max_rows = fp32_max_rows
        if long_fp32_max_rows is not None:
            o.long_fp32_max_rows = long_fp32_max_rows
        o.watchdog_spins = watchdog_spins
        o.timing = int(bool(timing))
        o.route_diverse_fp64 = int(bool(route_diverse_fp64))
        h = ctypes.c_void_p()
        _check(L.phmm_create(ctypes.byref(h), device, ctypes.byref(o)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def autotune(self, seed: int = 0) -> np.ndarray:
        """Measure the per-class wavefront-row costs on this device and use them
        for packing; returns them as a (2, n_classes) array (FP32, FP64), ns."""
        c = np.zeros(2 * phmm_num_classes(), np.float32)
        _check(lib().phmm_autotune(self._h, seed, c.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return c.reshape(2, -1)

    def autotune_sample(self, db, workspace, stream=None) -> np.ndarray:
        """Pick the cost table that runs a sample of the real workload (a
        DeviceBatch) fastest; returns it as a (2, n_classes) array."""
        c = np.zeros(2 * phmm_num_classes(), np.float32)
        st = db.struct()
        h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
        _check(lib().phmm_autotune_sample(self._h, ctypes.byref(st), workspace.data_ptr(),
                                          workspace.numel() * workspace.element_size(), h,
                                          c.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return c.reshape(2, -1)

    def class_costs(self) -> np.ndarray:
        c = np.zeros(2 * phmm_num_classes(), np.float32)
        _check(lib().phmm_get_class_costs(self._h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return c.reshape(2, -1)

    def set_class_costs(self, costs) -> None:
        c = np.ascontiguousarray(np.asarray(costs, np.float32).reshape(-1))
        if c.size != 2 * phmm_num_classes():
            raise ValueError("set_class_costs: need 2 x %d costs" % phmm_num_classes())
        _check(lib().phmm_set_class_costs(self._h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def close(self):
        if getattr(self, "_h", None):
            lib().phmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _batch_args(batch):
    keep = []
    args = []
    for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp"):
        a, p = _u8(batch[k])
        keep.append(a)
        args.append(p)
    ro, pro = _u64(batch["read_offsets"])
    haps, ph = _u8(batch["haplotypes"])
    ho, pho = _u64(batch["hap_offsets"])
    pl, ppl = _u32(np.asarray(batch["pair_list"]).reshape(-1))
    keep += [ro, haps, ho, pl]
    args += [pro, len(ro) - 1, ph, pho, len(ho) - 1, ppl, len(pl) // 2]
    return keep, args


def phmm_validate_batch(batch) -> tuple[int, int]:
    """Host-side validation; returns (max_read_len, max_hap_len)."""
    keep, args = _batch_args(batch)
    ml, mk = ctypes.c_uint32(0), ctypes.c_uint32(0)
    _check(lib().phmm_validate_batch(*args, ctypes.byref(ml), ctypes.byref(mk)))
    return ml.value, mk.value


def phmm_forward_batch(ctx: Context, batch):
    """Synchronous batch from host numpy arrays -> (log10 L, flags)."""
    keep, args = _batch_args(batch)
    n = args[-1]
    out = np.empty(n, np.float64)
    flags = np.empty(n, np.uint8)
    _check(lib().phmm_forward_batch(ctx.handle, *args,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return out, flags


def phmm_forward_one(read, base_quals, ins_quals, del_quals, gcp, hap) -> float:
    def seq(s):
        if isinstance(s, str):
            s = s.encode("ascii")
        return _u8(np.frombuffer(bytes(s), np.uint8) if isinstance(s, (bytes, bytearray)) else s)
    r, pr = seq(read)
    h, ph = seq(hap)
    q = [_u8(x) for x in (base_quals, ins_quals, del_quals, gcp)]
    out = ctypes.c_double(0.0)
    _check(lib().phmm_forward_one(pr, *[x[1] for x in q], len(r), ph, len(h), ctypes.byref(out)))
    return out.value


def phmm_workspace_bytes(ctx: Context, n_pairs: int, max_read_len: int, max_hap_len: int) -> int:
    return lib().phmm_workspace_bytes(ctx.handle, n_pairs, max_read_len, max_hap_len)


class DeviceBatch:
    """A batch resident in device memory (torch tensors are the allocator)."""

    def __init__(self, batch, device="cuda:0"):
        import torch
        self.n_pairs = int(len(batch["pair_list"]))
        self.n_reads = int(len(batch["read_offsets"]) - 1)
        self.n_haps = int(len(batch["hap_offsets"]) - 1)
        rl = np.diff(np.asarray(batch["read_offsets"], np.int64))
        hl = np.diff(np.asarray(batch["hap_offsets"], np.int64))
        self.max_read_len = int(rl.max()) if len(rl) else 0
        self.max_hap_len = int(hl.max()) if len(hl) else 0

        def up(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        self.t = {k: up(batch[k], np.uint8) for k in ("reads", "base_quals", "ins_quals",
                                                        "del_quals", "gcp", "haplotypes")}
        self.t["read_offsets"] = up(np.asarray(batch["read_offsets"]).view(np.int64), np.int64)
        self.t["hap_offsets"] = up(np.asarray(batch["hap_offsets"]).view(np.int64), np.int64)
        self.t["pair_list"] = up(np.asarray(batch["pair_list"], np.uint32).reshape(-1).view(np.int32),
                                 np.int32)

    def struct(self) -> _DeviceBatch:
        t = self.t
        s = _DeviceBatch()
        for k in ("reads", "base_quals", "ins_quals", "del_quals", "gcp", "read_offsets",
                  "haplotypes", "hap_offsets", "pair_list"):
            setattr(s, k, t[k].data_ptr())
        s.n_reads, s.n_haps, s.n_pairs = self.n_reads, self.n_haps, self.n_pairs
        s.max_read_len, s.max_hap_len = self.max_read_len, self.max_hap_len
        return s


def phmm_forward_batch_async(ctx: Context, db: DeviceBatch, out, flags, workspace, stream=None):
    """Enqueue on a HIP stream (torch stream or raw handle); device tensors in/out."""
    s = db.struct()
    if stream is None:
        h = None
    elif hasattr(stream, "cuda_stream"):
        h = stream.cuda_stream
    else:
        h = stream
    _check(lib().phmm_forward_batch_async(
        ctx.handle, ctypes.byref(s), out.data_ptr(),
        flags.data_ptr() if flags is not None else None, workspace.data_ptr(),
        workspace.numel() * workspace.element_size(), h))


def phmm_forward_batch_graph(ctx: Context, db: DeviceBatch, out, flags, workspace, stream=None):
    """phmm_forward_batch_async replayed from the context's captured HIP graphs."""
    s = db.struct()
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib().phmm_forward_batch_graph(
        ctx.handle, ctypes.byref(s), out.data_ptr(),
        flags.data_ptr() if flags is not None else None, workspace.data_ptr(),
        workspace.numel() * workspace.element_size(), h))


def phmm_forward_batch_noalloc(ctx: Context, db: DeviceBatch, out, flags, stream=None):
    """phmm_forward_batch_async with the library's static device scratch
    instead of a caller workspace (allocates nothing)."""
    s = db.struct()
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib().phmm_forward_batch_noalloc(
        ctx.handle, ctypes.byref(s), out.data_ptr(),
        flags.data_ptr() if flags is not None else None, h))


def genotype_offsets(region_haps) -> tuple[np.ndarray, int]:
    """Back-to-back genotype blocks: the offset of each region's H(H+1)/2
    genotypes and their total."""
    h = np.asarray(region_haps, dtype=np.uint64)
    g = h * (h + np.uint64(1)) // np.uint64(2)
    off = np.zeros(len(h), np.uint64)
    if len(h) > 1:
        off[1:] = np.cumsum(g[:-1], dtype=np.uint64)
    return off, int(g.sum()) if len(h) else 0


def phmm_genotype_batch(ctx: Context | None, lk, lk_offsets, region_reads, region_haps,
                        gl_offsets=None, gl=None):
    """Diploid genotype log10-likelihoods per region from the read x haplotype
    log10 matrix (host arrays) -> (gl, best).  gl_offsets None: back-to-back
    blocks; gl None: a new array of the needed size.  ctx None only exercises
    the host-side checks (a valid batch then fails with PHMM_EINVAL)."""
    lk = np.ascontiguousarray(lk, dtype=np.float64)
    lo, lo_p = _u64(lk_offsets)
    nr, nr_p = _u32(region_reads)
    nh, nh_p = _u32(region_haps)
    if gl_offsets is None:
        gl_offsets, n_gl = genotype_offsets(nh)
    else:
        n_gl = None
    go, go_p = _u64(gl_offsets)
    if gl is None:
        gl = np.zeros(n_gl if n_gl is not None else 0, np.float64)
    gl = np.ascontiguousarray(gl, dtype=np.float64)
    best = np.zeros(len(nh), np.uint32)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().phmm_genotype_batch(ctx.handle if ctx is not None else None,
                                     lk.ctypes.data_as(dp), lk.size, lo_p, nr_p, nh_p, go_p,
                                     len(nh), gl.ctypes.data_as(dp), gl.size,
                                     best.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))))
    return gl, best


def phmm_genotype_batch_async(ctx: Context, lk, lk_offsets, region_reads, region_haps,
                              gl_offsets, gl, best, stream=None):
    """Stream-ordered genotype likelihoods on device tensors (float64 lk and
    gl, int64 offsets, int32 counts and best)."""
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib().phmm_genotype_batch_async(
        ctx.handle, lk.data_ptr(), lk.numel(), lk_offsets.data_ptr(), region_reads.data_ptr(),
        region_haps.data_ptr(), gl_offsets.data_ptr(), region_haps.numel(), gl.data_ptr(),
        gl.numel(), best.data_ptr(), h))


def phmm_device_status(ctx: Context, workspace):
    _check(lib().phmm_device_status(ctx.handle, workspace.data_ptr()))


def phmm_last_counts(ctx: Context, workspace) -> dict:
    c = _Counts()
    _check(lib().phmm_last_counts(ctx.handle, workspace.data_ptr(), ctypes.byref(c)))
    return {n: getattr(c, n) for n, _ in _Counts._fields_}


def phmm_vector_peak(device: int = 0) -> tuple[float, float]:
    """Measured (FP32, FP64) vector FMA TFLOP/s of the device."""
    a, b = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().phmm_vector_peak(device, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class Server:
    """A phmm_server: continuous batching of submitted regions (the C
    runtime's worker threads do the batching; this class marshals)."""

    def __init__(self, device: int = 0, precision: int = PHMM_FP32_RERUN, lanes: int | None = None,
                 long_lanes: int | None = None, hbm_budget_bytes: int | None = None,
                 max_batch_regions: int | None = None, short_cu_percent: int | None = None,
                 long_read_min: int | None = None, long_grid_percent: int | None = None):
        L = lib()
        o = _ServerOptions()
        L.phmm_server_default_options(ctypes.byref(o))
        o.precision = precision
        for k, v in (("lanes", lanes), ("long_lanes", long_lanes),
                     ("hbm_budget_bytes", hbm_budget_bytes),
                     ("max_batch_regions", max_batch_regions),
                     ("short_cu_percent", short_cu_percent), ("long_read_min", long_read_min),
                     ("long_grid_percent", long_grid_percent)):
            if v is not None:
                setattr(o, k, v)
        h = ctypes.c_void_p()
        _check(L.phmm_server_create(ctypes.byref(h), device, ctypes.byref(o)))
        self._h = h
        self._np = {}

    def submit(self, region) -> int:
        """Submit one region (a batch dict); returns its ticket."""
        keep, args = _batch_args(region)
        t = ctypes.c_uint64(0)
        _check(lib().phmm_server_submit(self._h, *args, ctypes.byref(t)))
        self._np[t.value] = args[-1]
        return t.value

    def _collect(self, fn, ticket):
        n = self._np[ticket]
        out = np.empty(n, np.float64)
        flags = np.empty(n, np.uint8)
        info = _RequestInfo()
        rc = fn(self._h, ticket, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(info))
        if rc == PHMM_PENDING:
            return None
        del self._np[ticket]
        _check(rc)
        return out, flags, {n_: getattr(info, n_) for n_, _ in _RequestInfo._fields_}

    def wait(self, ticket: int):
        """Block until the region is done -> (log10 L, flags, info dict)."""
        return self._collect(lib().phmm_server_wait, ticket)

    def poll(self, ticket: int):
        """(log10 L, flags, info) if done, else None."""
        return self._collect(lib().phmm_server_poll, ticket)

    def stats(self) -> dict:
        c = _ServerCounters()
        _check(lib().phmm_server_stats(self._h, ctypes.byref(c)))
        return {n: getattr(c, n) for n, _ in _ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().phmm_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def phmm_copy_calib(src, dst, stream=None) -> None:
    """Plain device copy of src into dst (torch uint8 device tensors of equal
    size), the reference kernel of traffic-counter calibration."""
    if src.numel() != dst.numel() or src.element_size() != 1 or dst.element_size() != 1:
        raise ValueError("phmm_copy_calib: src and dst must be byte tensors of equal size")
    s = stream.cuda_stream if stream is not None else None
    _check(lib().phmm_copy_calib(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                 src.numel(), ctypes.c_void_p(s)))


def phmm_last_timing(ctx: Context) -> dict:
    t = _Timing()
    _check(lib().phmm_last_timing(ctx.handle, ctypes.byref(t)))
    return {n: getattr(t, n) for n, _ in _Timing._fields_}
