"""ctypes binding of libbsw.so (argument marshalling only).

Every step of the extension runs in the library's HIP kernels; this module
only converts NumPy arrays / torch tensors into the C ABI's pointers and
sizes.  PyTorch is used for device memory and streams.  The library must
have been built (``python -m paper_1907_12931_amd.build``); there is no
other implementation to fall back to, so a missing or unloadable library
raises ``BswError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsw.so")

OK, EINVAL, ENOMEM, EDEVICE, ETOOBIG, EBUSY, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
NOALLOC_MAX_PAIRS = 131072
PATH_BATCHED, PATH_PLAIN = 0, 1
STATUS_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE",
                ETOOBIG: "ETOOBIG", EBUSY: "EBUSY", ETIMEOUT: "ETIMEOUT"}


class BswError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("mat", ctypes.c_int8 * 25), ("pad_", ctypes.c_int8 * 3),
                ("o_del", ctypes.c_int32), ("e_del", ctypes.c_int32),
                ("o_ins", ctypes.c_int32), ("e_ins", ctypes.c_int32),
                ("w", ctypes.c_int32), ("zdrop", ctypes.c_int32),
                ("end_bonus", ctypes.c_int32)]


class CtxOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("min_lane_bits", ctypes.c_int32),
                ("max_groups", ctypes.c_int32), ("path", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t), ("tune_cache", ctypes.c_char_p),
                ("no_graph", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("max_batch_pairs", ctypes.c_int64), ("hbm_budget", ctypes.c_size_t),
                ("max_queued", ctypes.c_int32), ("min_lane_bits", ctypes.c_int32)]


class ServerReport(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("submitted", "completed", "failed", "batches", "pairs", "cells")] + \
               [(k, ctypes.c_double) for k in
                ("mean_batch_pairs", "lat_p50_ms", "lat_p99_ms", "lat_p999_ms",
                 "lat_max_ms", "admit_wait_mean_ms", "admit_wait_p99_ms", "window_s",
                 "gcups")]


RESULT_DTYPE = np.dtype([("score", "<i4"), ("qle", "<i4"), ("tle", "<i4"),
                         ("gtle", "<i4"), ("gscore", "<i4"), ("max_off", "<i4")])
DIAG_DTYPE = np.dtype([("rows", "<i4"), ("stop", "<i4"), ("cells", "<i8")])
# read-level seed extension (bsw_seed / bsw_seed_result)
SEED_DTYPE = np.dtype([("read", "<i4"), ("qb", "<i4"), ("qe", "<i4"), ("h0", "<i4"),
                       ("rb", "<i8")])
SEED_RESULT_DTYPE = np.dtype([("score", "<i4"), ("qbeg", "<i4"), ("qend", "<i4"),
                              ("how", "<i4"), ("rbeg", "<i8"), ("rend", "<i8")])
END_LOCAL, END_READ, END_NONE = 0, 1, 2
# suffix-array lookup (bsw_sa_interval): rows [k, k + s)
SA_INTERVAL_DTYPE = np.dtype([("k", "<u8"), ("s", "<u8")])
# FM-index (bsw_fm_entry, bsw_bi_interval)
FM_ENTRY_DTYPE = np.dtype([("count", "<u4", (4,)), ("bwt", "u1", (32,)), ("pad_", "u1", (16,))])
BI_INTERVAL_DTYPE = np.dtype([("k", "<u8"), ("l", "<u8"), ("s", "<u8"), ("matched", "<i4"),
                              ("pad_", "<i4")])
SMEM_DTYPE = np.dtype([("start", "<u4"), ("end", "<u4"), ("k", "<u8"), ("l", "<u8"),
                       ("s", "<u8")])


class FmMeta(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_uint64), ("C", ctypes.c_uint64 * 4),
                ("primary", ctypes.c_uint64), ("entries", ctypes.c_uint64)]

_lib = None
_VP = ctypes.c_void_p


def lib():
    """Load libbsw.so (raises BswError if it is not built).

    torch is imported first when it is installed: its wheel carries its own
    HIP runtime with the same soname as ROCm's, and loading ours first would
    put two HIP runtimes in the process (torch then finds no GPU).  With
    torch loaded, libbsw.so binds to torch's runtime and device pointers and
    streams are shared."""
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise BswError(EDEVICE, f"{LIB_PATH} is not built; run "
                           "python -m paper_1907_12931_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.bsw_abi_version.restype = ctypes.c_int
        L.bsw_last_error.restype = ctypes.c_char_p
        L.bsw_ctx_create.restype = ctypes.c_int
        L.bsw_ctx_create.argtypes = [ctypes.POINTER(_VP), ctypes.POINTER(CtxOpts)]
        L.bsw_ctx_destroy.restype = None
        L.bsw_ctx_destroy.argtypes = [_VP]
        L.bsw_extend_batch.restype = ctypes.c_int
        L.bsw_extend_batch.argtypes = [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP,
                                       _VP, ctypes.POINTER(Params), ctypes.c_int32,
                                       _VP, _VP]
        L.bsw_extend_batch_device.restype = ctypes.c_int
        L.bsw_extend_batch_device.argtypes = [
            _VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP,
            ctypes.POINTER(Params), ctypes.c_int32, _VP, _VP, _VP, ctypes.c_int32]
        L.bsw_ctx_wait.restype = ctypes.c_int
        L.bsw_ctx_wait.argtypes = [_VP]
        L.bsw_ctx_last_kernels.restype = ctypes.c_int
        L.bsw_ctx_last_kernels.argtypes = [_VP, _VP, _VP, _VP, ctypes.c_int32]
        L.bsw_class_name.restype = ctypes.c_char_p
        L.bsw_class_name.argtypes = [ctypes.c_int32]
        L.bsw_ctx_last_timing.restype = ctypes.c_int
        L.bsw_ctx_last_timing.argtypes = [_VP, ctypes.POINTER(ctypes.c_double)]
        L.bsw_ctx_tune.restype = ctypes.c_int
        L.bsw_ctx_tune.argtypes = [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP,
                                   ctypes.POINTER(Params), ctypes.c_int32, _VP,
                                   ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.bsw_ctx_last_cells.restype = ctypes.c_int
        L.bsw_ctx_last_cells.argtypes = [_VP, ctypes.POINTER(ctypes.c_int64)]
        L.bsw_extend_seeds.restype = ctypes.c_int
        L.bsw_extend_seeds.argtypes = [_VP, _VP, _VP, ctypes.c_int64, _VP, ctypes.c_uint64,
                                       _VP, ctypes.c_int64, ctypes.POINTER(Params), _VP]
        L.bsw_extend_seeds_device.restype = ctypes.c_int
        L.bsw_extend_seeds_device.argtypes = [
            _VP, _VP, ctypes.c_uint64, _VP, ctypes.c_int64, _VP, _VP, ctypes.c_uint64,
            _VP, ctypes.c_int64, ctypes.POINTER(Params), _VP, _VP, ctypes.c_int32]
        L.bsw_ctx_tune_seeds.restype = ctypes.c_int
        L.bsw_ctx_tune_seeds.argtypes = [
            _VP, _VP, ctypes.c_uint64, _VP, ctypes.c_int64, _VP, _VP, ctypes.c_uint64,
            _VP, ctypes.c_int64, ctypes.POINTER(Params), _VP, ctypes.c_int32,
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
        L.bsw_sa_lookup_device.restype = ctypes.c_int
        L.bsw_sa_lookup_device.argtypes = [
            _VP, _VP, ctypes.c_uint64, _VP, ctypes.c_int64, _VP, _VP, ctypes.c_uint64,
            ctypes.POINTER(ctypes.c_uint64), _VP, ctypes.c_int32]
        L.bsw_fm_build.restype = ctypes.c_int
        L.bsw_fm_build.argtypes = [_VP, ctypes.c_uint64, _VP, _VP, ctypes.POINTER(FmMeta)]
        L.bsw_fm_backward_search_device.restype = ctypes.c_int
        L.bsw_fm_backward_search_device.argtypes = [
            _VP, _VP, ctypes.POINTER(FmMeta), _VP, _VP, ctypes.c_int64, _VP, _VP,
            ctypes.c_int32]
        L.bsw_fm_smem_device.restype = ctypes.c_int
        L.bsw_fm_smem_device.argtypes = [_VP, _VP, ctypes.POINTER(FmMeta), _VP, _VP,
                                         ctypes.c_int64, ctypes.c_uint32, _VP, _VP, _VP,
                                         ctypes.c_int32]
        L.bsw_ctx_tune_info.restype = ctypes.c_int
        L.bsw_ctx_tune_info.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32)]
        L.bsw_server_create.restype = ctypes.c_int
        L.bsw_server_create.argtypes = [ctypes.POINTER(_VP), ctypes.POINTER(ServerOpts),
                                        ctypes.POINTER(Params), ctypes.c_int32]
        L.bsw_server_destroy.restype = None
        L.bsw_server_destroy.argtypes = [_VP]
        L.bsw_server_submit.restype = ctypes.c_int
        L.bsw_server_submit.argtypes = [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP,
                                        _VP, _VP, ctypes.POINTER(ctypes.c_uint64)]
        L.bsw_server_wait.restype = ctypes.c_int
        L.bsw_server_wait.argtypes = [_VP, ctypes.c_uint64, ctypes.c_int32]
        L.bsw_server_stats.restype = ctypes.c_int
        L.bsw_server_stats.argtypes = [_VP, ctypes.POINTER(ServerReport), ctypes.c_int32]
        L.bsw_extend_batch_device_noalloc.restype = ctypes.c_int
        L.bsw_extend_batch_device_noalloc.argtypes = [
            _VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP,
            ctypes.POINTER(Params), ctypes.c_int32, _VP, _VP, _VP, ctypes.c_int32]
        L.bsw_filter_seeds_device.restype = ctypes.c_int
        L.bsw_filter_seeds_device.argtypes = [_VP, _VP, ctypes.c_int64, _VP, _VP, _VP,
                                              ctypes.c_int32]
        L.bsw_ctx_shape.restype = ctypes.c_int
        L.bsw_ctx_shape.argtypes = [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
        L.bsw_ctx_last_work.restype = ctypes.c_int
        L.bsw_ctx_last_work.argtypes = [_VP, _VP, ctypes.c_int32]
        L.bsw_valu_peak.restype = ctypes.c_int
        L.bsw_valu_peak.argtypes = [ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        if L.bsw_abi_version() != 1:
            raise BswError(EDEVICE, "libbsw.so ABI version mismatch")
        _lib = L
    return _lib


PEAK_KINDS = {"v_add_u32": 0, "v_max3_i32": 1, "v_pk_add_u16": 2, "v_pk_max_i16": 3}


def valu_peak(kind, device=0):
    """Measured integer-VALU rate (``bsw_valu_peak``): returns
    (lane-instructions/s, operations/s) for one instruction kind."""
    ip, op = ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().bsw_valu_peak(device, PEAK_KINDS[kind], ctypes.byref(ip), ctypes.byref(op)))
    return ip.value, op.value


def last_error() -> str:
    return lib().bsw_last_error().decode()


def _check(rc):
    if rc != OK:
        raise BswError(rc, last_error())


def make_params(scorings):
    arr = (Params * len(scorings))()
    for i, sc in enumerate(scorings):
        mat = np.asarray(sc["mat"], dtype=np.int64).reshape(25)
        for k in range(25):
            arr[i].mat[k] = int(mat[k])
        for name in ("o_del", "e_del", "o_ins", "e_ins", "w", "zdrop", "end_bonus"):
            setattr(arr[i], name, int(sc[name]))
    return arr


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class Context:
    """A library context on one device (see ``bsw_ctx_create``)."""

    def __init__(self, device=0, min_lane_bits=0, path=PATH_BATCHED,
                 hbm_budget=0, tune_cache=None, graph=True, max_groups=0):
        # the library copies the path; the bytes only need to live for the call
        tc = tune_cache.encode() if tune_cache else None
        o = CtxOpts(device, min_lane_bits, max_groups, path, hbm_budget, tc,
                    0 if graph else 1)
        h = _VP()
        _check(lib().bsw_ctx_create(ctypes.byref(h), ctypes.byref(o)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().bsw_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def extend(self, batch, with_diag=False):
        """Host-memory batch (NumPy arrays, see ``synth``) -> results[, diag]."""
        q = np.ascontiguousarray(batch["q"], dtype=np.uint8)
        t = np.ascontiguousarray(batch["t"], dtype=np.uint8)
        qo = np.ascontiguousarray(batch["q_off"], dtype=np.uint64)
        to = np.ascontiguousarray(batch["t_off"], dtype=np.uint64)
        h0 = np.ascontiguousarray(batch["h0"], dtype=np.int32)
        pid = batch.get("param_id")
        pid = None if pid is None else np.ascontiguousarray(pid, dtype=np.uint8)
        n = len(h0)
        params = make_params(batch["scorings"])
        out = np.zeros(n, dtype=RESULT_DTYPE)
        diag = np.zeros(n, dtype=DIAG_DTYPE) if with_diag else None
        _check(lib().bsw_extend_batch(
            self._h, n, _ptr(q), qo.ctypes.data, _ptr(t), to.ctypes.data,
            _ptr(h0), _ptr(pid), params, len(params), _ptr(out), _ptr(diag)))
        return (out, diag) if with_diag else out

    def extend_device(self, dev, scorings, out, diag=None, stream=None, async_=False):
        """Device batch: ``dev`` maps q, q_off, t, t_off, h0[, param_id] to
        torch tensors on the GPU; ``out`` (and ``diag``) are torch tensors of
        n*24 (n*16) bytes.  ``stream``: a torch.cuda.Stream or None."""
        n = dev["h0"].numel()
        params = make_params(scorings)
        pid = dev.get("param_id")
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_extend_batch_device(
            self._h, n, dev["q"].data_ptr(), dev["q_off"].data_ptr(),
            dev["t"].data_ptr(), dev["t_off"].data_ptr(), dev["h0"].data_ptr(),
            pid.data_ptr() if pid is not None else None, params, len(params),
            out.data_ptr(), diag.data_ptr() if diag is not None else None, s,
            1 if async_ else 0))

    def extend_device_noalloc(self, dev, scorings, out, diag=None, stream=None,
                              async_=False):
        """As ``extend_device``, through the allocation-free entry point
        (``bsw_extend_batch_device_noalloc``)."""
        n = dev["h0"].numel()
        params = make_params(scorings)
        pid = dev.get("param_id")
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_extend_batch_device_noalloc(
            self._h, n, dev["q"].data_ptr(), dev["q_off"].data_ptr(),
            dev["t"].data_ptr(), dev["t_off"].data_ptr(), dev["h0"].data_ptr(),
            pid.data_ptr() if pid is not None else None, params, len(params),
            out.data_ptr(), diag.data_ptr() if diag is not None else None, s,
            1 if async_ else 0))

    def wait(self):
        _check(lib().bsw_ctx_wait(self._h))

    def extend_seeds(self, reads, read_off, ref, seeds, scoring):
        """Read-level seed extension from host memory (``bsw_extend_seeds``):
        reads/ref are uint8 code arrays, read_off the n_reads + 1 offsets,
        seeds a SEED_DTYPE array; returns SEED_RESULT_DTYPE records."""
        reads = np.ascontiguousarray(reads, dtype=np.uint8)
        read_off = np.ascontiguousarray(read_off, dtype=np.uint64)
        ref = np.ascontiguousarray(ref, dtype=np.uint8)
        seeds = np.ascontiguousarray(seeds, dtype=SEED_DTYPE)
        out = np.zeros(len(seeds), dtype=SEED_RESULT_DTYPE)
        params = make_params([scoring])
        _check(lib().bsw_extend_seeds(
            self._h, _ptr(reads), read_off.ctypes.data, len(read_off) - 1, _ptr(ref),
            len(ref), _ptr(seeds), len(seeds), params, _ptr(out)))
        return out

    def extend_seeds_device(self, dev, scoring, out, stream=None, async_=False):
        """Device form (``bsw_extend_seeds_device``): ``dev`` as made by
        ``seeds_to_device``; ``out`` a torch tensor of n*32 bytes."""
        n = dev["seeds"].numel() // SEED_DTYPE.itemsize
        params = make_params([scoring])
        rev = dev.get("ref_rev")
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_extend_seeds_device(
            self._h, dev["reads"].data_ptr(), dev["reads"].numel(),
            dev["read_off"].data_ptr(), dev["read_off"].numel() - 1,
            dev["ref"].data_ptr(), rev.data_ptr() if rev is not None else None,
            dev["ref"].numel(), dev["seeds"].data_ptr(), n, params, out.data_ptr(), s,
            1 if async_ else 0))

    def filter_seeds_device(self, seeds, res, keep, stream=None, async_=False):
        """Keep flags after extending every seed (``bsw_filter_seeds_device``):
        seeds and res torch tensors of SEED_DTYPE / SEED_RESULT_DTYPE bytes,
        keep a uint8 tensor of one byte per seed."""
        n = seeds.numel() // SEED_DTYPE.itemsize
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_filter_seeds_device(self._h, seeds.data_ptr(), n, res.data_ptr(),
                                             keep.data_ptr(), s, 1 if async_ else 0))

    def tune_seeds(self, dev, scoring, out, reps=2):
        """Autotune the seed driver's launch shape on a device seed workload
        (as for ``extend_seeds_device``); returns (best_ms, shape dict)."""
        n = dev["seeds"].numel() // SEED_DTYPE.itemsize
        params = make_params([scoring])
        rev = dev.get("ref_rev")
        ms = ctypes.c_double(0)
        v = (ctypes.c_int32 * 3)()
        _check(lib().bsw_ctx_tune_seeds(
            self._h, dev["reads"].data_ptr(), dev["reads"].numel(),
            dev["read_off"].data_ptr(), dev["read_off"].numel() - 1,
            dev["ref"].data_ptr(), rev.data_ptr() if rev is not None else None,
            dev["ref"].numel(), dev["seeds"].data_ptr(), n, params, out.data_ptr(), reps,
            ctypes.byref(ms), v))
        return ms.value, {"side_streams": v[0], "occ8_pct": v[1], "spec16": v[2]}

    def sa_lookup_device(self, sa, iv, out_off, out_pos, stream=None, async_=False):
        """Suffix-array lookup (``bsw_sa_lookup_device``): sa an int64 tensor,
        iv a tensor of n*16 bytes (SA_INTERVAL_DTYPE records), out_off an
        int64 tensor of n + 1 entries, out_pos an int64 tensor (its length is
        the capacity).  Returns the number of coordinates (None if async)."""
        n = iv.numel() * iv.element_size() // SA_INTERVAL_DTYPE.itemsize
        tot = ctypes.c_uint64(0)
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_sa_lookup_device(
            self._h, sa.data_ptr(), sa.numel(), iv.data_ptr(), n, out_off.data_ptr(),
            out_pos.data_ptr() if out_pos is not None and out_pos.numel() else None,
            out_pos.numel() if out_pos is not None else 0, ctypes.byref(tot), s,
            1 if async_ else 0))
        return None if async_ else tot.value

    def fm_backward_search_device(self, entries, meta, pat, pat_off, out, stream=None,
                                  async_=False):
        """Backward search (``bsw_fm_backward_search_device``): entries the
        index (a GPU tensor of meta.entries * 64 bytes), pat a uint8 tensor,
        pat_off an int64 tensor of n + 1 offsets, out a tensor of n * 32
        bytes (BI_INTERVAL_DTYPE records)."""
        n = pat_off.numel() - 1
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_fm_backward_search_device(
            self._h, entries.data_ptr(), ctypes.byref(meta),
            pat.data_ptr() if pat.numel() else None, pat_off.data_ptr(), n, out.data_ptr(),
            s, 1 if async_ else 0))

    def fm_smem_device(self, entries, meta, reads, read_off, max_len, out, counts,
                       stream=None, async_=False):
        """SMEMs of every read (``bsw_fm_smem_device``): reads a uint8 tensor,
        read_off int64 (n + 1), out a tensor of (read bases) * 32 bytes
        (SMEM_DTYPE records, read r's at its own offset), counts int32 (n)."""
        n = read_off.numel() - 1
        s = stream.cuda_stream if stream is not None else None
        _check(lib().bsw_fm_smem_device(
            self._h, entries.data_ptr(), ctypes.byref(meta),
            reads.data_ptr() if reads.numel() else None, read_off.data_ptr(), n, max_len,
            out.data_ptr() if out.numel() else None, counts.data_ptr(), s,
            1 if async_ else 0))

    def last_cells(self):
        """Band cells settled by the last completed call (all its passes)."""
        v = ctypes.c_int64(0)
        _check(lib().bsw_ctx_last_cells(self._h, ctypes.byref(v)))
        return v.value

    def tune(self, dev, scorings, out, reps=2):
        """Autotune the batched path's launch shapes on a device batch;
        returns (best_ms, shape dict)."""
        n = dev["h0"].numel()
        params = make_params(scorings)
        pid = dev.get("param_id")
        ms = ctypes.c_double(0)
        _check(lib().bsw_ctx_tune(
            self._h, n, dev["q"].data_ptr(), dev["q_off"].data_ptr(),
            dev["t"].data_ptr(), dev["t_off"].data_ptr(), dev["h0"].data_ptr(),
            pid.data_ptr() if pid is not None else None, params, len(params),
            out.data_ptr(), reps, ctypes.byref(ms)))
        return ms.value, self.tune_info()

    def tune_info(self):
        """The context's launch shape for pair batches (``bsw_ctx_shape``)."""
        v = (ctypes.c_int32 * 4)()
        n = lib().bsw_ctx_shape(self._h, v, 4)
        if n < 0:
            _check(n)
        return {"side_streams": v[0], "occ8_pct": v[1], "spec16": v[2],
                "wave32_min_cap": v[3]}

    def last_kernels(self):
        """Per DP launch of the last call: list of (class name, cells, ms)."""
        cls = np.zeros(32, dtype=np.int32)
        cells = np.zeros(32, dtype=np.int64)
        ms = np.zeros(32, dtype=np.float64)
        n = lib().bsw_ctx_last_kernels(self._h, cls.ctypes.data, cells.ctypes.data,
                                       ms.ctypes.data, 32)
        if n < 0:
            _check(n)
        return [(lib().bsw_class_name(int(cls[k])).decode(), int(cells[k]), float(ms[k]))
                for k in range(min(n, 32))]

    def last_work(self):
        """Per DP launch of the last call (order of ``last_kernels``): the
        lane-cells it stepped through (``bsw_ctx_last_work``)."""
        work = np.zeros(32, dtype=np.int64)
        n = lib().bsw_ctx_last_work(self._h, work.ctypes.data, 32)
        if n < 0:
            _check(n)
        return [int(x) for x in work[:min(n, 32)]]

    def last_timing(self):
        """(pipeline_ms, prep_bin_ms, dp_ms, dp_launches) of the last call."""
        buf = (ctypes.c_double * 4)()
        _check(lib().bsw_ctx_last_timing(self._h, buf))
        return tuple(buf)


def to_device(batch, device="cuda"):
    """Copy a host batch's arrays into torch tensors on the GPU."""
    import torch
    dev = {}
    for k in ("q", "q_off", "t", "t_off", "h0", "param_id"):
        if k in batch and batch[k] is not None:
            a = np.ascontiguousarray(batch[k])
            if a.dtype == np.uint64:
                a = a.view(np.int64)
            dev[k] = torch.from_numpy(a).to(device)
    return dev


def fm_build(text, sa):
    """The FM-index of a text (codes 0..3) from its suffix array
    (``bsw_fm_build``, host memory): (entries, FmMeta)."""
    text = np.ascontiguousarray(text, dtype=np.uint8)
    sa = np.ascontiguousarray(sa, dtype=np.int64)
    rows = len(text) + 1
    entries = np.zeros((rows + 31) // 32, dtype=FM_ENTRY_DTYPE)
    meta = FmMeta()
    _check(lib().bsw_fm_build(_ptr(text), len(text), sa.ctypes.data, entries.ctypes.data,
                              ctypes.byref(meta)))
    return entries, meta


def seeds_to_device(reads, read_off, ref, seeds, device="cuda", with_ref_rev=False):
    """Copy a seed workload (host arrays) into torch tensors on the GPU; the
    reversed reference is made on the host when asked for."""
    import torch
    dev = {"reads": torch.from_numpy(np.ascontiguousarray(reads, dtype=np.uint8)).to(device),
           "read_off": torch.from_numpy(
               np.ascontiguousarray(read_off, dtype=np.uint64).view(np.int64)).to(device),
           "ref": torch.from_numpy(np.ascontiguousarray(ref, dtype=np.uint8)).to(device),
           "seeds": torch.from_numpy(
               np.ascontiguousarray(seeds, dtype=SEED_DTYPE).view(np.uint8)).to(device)}
    if with_ref_rev:
        rev = np.ascontiguousarray(np.asarray(ref, dtype=np.uint8)[::-1])
        dev["ref_rev"] = torch.from_numpy(rev).to(device)
    return dev


def alloc_outputs(n, device="cuda", with_diag=False):
    import torch
    out = torch.empty(n * RESULT_DTYPE.itemsize, dtype=torch.uint8, device=device)
    diag = (torch.empty(n * DIAG_DTYPE.itemsize, dtype=torch.uint8, device=device)
            if with_diag else None)
    return out, diag


def outputs_to_numpy(out, diag=None):
    r = out.cpu().numpy().view(RESULT_DTYPE)
    if diag is None:
        return r
    return r, diag.cpu().numpy().view(DIAG_DTYPE)


class Server:
    """Serving loop of the library (bsw_server_*): requests are submitted
    from host memory, admitted in arrival order under the device budget and
    run in batches formed from every resident request when a slot frees."""

    def __init__(self, scorings, device=0, max_inflight=0, max_batch_pairs=0,
                 hbm_budget=0, max_queued=0, min_lane_bits=0):
        o = ServerOpts(device, max_inflight, max_batch_pairs, hbm_budget, max_queued,
                       min_lane_bits)
        params = make_params(scorings)
        h = _VP()
        _check(lib().bsw_server_create(ctypes.byref(h), ctypes.byref(o), params,
                                       len(params)))
        self._h = h
        self._live = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().bsw_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, batch, with_diag=False):
        """Submit a host batch (see ``synth``); returns a ticket."""
        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            return a if a.size else np.zeros(1, dtype=dt)
        q = arr(batch["q"], np.uint8)
        t = arr(batch["t"], np.uint8)
        qo = np.ascontiguousarray(batch["q_off"], dtype=np.uint64)
        to = np.ascontiguousarray(batch["t_off"], dtype=np.uint64)
        h0 = np.ascontiguousarray(batch["h0"], dtype=np.int32)
        pid = batch.get("param_id")
        pid = None if pid is None else np.ascontiguousarray(pid, dtype=np.uint8)
        n = len(h0)
        out = np.zeros(n, dtype=RESULT_DTYPE)
        diag = np.zeros(n, dtype=DIAG_DTYPE) if with_diag else None
        tk = ctypes.c_uint64(0)
        _check(lib().bsw_server_submit(
            self._h, n, q.ctypes.data, qo.ctypes.data, t.ctypes.data, to.ctypes.data,
            h0.ctypes.data, _ptr(pid), out.ctypes.data, _ptr(diag), ctypes.byref(tk)))
        # the library reads these buffers until the request completes
        self._live[tk.value] = (q, t, qo, to, h0, pid, out, diag)
        return tk.value

    def wait(self, ticket, timeout_ms=-1):
        """Results (and diagnostics if asked at submit) of a ticket."""
        rc = lib().bsw_server_wait(self._h, ticket, timeout_ms)
        if rc == ETIMEOUT:
            raise BswError(rc, last_error())
        keep = self._live.pop(ticket, None)
        _check(rc)
        out, diag = keep[6], keep[7]
        return (out, diag) if diag is not None else out

    def stats(self, reset=False):
        r = ServerReport()
        _check(lib().bsw_server_stats(self._h, ctypes.byref(r), 1 if reset else 0))
        return {k: getattr(r, k) for k, _ in ServerReport._fields_}
