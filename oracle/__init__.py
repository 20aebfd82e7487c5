"""CPU oracle for banded Smith-Waterman seed extension (BSW).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by ``smoke()`` in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``; the
product package never imports it, and this package never imports the
product.  Three independent formulations live here:

* ``libbsw_ref.so`` (``bsw_ref.c``): the plain scalar C oracle, one row
  buffer, the method's steps in the paper's order (Sec. 5.1, Eq. (2),(3)).
* ``model2d``: a NumPy full-matrix re-statement of the same rules with
  explicit H/E matrices, last-write resolution of the row buffer and a
  closed-form F, used to pin the C oracle's band bookkeeping.
* ``brute``: exhaustive enumeration of alignment paths on tiny inputs, used
  to pin the recurrence and boundaries where no heuristic fires.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsw_ref.so")
SRC = os.path.join(HERE, "bsw_ref.c")

STOP_END, STOP_ZERO, STOP_ZDROP = 0, 1, 2


class Params(ctypes.Structure):
    """Mirror of ``bsw_ref_params`` (see bsw_ref.h)."""

    _fields_ = [
        ("mat", ctypes.c_int8 * 25),
        ("pad_", ctypes.c_int8 * 3),
        ("o_del", ctypes.c_int32),
        ("e_del", ctypes.c_int32),
        ("o_ins", ctypes.c_int32),
        ("e_ins", ctypes.c_int32),
        ("w", ctypes.c_int32),
        ("zdrop", ctypes.c_int32),
        ("end_bonus", ctypes.c_int32),
    ]


RESULT_DTYPE = np.dtype(
    [("score", "<i4"), ("qle", "<i4"), ("tle", "<i4"), ("gtle", "<i4"),
     ("gscore", "<i4"), ("max_off", "<i4")])
DIAG_DTYPE = np.dtype([("rows", "<i4"), ("stop", "<i4"), ("cells", "<i8")])


def build(force: bool = False) -> str:
    """Compile libbsw_ref.so with the host C compiler (-O2, no intrinsics)."""
    if force or not os.path.exists(LIB_PATH) or (
            os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC)):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-Wall",
             "-Wextra", "-shared", "-fPIC", "-o", tmp, SRC, "-lpthread"],
            check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.bsw_ref_extend_batch.restype = ctypes.c_int
        L.bsw_ref_extend_batch.argtypes = [
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        L.bsw_ref_extend_one.restype = ctypes.c_int
        L.bsw_ref_extend_one.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
            ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
            ctypes.c_void_p]
        L.bsw_ref_extend_one_bits.restype = ctypes.c_int
        L.bsw_ref_extend_one_bits.argtypes = [
            ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
            ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_int32]
        _lib = L
    return _lib


def make_params(scoring) -> Params:
    """Build a ``Params`` from a mapping with keys mat (5x5 or 25 ints),
    o_del, e_del, o_ins, e_ins, w, zdrop, end_bonus."""
    p = Params()
    mat = np.asarray(scoring["mat"], dtype=np.int64).reshape(25)
    for k in range(25):
        p.mat[k] = int(mat[k])
    for name in ("o_del", "e_del", "o_ins", "e_ins", "w", "zdrop", "end_bonus"):
        setattr(p, name, int(scoring[name]))
    return p


class OracleError(RuntimeError):
    def __init__(self, code, bad_index):
        super().__init__(f"oracle rejected the batch (status {code}, pair {bad_index})")
        self.code = code
        self.bad_index = bad_index


def extend_batch(batch, scorings, n_threads: int = 0):
    """Run the C oracle on a batch.

    ``batch`` holds numpy arrays q (u8), q_off (u64, n+1), t (u8), t_off
    (u64, n+1), h0 (i32), and optionally param_id (u8).  ``scorings`` is a
    list of scoring mappings.  Returns (results, diags) as structured arrays.
    """
    q = np.ascontiguousarray(batch["q"], dtype=np.uint8)
    t = np.ascontiguousarray(batch["t"], dtype=np.uint8)
    q_off = np.ascontiguousarray(batch["q_off"], dtype=np.uint64)
    t_off = np.ascontiguousarray(batch["t_off"], dtype=np.uint64)
    h0 = np.ascontiguousarray(batch["h0"], dtype=np.int32)
    pid = batch.get("param_id")
    if pid is not None:
        pid = np.ascontiguousarray(pid, dtype=np.uint8)
    n = len(h0)
    if n_threads <= 0:
        # the CPUs this process may use, at most 16 (a one-GPU host share)
        try:
            n_threads = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            n_threads = min(16, os.cpu_count() or 1)
    params = (Params * len(scorings))(*[make_params(s) for s in scorings])
    out = np.zeros(n, dtype=RESULT_DTYPE)
    diag = np.zeros(n, dtype=DIAG_DTYPE)
    bad = ctypes.c_int64(-1)
    # numpy arrays of length 0 still have a valid (non-null) data pointer
    rc = lib().bsw_ref_extend_batch(
        n, q.ctypes.data if len(q) else None, q_off.ctypes.data,
        t.ctypes.data if len(t) else None, t_off.ctypes.data, h0.ctypes.data,
        pid.ctypes.data if pid is not None else None, params, len(scorings),
        out.ctypes.data, diag.ctypes.data, int(n_threads), ctypes.byref(bad))
    if rc != 0:
        raise OracleError(rc, bad.value)
    return out, diag


def extend_one(q, t, h0, scoring, bits=32):
    """Convenience wrapper for a single pair given as code sequences; bits
    = 8 or 16 runs it in saturating lanes of that width."""
    q = np.ascontiguousarray(np.asarray(q, dtype=np.uint8))
    t = np.ascontiguousarray(np.asarray(t, dtype=np.uint8))
    out = np.zeros(1, dtype=RESULT_DTYPE)
    diag = np.zeros(1, dtype=DIAG_DTYPE)
    p = make_params(scoring)
    args = (len(q), q.ctypes.data if len(q) else None, len(t),
            t.ctypes.data if len(t) else None, int(h0), ctypes.byref(p),
            out.ctypes.data, diag.ctypes.data)
    rc = (lib().bsw_ref_extend_one(*args) if bits == 32
          else lib().bsw_ref_extend_one_bits(*args, int(bits)))
    if rc != 0:
        raise OracleError(rc, 0)
    r = out[0]
    return (tuple(int(r[k]) for k in RESULT_DTYPE.names),
            tuple(int(diag[0][k]) for k in DIAG_DTYPE.names))
