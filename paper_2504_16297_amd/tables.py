"""Host-side view of the device tables a trajectory set uploads (fused tile
passes, ops, slot matrices, per-trajectory overrides, execution steps), as
exported by ptsbe_trajset_tables / ptsbe_trajset_adjoint_tables, plus the
useful-work count of each pass used to place the tile-pass kernel on its
arithmetic roofline.  Inspection only: nothing here runs on the hot path."""

import ctypes as C

import numpy as np

from . import _lib as L
from ._lib import check

PASS_DT = np.dtype([("k", "<u4"), ("n_ops", "<u4"), ("op_begin", "<u4"), ("slot_begin", "<u4"),
                    ("n_slots", "<u4"), ("flags", "<u4"), ("tq", "u1", 16), ("oq", "u1", 48)])
OP_DT = np.dtype([("type", "u1"), ("a", "u1"), ("b", "u1"), ("ga", "u1"), ("gb", "u1"), ("mask", "u1"),
                  ("pad0", "u1"), ("pad1", "u1"), ("slots", "<u2", 4)])
OV_DT = np.dtype([("slot", "<u4"), ("off", "<u4")])
EXEC_DT = np.dtype([("pass", "<u4"), ("nq", "<u4"), ("q", "<u4", 16), ("idx", "<u4", 16)])
M1, M2, D1, D2, MR, DSIGN, PHASE, M1G, SFLIP, DOT = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10

def _ptr(params):
    if params is None or not len(params):
        return None, None
    pa = np.ascontiguousarray(params, dtype=np.float64)
    return pa, C.cast(pa.ctypes.data, C.POINTER(C.c_double))


def decode(ts, buf, offs):
    o = [int(x) for x in offs]
    prec = ts.plan.info["precision"]
    cdt = np.complex64 if prec == L.C64 else np.complex128
    B = ts.n_traj
    return {
        "passes": np.frombuffer(buf, PASS_DT, o[9], o[0]),
        "ops": np.frombuffer(buf, OP_DT, o[10], o[1]),
        "slot_default": np.frombuffer(buf, "<u4", o[11], o[2]),
        "pool": np.frombuffer(buf, cdt, o[12], o[3]).astype(np.complex128),
        "ov_off": np.frombuffer(buf, "<u4", B * o[9] + 1, o[4]),
        "ov": np.frombuffer(buf, OV_DT, o[13], o[5]),
        "shot_off": np.frombuffer(buf, "<u8", B + 1, o[6]),
        "chunk_off": np.frombuffer(buf, "<u8", B + 1, o[7]),
        "exec": np.frombuffer(buf, EXEC_DT, o[14], o[8]),
    }


def export_tables(ts, params=None, sort_chunk=0):
    """Decoded forward tables of a trajectory set."""
    keep, pp = _ptr(params)
    n = C.c_size_t()
    offs = np.zeros(16, dtype=np.uint64)
    check(L.lib().ptsbe_trajset_tables(ts.handle, pp, sort_chunk, None, C.byref(n), offs.ctypes.data))
    buf = np.zeros(n.value, dtype=np.uint8)
    check(L.lib().ptsbe_trajset_tables(ts.handle, pp, sort_chunk, buf.ctypes.data, C.byref(n), offs.ctypes.data))
    del keep
    return decode(ts, buf, offs)


def export_adjoint_tables(ts, params):
    """(decoded tables of the reverse-sweep program, gradient term -> parameter index)."""
    keep, pp = _ptr(params)
    n = C.c_size_t()
    offs = np.zeros(16, dtype=np.uint64)
    nd = C.c_uint32()
    check(L.lib().ptsbe_trajset_adjoint_tables(ts.handle, pp, None, C.byref(n), offs.ctypes.data, C.byref(nd),
                                               None))
    buf = np.zeros(n.value, dtype=np.uint8)
    dp = np.zeros(max(1, nd.value), dtype=np.uint32)
    check(L.lib().ptsbe_trajset_adjoint_tables(ts.handle, pp, buf.ctypes.data, C.byref(n), offs.ctypes.data,
                                               C.byref(nd), dp.ctypes.data))
    del keep
    return decode(ts, buf, offs), dp[:nd.value]
