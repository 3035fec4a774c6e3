"""ctypes declarations of libptsbe.so (the C ABI in include/ptsbe.h).

The library is loaded from this package directory.  There is no fallback: if
the shared object is missing the import of any entry point raises, naming the
build command.
"""

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PTSBE_LIB selects another build of the same library (the host-sanitized one of
# `python -m paper_2504_16297_amd.build --sanitize`, for CPU test runs)
LIB_PATH = os.environ.get("PTSBE_LIB") or os.path.join(_HERE, "libptsbe.so")

PTSBE_OK = 0
STATUS_NAMES = {0: "PTSBE_OK", 1: "PTSBE_E_ARG", 2: "PTSBE_E_NOT_CPTP", 3: "PTSBE_E_UNSUPPORTED",
                4: "PTSBE_E_CAPACITY", 5: "PTSBE_E_OOM", 6: "PTSBE_E_DEVICE", 7: "PTSBE_E_NONDET_MEASURE"}

OP_GATE, OP_PARAM, OP_NOISE, OP_MEASURE_RESET, OP_PROJECT0 = range(5)
GEN = {"X": 1, "Y": 2, "Z": 3}
ATTACH_AFTER_TAG, ATTACH_BEFORE_MEASURE, ATTACH_BEFORE_READOUT = range(3)
C64, C128 = 0, 1
PTS_MODES = {"proportional": 0, "alg2_literal": 1, "most_likely": 2, "per_shot": 3}
ALLOCS = {"multiplicity": 0, "reweight": 1, "uniform": 2}
RUN_SHOTS, RUN_STATES, RUN_EXPECTATION, RUN_ADJOINT = range(4)
RUN_NO_PREFIX_SHARING = 1
RUN_NO_SUPPORT_LISTS = 2
PLAN_NO_COMPILE = 8
PLAN_HALF_TILE_LDS = 16
PLAN_NO_PHASE_FRAMES = 32
PLAN_WAVES_SHIFT = 8
PLAN_TWIRL = 64
PLAN_NO_PAIR_FUSION = 128
PLAN_NO_SWIZZLE = 4096
PLAN_NONTEMPORAL = 16384
PLAN_TWO_TILES = 32768
PLAN_SWIZZLE = 8192
SWIZZLE_MIN_QUBITS = 22
PLAN_NO_TILE_SEARCH = 65536
NOALLOC_SCRATCH_BYTES = 64 << 20


class Op(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("nq", C.c_uint32), ("q", C.c_uint32 * 4),
                ("mat", C.POINTER(C.c_double)), ("index", C.c_int32), ("gen", C.c_uint32),
                ("tag", C.c_uint32), ("reserved", C.c_uint32)]


class Circuit(C.Structure):
    _fields_ = [("n_qubits", C.c_uint32), ("n_ops", C.c_uint32), ("ops", C.POINTER(Op))]


class Channel(C.Structure):
    _fields_ = [("nq", C.c_uint32), ("n_kraus", C.c_uint32), ("kraus", C.POINTER(C.c_double))]


class Attach(C.Structure):
    _fields_ = [("when", C.c_uint32), ("tag", C.c_uint32), ("channel", C.c_uint32),
                ("reserved", C.c_uint32), ("qmask", C.c_uint64)]


class NoiseModel(C.Structure):
    _fields_ = [("n_channels", C.c_uint32), ("channels", C.POINTER(Channel)),
                ("n_rules", C.c_uint32), ("rules", C.POINTER(Attach))]


class PlanOpts(C.Structure):
    _fields_ = [("precision", C.c_uint32), ("tile_qubits", C.c_uint32), ("flags", C.c_uint32),
                ("reserved", C.c_uint32)]


class PlanInfo(C.Structure):
    _fields_ = [(f, C.c_uint32) for f in ("n_qubits", "n_sites", "n_params", "n_measure", "n_passes",
                                          "n_steps", "precision", "tile_qubits", "max_kraus",
                                          "total_kraus", "swizzled")]


class PtsOpts(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("alloc", C.c_uint32), ("n_draws", C.c_uint64),
                ("k_max", C.c_uint64), ("total_shots", C.c_uint64), ("nshots", C.c_uint64),
                ("seed", C.c_uint64), ("cfg", C.c_uint32), ("stream", C.c_uint32),
                ("p_min", C.c_double), ("p_max", C.c_double),
                ("kraus_allow", C.c_void_p), ("min_errors", C.c_uint32), ("max_errors", C.c_uint32),
                ("error_parity", C.c_uint32), ("reserved", C.c_uint32)]


PARITY = {None: 0, "any": 0, "even": 1, "odd": 2}
SITE_ORIGINS = ("noise_op", "after_tag", "before_measure", "before_readout")


class SiteFilter(C.Structure):
    _fields_ = [("tags", C.c_void_p), ("n_tags", C.c_uint32), ("qubits", C.c_void_p), ("n_qubits", C.c_uint32),
                ("ops", C.c_void_p), ("n_ops", C.c_uint32), ("origins", C.c_void_p), ("n_origins", C.c_uint32),
                ("kraus", C.c_void_p), ("n_kraus", C.c_uint32)]


class RunOpts(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("cfg", C.c_uint32), ("seed", C.c_uint64),
                ("sort_chunk", C.c_uint32), ("max_batch", C.c_uint32),
                ("d_uniforms", C.c_void_p), ("params", C.POINTER(C.c_double)),
                ("d_state_out", C.c_void_p), ("d_expval", C.c_void_p),
                ("obs_coef", C.POINTER(C.c_double)), ("obs_zmask", C.POINTER(C.c_uint64)),
                ("n_terms", C.c_uint32), ("flags", C.c_uint32),
                ("timing", C.POINTER(C.c_double)), ("d_ensemble", C.c_void_p)]


_lib = None

_SIGS = {
    "ptsbe_last_error": (C.c_char_p, []),
    "ptsbe_version": (C.c_char_p, []),
    "ptsbe_plan": (C.c_int, [C.POINTER(Circuit), C.POINTER(NoiseModel), C.POINTER(PlanOpts),
                             C.POINTER(C.c_void_p)]),
    "ptsbe_plan_get_info": (C.c_int, [C.c_void_p, C.POINTER(PlanInfo)]),
    "ptsbe_plan_get_sites": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_plan_destroy": (None, [C.c_void_p]),
    "ptsbe_sample_kraus": (C.c_int, [C.c_void_p, C.POINTER(PtsOpts), C.POINTER(C.c_void_p)]),
    "ptsbe_trajset_from_records": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                             C.c_void_p, C.c_void_p, C.c_uint64,
                                             C.POINTER(C.c_void_p)]),
    "ptsbe_trajset_slice": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(C.c_void_p)]),
    "ptsbe_trajset_get": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_uint32), C.POINTER(C.c_uint64), C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_trajset_destroy": (None, [C.c_void_p]),
    "ptsbe_trajset_weights": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ptsbe_site_selection": (C.c_int, [C.c_void_p, C.POINTER(SiteFilter), C.c_void_p]),
    "ptsbe_workspace_size": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RunOpts),
                                       C.POINTER(C.c_size_t)]),
    "ptsbe_run_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RunOpts), C.c_void_p,
                                  C.c_size_t, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                  C.c_void_p]),
    "ptsbe_run_status": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_run_batch_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RunOpts), C.c_void_p,
                                          C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_pauli_twirl": (C.c_int, [C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p]),
    "ptsbe_plan_get_record_info": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_plan_get_site_ops": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_unique_workspace_size": (C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(C.c_size_t)]),
    "ptsbe_unique_shots": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "ptsbe_graph_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(RunOpts), C.c_void_p,
                                     C.c_size_t, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                     C.c_void_p, C.POINTER(C.c_void_p)]),
    "ptsbe_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "ptsbe_graph_destroy": (None, [C.c_void_p]),
    "ptsbe_trajset_tables": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_uint32, C.c_void_p,
                                       C.POINTER(C.c_size_t), C.c_void_p]),
    "ptsbe_plan_compile": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_double)]),
    "ptsbe_plan_pass_source": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_char_p,
                                         C.POINTER(C.c_size_t)]),
    "ptsbe_trajset_adjoint_tables": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p,
                                               C.POINTER(C.c_size_t), C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_adjoint_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.c_uint32,
                                     C.c_uint64, C.c_uint32,
                                     C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ptsbe_std_gate": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(C.c_uint32)]),
    "ptsbe_std_channel": (C.c_int, [C.c_char_p, C.c_uint32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_uint32)]),
}

EXPORTED = tuple(_SIGS)


def lib():
    global _lib
    if _lib is None:
        # torch first: its HIP runtime (SONAME libamdhip64.so.7) is then the one the
        # library binds to, so streams and device pointers from torch are valid in
        # it; loaded the other way round the process would hold two HIP runtimes
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2504_16297_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class PtsbeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status):
    if status != PTSBE_OK:
        raise PtsbeError(status, lib().ptsbe_last_error().decode())
