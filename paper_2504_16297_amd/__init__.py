"""PTSBE on MI355X: Python binding of libptsbe (include/ptsbe.h).

Argument marshalling only: circuits described as plain dictionaries (see
``workloads``) are turned into the C structures of the ABI, torch tensors are
passed as raw device pointers with torch's current HIP stream, and every step
of planning, pre-trajectory sampling and batched execution runs inside the
library (host planner in C++, hot path in gfx950 HIP kernels).
"""

import ctypes as C
import zlib

import numpy as np

from . import _lib as L
from ._lib import PtsbeError, lib, check

__all__ = ["ptsbe_plan", "ptsbe_plan_compile", "ptsbe_sample_kraus", "ptsbe_trajset_from_records",
           "ptsbe_workspace_size", "ptsbe_run_batch", "ptsbe_run_status", "ptsbe_unique_workspace_size",
           "ptsbe_unique_shots", "ptsbe_adjoint_grad", "site_selection", "pauli_twirl", "std_gate",
           "std_channel", "Plan", "TrajSet", "RunGraph", "PtsbeError", "tag_id"]


def tag_id(tag):
    return zlib.crc32(str(tag).encode()) & 0xFFFFFFFF


def _dptr(a):
    return C.cast(a.ctypes.data, C.POINTER(C.c_double))


def std_gate(name, params=()):
    out = np.zeros(32, dtype=np.float64)
    p = np.asarray(params, dtype=np.float64) if len(params) else np.zeros(1)
    nq = C.c_uint32()
    check(lib().ptsbe_std_gate(name.encode(), _dptr(p), _dptr(out), C.byref(nq)))
    d = 1 << nq.value
    return out[:2 * d * d].copy(), nq.value


def std_channel(ch):
    """(interleaved complex128 Kraus operators, nq, n_kraus) of a channel given by
    name, or by an explicit ``{"kraus": [K_0, K_1, ...]}`` list of matrices."""
    if "kraus" in ch:
        ks = [np.asarray(k, dtype=np.complex128) for k in ch["kraus"]]
        d = ks[0].shape[0]
        nq = d.bit_length() - 1
        flat = np.concatenate([k.reshape(-1) for k in ks])
        out = np.empty(2 * flat.size, dtype=np.float64)
        out[0::2], out[1::2] = flat.real, flat.imag
        return out, nq, len(ks)
    name = ch["name"]
    if name in ("depolarizing", "xflip"):
        p = [ch["p"]]
    elif name == "pauli":
        p = list(ch["probs"])
    elif name == "u3_mixture":
        p = [ch["p"]] + list(ch["params"])
    elif name == "amplitude_damping":
        p = [ch["gamma"]]
    else:
        raise ValueError(name)
    nq = int(ch.get("nq", 1))
    out = np.zeros(16 * 2 * 16, dtype=np.float64)
    pa = np.asarray(p, dtype=np.float64)
    nk = C.c_uint32()
    check(lib().ptsbe_std_channel(name.encode(), nq, _dptr(pa), _dptr(out), C.byref(nk)))
    d = 1 << nq
    return out[:2 * d * d * nk.value].copy(), nq, nk.value


class Plan:
    """Owning wrapper of a ptsbe_plan_t."""

    def __init__(self, handle, keep):
        self.handle = handle
        self._keep = keep
        info = L.PlanInfo()
        check(lib().ptsbe_plan_get_info(handle, C.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in L.PlanInfo._fields_}

    def site_probs(self):
        ns = self.info["n_sites"]
        off = np.zeros(ns + 1, dtype=np.uint32)
        p = np.zeros(max(1, self.info["total_kraus"]), dtype=np.float64)
        q = np.zeros(max(1, 2 * ns), dtype=np.uint32)
        check(lib().ptsbe_plan_get_sites(self.handle, off.ctypes.data, p.ctypes.data, q.ctypes.data))
        return [p[off[s]:off[s + 1]].copy() for s in range(ns)], q[:2 * ns].reshape(-1, 2)

    def record_info(self):
        """Per record entry: (channel index or -1 for a measure-reset, uniform word)."""
        nm = self.info["n_measure"]
        ch = np.zeros(max(1, nm), dtype=np.uint32)
        gi = np.zeros(max(1, nm), dtype=np.uint32)
        check(lib().ptsbe_plan_get_record_info(self.handle, C.c_void_p(ch.ctypes.data), C.c_void_p(gi.ctypes.data)))
        return [(-1 if c == 0xFFFFFFFF else int(c), int(g)) for c, g in zip(ch[:nm], gi[:nm])]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib().ptsbe_plan_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


def ptsbe_plan_compile(plan):
    """Compile the plan's tile passes now (else the first run does); returns
    (number of kernels, seconds)."""
    nk = C.c_uint32()
    sec = C.c_double()
    check(lib().ptsbe_plan_compile(plan.handle, C.byref(nk), C.byref(sec)))
    return nk.value, sec.value


def ptsbe_plan(circuit, precision="c64", tile_qubits=0, compile=True, min_fill=0, half_tile=False,
               phase_frames=True, waves=0, twirl=False, pair_fusion=True, swizzle=None, nontemporal=False,
               two_tiles=False, tile_search=True):
    """Build the execution plan of a circuit dictionary (ops, channels, rules).
    ``compile=False`` runs the passes through the generic tile kernels instead of
    per-pass compiled kernels; ``min_fill`` (1..7, 0 = 2) is the fewest 2x2
    matrices a partial register group must hold; ``half_tile`` moves amplitudes
    between register sets through half a tile of LDS; ``phase_frames=False``
    keeps every slot matrix as it is (no pending diagonals between matrices);
    ``waves`` (1..8, 0 = compiler's choice for the forward passes, three for
    the adjoint's reverse sweep) sets the compiled passes' register budget to
    512 / waves VGPRs; ``twirl`` replaces channels that are not unitary
    mixtures by their Pauli twirl (else they are rejected); ``pair_fusion=False``
    keeps diagonal 2-qubit gates apart from the 2x2 runs on their qubits; ``swizzle``: None
    stores states of PTSBE_SWIZZLE_MIN_QUBITS qubits or more swizzled, True every state above
    12 qubits (PTSBE_PLAN_SWIZZLE), False none (PTSBE_PLAN_NO_SWIZZLE); ``nontemporal`` gives
    the compiled passes' state loads and stores streaming cache hints; ``two_tiles`` has each
    workgroup of a compiled forward pass run two tiles (PTSBE_PLAN_TWO_TILES);
    ``tile_search=False`` builds every tile greedily in circuit order only
    (PTSBE_PLAN_NO_TILE_SEARCH)."""
    ops = circuit["ops"]
    arr = (L.Op * max(1, len(ops)))()
    keep = []
    for i, op in enumerate(ops):
        o = arr[i]
        qs = tuple(op["qubits"])
        o.nq = len(qs)
        for j, q in enumerate(qs):
            o.q[j] = int(q)
        kind = op["kind"]
        if kind == "gate":
            m, nq = std_gate(op["name"], op.get("params", ()))
            if nq != len(qs):
                raise ValueError(f"op {i}: {op['name']} acts on {nq} qubits")
            keep.append(m)
            o.kind = L.OP_GATE
            o.mat = _dptr(m)
            o.tag = tag_id(op.get("tag", op["name"]))
        elif kind == "param":
            o.kind = L.OP_PARAM
            o.index = int(op["index"])
            o.gen = L.GEN[op["gen"]]
            o.tag = tag_id(op.get("tag", "R" + op["gen"]))
        elif kind == "noise":
            o.kind = L.OP_NOISE
            o.index = int(op["channel"])
        elif kind == "measure_reset":
            o.kind = L.OP_MEASURE_RESET
        elif kind == "project0":
            o.kind = L.OP_PROJECT0
        else:
            raise ValueError(kind)
    chans = circuit.get("channels", [])
    carr = (L.Channel * max(1, len(chans)))()
    for i, ch in enumerate(chans):
        k, nq, nk = std_channel(ch)
        keep.append(k)
        carr[i].nq = nq
        carr[i].n_kraus = nk
        carr[i].kraus = _dptr(k)
    rules = circuit.get("rules", [])
    rarr = (L.Attach * max(1, len(rules)))()
    for i, r in enumerate(rules):
        w = r["when"]
        rarr[i].channel = int(r["channel"])
        if w == "after_tag":
            rarr[i].when = L.ATTACH_AFTER_TAG
            rarr[i].tag = tag_id(r["tag"])
        elif w == "before_measure":
            rarr[i].when = L.ATTACH_BEFORE_MEASURE
        elif w == "before_readout":
            rarr[i].when = L.ATTACH_BEFORE_READOUT
            mask = 0
            for q in r["qubits"]:
                mask |= 1 << int(q)
            rarr[i].qmask = mask
        else:
            raise ValueError(w)
    c = L.Circuit(circuit["n_qubits"], len(ops), arr)
    nm = L.NoiseModel(len(chans), carr, len(rules), rarr)
    if not 0 <= int(min_fill) <= 7:
        raise ValueError("min_fill must be in 0..7")
    if not 0 <= int(waves) <= 8:
        raise ValueError("waves must be in 0..8")
    po = L.PlanOpts({"c64": L.C64, "c128": L.C128}[precision], int(tile_qubits),
                    int(min_fill) | (0 if compile else L.PLAN_NO_COMPILE) |
                    (L.PLAN_HALF_TILE_LDS if half_tile else 0) |
                    (0 if phase_frames else L.PLAN_NO_PHASE_FRAMES) | (int(waves) << L.PLAN_WAVES_SHIFT) |
                    (L.PLAN_TWIRL if twirl else 0) | (0 if pair_fusion else L.PLAN_NO_PAIR_FUSION) |
                    ({None: 0, True: L.PLAN_SWIZZLE, False: L.PLAN_NO_SWIZZLE}[swizzle]) |
                    (L.PLAN_NONTEMPORAL if nontemporal else 0) | (L.PLAN_TWO_TILES if two_tiles else 0) |
                    (0 if tile_search else L.PLAN_NO_TILE_SEARCH), 0)
    h = C.c_void_p()
    check(lib().ptsbe_plan(C.byref(c), C.byref(nm), C.byref(po), C.byref(h)))
    return Plan(h, None)


class TrajSet:
    """Owning wrapper of a ptsbe_trajset_t (PTS output: records, m_alpha, p_alpha)."""

    def __init__(self, handle, plan):
        self.handle = handle
        self.plan = plan

    def get(self):
        n = C.c_uint32()
        tot = C.c_uint64()
        ne = C.c_uint32()
        a0 = C.c_uint64()
        check(lib().ptsbe_trajset_get(self.handle, C.byref(n), C.byref(tot), C.byref(ne), C.byref(a0),
                                      None, None, None, None, None, None))
        B = n.value
        m = np.zeros(max(1, B), dtype=np.uint64)
        p = np.zeros(max(1, B), dtype=np.float64)
        cnt = np.zeros(max(1, B), dtype=np.uint64)
        off = np.zeros(B + 1, dtype=np.uint32)
        site = np.zeros(max(1, ne.value), dtype=np.uint32)
        kr = np.zeros(max(1, ne.value), dtype=np.uint8)
        check(lib().ptsbe_trajset_get(self.handle, None, None, None, None, m.ctypes.data, p.ctypes.data,
                                      cnt.ctypes.data, off.ctypes.data, site.ctypes.data, kr.ctypes.data))
        recs = [tuple((int(site[j]), int(kr[j])) for j in range(off[a], off[a + 1])) for a in range(B)]
        return {"records": recs, "m": m[:B], "p": p[:B], "count": cnt[:B], "total_shots": tot.value,
                "alpha0": a0.value, "rec_off": off, "rec_site": site[:ne.value], "rec_kraus": kr[:ne.value]}

    @property
    def n_traj(self):
        n = C.c_uint32()
        check(lib().ptsbe_trajset_get(self.handle, C.byref(n), None, None, None, None, None, None, None,
                                      None, None))
        return n.value

    def weights(self):
        """Ensemble weights w_alpha (ptsbe_trajset_weights), float64 [n_traj]."""
        B = self.n_traj
        w = np.zeros(max(1, B), dtype=np.float64)
        check(lib().ptsbe_trajset_weights(self.handle, w.ctypes.data))
        return w[:B]

    def slice(self, begin, end):
        h = C.c_void_p()
        check(lib().ptsbe_trajset_slice(self.handle, begin, end, C.byref(h)))
        return TrajSet(h, self.plan)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib().ptsbe_trajset_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


def ptsbe_sample_kraus(plan, mode="proportional", n_draws=0, k_max=0, total_shots=0, nshots=0, seed=0,
                       cfg=0, alloc=None, stream=0, p_band=None, kraus_allow=None, min_errors=0, max_errors=0,
                       parity=None):
    """Pre-trajectory sampling (Sec. 3.1) with the library's samplers.  Selection
    criteria: ``kraus_allow`` (one flag per (site, Kraus index) in the order of
    plan.site_probs(); see site_selection), ``min_errors`` / ``max_errors``
    (0 = no limit) on the number of non-identity operators of a record, and
    ``parity`` ("even" / "odd") of that number."""
    if alloc is None:
        alloc = {"proportional": "multiplicity", "alg2_literal": "uniform", "most_likely": "reweight",
                 "per_shot": "multiplicity"}[mode]
    allow = None
    if kraus_allow is not None:
        allow = np.ascontiguousarray(kraus_allow, dtype=np.uint8)
        if allow.size != plan.info["total_kraus"]:
            raise ValueError("kraus_allow needs one flag per (site, Kraus index)")
    o = L.PtsOpts(L.PTS_MODES[mode], L.ALLOCS[alloc], int(n_draws), int(k_max), int(total_shots),
                  int(nshots), int(seed), int(cfg), int(stream),
                  float(p_band[0]) if p_band else 0.0, float(p_band[1]) if p_band else 0.0,
                  C.c_void_p(allow.ctypes.data) if allow is not None else None, int(min_errors), int(max_errors),
                  L.PARITY[parity], 0)
    h = C.c_void_p()
    check(lib().ptsbe_sample_kraus(plan.handle, C.byref(o), C.byref(h)))
    return TrajSet(h, plan)


def pauli_twirl(channel):
    """Pauli-twirl probabilities of a channel dict (as in circuit["channels"]):
    4^nq values, string index digit j (0 I, 1 X, 2 Y, 3 Z) on the site's qubit j."""
    k, nq, nk = std_channel(channel)
    out = np.zeros(4 ** nq, dtype=np.float64)
    check(lib().ptsbe_pauli_twirl(nq, C.c_void_p(k.ctypes.data), nk, C.c_void_p(out.ctypes.data)))
    return out


def site_selection(plan, tags=None, qubits=None, ops=None, origins=None, kraus=None):
    """Flags for ptsbe_sample_kraus(kraus_allow=...) from ptsbe_site_selection:
    operator k >= 1 of site s is allowed when the site's op tag is in ``tags``
    (gate type), every qubit of the site is in ``qubits`` and its op index in
    ``ops`` (location), its origin in ``origins`` ("noise_op", "after_tag",
    "before_measure", "before_readout") and k in ``kraus`` (error type); None
    accepts anything."""
    keep = []

    def arr(v):
        if v is None:
            return None, 0
        a = np.ascontiguousarray(list(v), dtype=np.uint32)
        n = a.size
        if n == 0:                       # an empty list accepts nothing: non-null pointer, no entries
            a = np.zeros(1, dtype=np.uint32)
        keep.append(a)
        return C.c_void_p(a.ctypes.data), n

    f = L.SiteFilter()
    f.tags, f.n_tags = arr(None if tags is None else [tag_id(t) for t in tags])
    f.qubits, f.n_qubits = arr(qubits)
    f.ops, f.n_ops = arr(ops)
    f.origins, f.n_origins = arr(None if origins is None else [L.SITE_ORIGINS.index(x) for x in origins])
    f.kraus, f.n_kraus = arr(kraus)
    flags = np.ones(max(1, plan.info["total_kraus"]), dtype=np.uint8)
    check(lib().ptsbe_site_selection(plan.handle, C.byref(f), C.c_void_p(flags.ctypes.data)))
    return flags[:plan.info["total_kraus"]]


def ptsbe_trajset_from_records(plan, records, m, alpha0=0):
    off = np.zeros(len(records) + 1, dtype=np.uint32)
    site = []
    kr = []
    for a, rec in enumerate(records):
        for s, k in rec:
            site.append(s)
            kr.append(k)
        off[a + 1] = len(site)
    site = np.asarray(site if site else [0], dtype=np.uint32)
    kr = np.asarray(kr if kr else [0], dtype=np.uint8)
    mm = np.asarray(m, dtype=np.uint64)
    h = C.c_void_p()
    check(lib().ptsbe_trajset_from_records(plan.handle, len(records), off.ctypes.data, site.ctypes.data,
                                           kr.ctypes.data, mm.ctypes.data, int(alpha0), C.byref(h)))
    return TrajSet(h, plan)


def _run_opts(mode, seed, cfg, sort_chunk, max_batch, uniforms, params, state_out, expval, observable,
              timing=None, prefix_sharing=True, support_lists=True):
    o = L.RunOpts()
    if timing is not None:
        if timing.dtype != np.float64 or timing.size < 10:
            raise ValueError("timing must be a float64 array of at least 10 entries")
        o.timing = _dptr(timing)
    o.mode = mode
    o.flags = (0 if prefix_sharing else L.RUN_NO_PREFIX_SHARING) | (0 if support_lists else L.RUN_NO_SUPPORT_LISTS)
    o.seed = int(seed)
    o.cfg = int(cfg)
    o.sort_chunk = int(sort_chunk)
    o.max_batch = int(max_batch)
    o.d_uniforms = uniforms.data_ptr() if uniforms is not None else None
    keep = []
    if params is not None and len(params):
        pa = np.ascontiguousarray(params, dtype=np.float64)
        keep.append(pa)
        o.params = _dptr(pa)
    o.d_state_out = state_out.data_ptr() if state_out is not None else None
    o.d_expval = expval.data_ptr() if expval is not None else None
    if observable:
        coef = np.asarray([c for c, _ in observable], dtype=np.float64)
        zm = np.asarray([sum(1 << int(q) for q in qs) for _, qs in observable], dtype=np.uint64)
        keep += [coef, zm]
        o.obs_coef = _dptr(coef)
        o.obs_zmask = C.cast(zm.ctypes.data, C.POINTER(C.c_uint64))
        o.n_terms = len(observable)
    return o, keep


def ptsbe_workspace_size(plan, ts, mode="shots", sort_chunk=0, max_batch=0, params=None, prefix_sharing=True,
                         support_lists=True):
    m = {"shots": L.RUN_SHOTS, "states": L.RUN_STATES, "expectation": L.RUN_EXPECTATION,
         "adjoint": L.RUN_ADJOINT}[mode]
    pa = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
    o, keep = _run_opts(m, 0, 0, sort_chunk, max_batch, None, pa, None, None, None,
                        prefix_sharing=prefix_sharing, support_lists=support_lists)
    n = C.c_size_t()
    check(lib().ptsbe_workspace_size(plan.handle, ts.handle, C.byref(o), C.byref(n)))
    return n.value


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _outputs(plan, ts, mode, res, dev, torch):
    """Shot, tag and measure-reset record buffers of a run (the caller's, or new)."""
    n = plan.info["n_qubits"]
    if mode == "shots":
        total = ts.get()["total_shots"]
        if res.get("bits") is None:
            res["bits"] = torch.empty(max(1, total), dtype=torch.int32 if n <= 32 else torch.int64, device=dev)
        if res.get("traj") is None:
            res["traj"] = torch.empty(max(1, total), dtype=torch.int32, device=dev)
    if plan.info["n_measure"] and res.get("mr_bits") is None:
        res["mr_bits"] = torch.empty((ts.n_traj, plan.info["n_measure"]), dtype=torch.uint8, device=dev)
    return res


def ptsbe_run_batch(plan, ts, mode="shots", seed=0, cfg=0, sort_chunk=0, max_batch=0, uniforms=None,
                    params=None, observable=None, workspace=None, out=None, stream=None, timing=None,
                    prefix_sharing=True, capture=False, noalloc=False, status=None, support_lists=True):
    """Batched execution (Sec. 3).  Returns a dict of device tensors:
    shots: bits (int32 or int64 basis indices), traj (int32 trajectory ids), mr_bits;
    states: states (n_traj x 2^n complex); expectation: expval (n_traj float64) and
    E (1 float64: the ensemble value sum_a w_a expval_a, w = ts.weights()).
    ``timing``: optional float64 numpy array of 10 entries filled by the library's
    HIP-event stage timer (the call then waits for the stream).
    ``prefix_sharing``: False runs every pass for every trajectory (same results).
    ``support_lists``: False draws every chunk through the sort and the full-CDF
    search (same shots).
    ``capture``: record the run as a HIP graph on ``stream`` (a created stream)
    instead of running it; the result's "graph" replays it (``graph.launch()``).
    ``noalloc``: run through ptsbe_run_batch_noalloc (the library's fixed device
    scratch instead of a workspace; ``workspace`` and ``timing`` must be None);
    ``status`` (optional int32 device tensor of one entry) then receives the
    run's status word."""
    import torch
    dev = torch.device("cuda")
    n = plan.info["n_qubits"]
    B = ts.n_traj
    mcode = {"shots": L.RUN_SHOTS, "states": L.RUN_STATES, "expectation": L.RUN_EXPECTATION}[mode]
    res = dict(out) if out else {}
    state_out = expval = None
    if mode == "states":
        dt = torch.complex64 if plan.info["precision"] == L.C64 else torch.complex128
        state_out = res.get("states")
        if state_out is None:
            state_out = torch.empty((B, 1 << n), dtype=dt, device=dev)
        res["states"] = state_out
    ensemble = None
    if mode == "expectation":
        expval = res.get("expval")
        if expval is None:
            expval = torch.empty(max(1, B), dtype=torch.float64, device=dev)
        ensemble = res.get("E")
        if ensemble is None:
            ensemble = torch.empty(1, dtype=torch.float64, device=dev)
        res["expval"], res["E"] = expval, ensemble
    o, keep = _run_opts(mcode, seed, cfg, sort_chunk, max_batch, uniforms, params, state_out, expval,
                        observable, timing, prefix_sharing, support_lists)
    if ensemble is not None:
        o.d_ensemble = ensemble.data_ptr()
    if noalloc:
        if workspace is not None or capture:
            raise ValueError("noalloc runs take no workspace and are not captured here")
        res = _outputs(plan, ts, mode, res, dev, torch)
        bits, traj, mr = res.get("bits"), res.get("traj"), res.get("mr_bits")
        check(lib().ptsbe_run_batch_noalloc(
            plan.handle, ts.handle, C.byref(o), C.c_void_p(bits.data_ptr()) if bits is not None else None,
            C.c_void_p(traj.data_ptr()) if traj is not None else None, bits.numel() if bits is not None else 0,
            C.c_void_p(mr.data_ptr()) if mr is not None else None,
            C.c_void_p(status.data_ptr()) if status is not None else None, _stream(torch, stream)))
        res["_keep"] = keep
        return res
    need = C.c_size_t()
    check(lib().ptsbe_workspace_size(plan.handle, ts.handle, C.byref(o), C.byref(need)))
    ws = workspace
    if ws is None:
        ws = torch.empty(need.value, dtype=torch.uint8, device=dev)
    res = _outputs(plan, ts, mode, res, dev, torch)
    bits, traj, mr = res.get("bits"), res.get("traj"), res.get("mr_bits")
    cap = bits.numel() if bits is not None else 0
    args = (plan.handle, ts.handle, C.byref(o), C.c_void_p(ws.data_ptr()), ws.numel(),
            C.c_void_p(bits.data_ptr()) if bits is not None else None,
            C.c_void_p(traj.data_ptr()) if traj is not None else None, cap,
            C.c_void_p(mr.data_ptr()) if mr is not None else None, _stream(torch, stream))
    res["workspace"] = ws
    res["_keep"] = keep
    if capture:
        h = C.c_void_p()
        check(lib().ptsbe_graph_create(*args, C.byref(h)))
        res["graph"] = RunGraph(h, plan, ts, res)
        return res
    check(lib().ptsbe_run_batch(*args))
    return res


class RunGraph:
    """A captured ptsbe_run_batch (HIP graph): launch() replays the whole run on
    a stream with the same inputs and outputs."""

    def __init__(self, handle, plan, ts, buffers):
        self.handle = handle
        self._refs = (plan, ts, buffers)

    def launch(self, stream=None):
        import torch
        check(lib().ptsbe_graph_launch(self.handle, _stream(torch, stream)))

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib().ptsbe_graph_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self.handle = None


def ptsbe_run_status(plan, workspace, stream=None):
    import torch
    check(lib().ptsbe_run_status(plan.handle, C.c_void_p(workspace.data_ptr()), _stream(torch, stream)))


def ptsbe_unique_workspace_size(ts, max_batch=0):
    n = C.c_size_t()
    check(lib().ptsbe_unique_workspace_size(ts.handle, int(max_batch), C.byref(n)))
    return n.value


def ptsbe_unique_shots(ts, bits, workspace=None, max_batch=0, pairs=False, stream=None):
    """Distinct basis indices among each trajectory's shots (``bits``: the device
    shot buffer of a run of ``ts``).  Returns {"unique": int64 tensor [n_traj]}
    and with ``pairs`` also "index" (dtype of ``bits``) and "count" (int32),
    indexed like the shots: trajectory a's distinct indices in order of first
    appearance, with their counts, from its first shot position on."""
    import torch
    dev = bits.device
    B = ts.n_traj
    ws = workspace
    if ws is None:
        ws = torch.empty(max(1, ptsbe_unique_workspace_size(ts, max_batch)), dtype=torch.uint8, device=dev)
    uniq = torch.empty(max(1, B), dtype=torch.int64, device=dev)
    out = {"unique": uniq[:B]}
    pi = pc = None
    if pairs:
        pi = torch.zeros_like(bits)
        pc = torch.zeros(bits.numel(), dtype=torch.int32, device=dev)
        out["index"], out["count"] = pi, pc
    check(lib().ptsbe_unique_shots(ts.handle, C.c_void_p(bits.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                   C.c_void_p(uniq.data_ptr()), C.c_void_p(pi.data_ptr() if pi is not None else 0),
                                   C.c_void_p(pc.data_ptr() if pc is not None else 0), _stream(torch, stream)))
    return out


def ptsbe_adjoint_grad(plan, ts, params, observable, workspace=None, max_batch=0, stream=None, seed=0, cfg=0):
    """Adjoint gradient of E(theta) = sum_a w_a <psi_a|O|psi_a> over the trajectory
    set (w = ts.weights()).  ``observable``: list of (coef, qubits) Z-strings.
    State-dependent channels are decided as ptsbe_run_batch decides them with the
    same ``seed`` and ``cfg``.  Returns (E, grad) as FP64 device tensors of shapes
    (1,) and (n_params,)."""
    import torch
    dev = torch.device("cuda")
    pa = np.ascontiguousarray(params, dtype=np.float64)
    coef = np.asarray([c for c, _ in observable], dtype=np.float64)
    zm = np.asarray([sum(1 << int(q) for q in qs) for _, qs in observable], dtype=np.uint64)
    ws = workspace
    if ws is None:
        need = ptsbe_workspace_size(plan, ts, "adjoint", max_batch=max_batch, params=pa)
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    E = torch.zeros(1, dtype=torch.float64, device=dev)
    G = torch.zeros(max(1, pa.size), dtype=torch.float64, device=dev)
    check(lib().ptsbe_adjoint_grad(plan.handle, ts.handle, _dptr(pa), _dptr(coef),
                                   C.cast(zm.ctypes.data, C.POINTER(C.c_uint64)), len(observable),
                                   int(seed), int(cfg),
                                   C.c_void_p(ws.data_ptr()), ws.numel(), C.c_void_p(E.data_ptr()),
                                   C.c_void_p(G.data_ptr()), _stream(torch, stream)))
    return E, G[:pa.size]
