"""NumPy emulator of the fused device program exported by ptsbe_trajset_tables.

It executes the tile passes, slot matrices, per-trajectory overrides and
measure-reset steps exactly as the tables describe them (complex128), so the
planner's fusion can be checked against the oracle on the CPU.  Test helper
only: it re-implements the device program's semantics, not the method.
"""

import numpy as np

from paper_2504_16297_amd.tables import (  # noqa: F401
    D1, D2, DOT, DSIGN, M1, M1G, M2, MR, PHASE, SFLIP, export_adjoint_tables, export_tables)


def _apply_1q(T, a, m):
    nt = T.shape[1]
    v = T.reshape(T.shape[0], nt >> (a + 1), 2, 1 << a)
    x0 = v[:, :, 0, :].copy()
    x1 = v[:, :, 1, :].copy()
    v[:, :, 0, :] = m[0, 0] * x0 + m[0, 1] * x1
    v[:, :, 1, :] = m[1, 0] * x0 + m[1, 1] * x1


def _geometry(tables, p, t, n):
    """Tile indices [tiles, 2^k] of pass p and trajectory t's slot offsets."""
    passes = tables["passes"]
    NP = len(passes)
    ps = passes[p]
    k = int(ps["k"])
    tq = [int(q) for q in ps["tq"][:k]]
    oq = [int(q) for q in ps["oq"][:n - k]]
    Lidx = np.arange(1 << k)
    off = np.zeros(1 << k, dtype=np.int64)
    for j, q in enumerate(tq):
        off |= ((Lidx >> j) & 1) << q
    tiles = np.arange(1 << (n - k))
    base = np.zeros(tiles.size, dtype=np.int64)
    for i, q in enumerate(oq):
        base |= ((tiles >> i) & 1) << q
    idx = base[:, None] + off[None, :]
    slot = [int(s) for s in tables["slot_default"][ps["slot_begin"]:ps["slot_begin"] + ps["n_slots"]]]
    ob, oe = tables["ov_off"][t * NP + p], tables["ov_off"][t * NP + p + 1]
    for e in tables["ov"][ob:oe]:
        slot[int(e["slot"])] = int(e["off"])
    return ps, k, idx, slot


def _apply_op(T, op, slot, pool, idx, k, reg, bits, norms):
    """Apply one table op to tiles T [tiles, 2^k]; returns the register-bit set."""
    nt = 1 << k
    Lidx = np.arange(nt)
    ty = int(op["type"])
    if reg is not None and ty in (M1, MR):
        assert int(op["a"]) in reg, "operation outside the register bits"
    if ty == PHASE:
        reg = {int(op["a"]), int(op["b"]), int(op["ga"]), int(op["gb"])}
        assert len(reg) == 4 and max(reg) < k
    elif ty == M1G:
        assert reg is not None, "grouped 2x2 op outside the register kernel"
        pos = sorted(reg)
        for j in range(4):            # idle positions carry the identity slot
            sj = slot[int(op["slots"][j])]
            m = pool[sj:sj + 4].reshape(2, 2)
            if not (int(op["mask"]) >> j) & 1:
                assert np.array_equal(m, np.eye(2)), "idle position without identity"
            _apply_1q(T, pos[j], m)
    elif ty == SFLIP:
        pass
    elif ty == M1:
        m = pool[slot[op["slots"][0]]:slot[op["slots"][0]] + 4].reshape(2, 2)
        _apply_1q(T, int(op["a"]), m)
    elif ty == M2:
        m = pool[slot[op["slots"][0]]:slot[op["slots"][0]] + 16].reshape(4, 4)
        a, b = int(op["a"]), int(op["b"])
        ba = (Lidx >> a) & 1
        bb = (Lidx >> b) & 1
        i00 = Lidx[(ba == 0) & (bb == 0)]
        grp = [i00, i00 | (1 << a), i00 | (1 << b), i00 | (1 << a) | (1 << b)]
        X = np.stack([T[:, g] for g in grp], axis=-1)
        Y = X @ m.T
        for j, g in enumerate(grp):
            T[:, g] = Y[..., j]
    elif ty in (D1, D2):
        dd = 3 if ty == D1 else 5
        m = pool[slot[op["slots"][0]]:slot[op["slots"][0]] + (4 if ty == D1 else 16)]
        ga = ((idx >> int(op["ga"])) & 1)
        gb = ((idx >> int(op["gb"])) & 1) if ty == D2 else 0
        T *= m[(ga + 2 * gb) * dd]
    elif ty == DSIGN:
        ga = ((idx >> int(op["ga"])) & 1)
        gb = 0 if int(op["b"]) == 254 else ((idx >> int(op["gb"])) & 1)
        neg = (int(op["slots"][0]) >> (ga + 2 * gb)) & 1
        T *= np.where(neg == 1, -1.0, 1.0)
    elif ty == MR:
        r = int(op["slots"][0])
        b = bits[r]
        a = int(op["a"])
        v = T.reshape(T.shape[0], nt >> (a + 1), 2, 1 << a)
        keep = v[:, :, b, :].copy() * norms[r]
        v[:, :, 0, :] = keep
        v[:, :, 1, :] = 0
    else:
        raise ValueError(ty)
    return reg


def run_program(tables, n, B, mr_tol=1e-6, normalise=True):
    """Return (states [B, 2^n], mr bits [B, n_measure] as lists)."""
    N = 1 << n
    ops = tables["ops"]
    states = []
    allbits = []
    x = np.arange(N, dtype=np.int64)
    for t in range(B):
        psi = np.zeros(N, dtype=np.complex128)
        bits = {}
        norms = {}
        for ex in tables["exec"]:
            if ex["pass"] != 0xFFFFFFFF:
                p = int(ex["pass"])
                ps, k, idx, slot = _geometry(tables, p, t, n)
                if ps["flags"] & 1:
                    T = np.zeros(idx.shape, dtype=np.complex128)
                    T[0, 0] = 1.0
                else:
                    T = psi[idx].copy()
                reg = set(range(k - 4, k)) if k >= 6 else None   # register bits of the register kernel
                for op in ops[ps["op_begin"]:ps["op_begin"] + ps["n_ops"]]:
                    reg = _apply_op(T, op, slot, tables["pool"], idx, k, reg, bits, norms)
                if reg is not None:
                    assert reg == set(range(k - 4, k)), "pass must end in the load/store register layout"
                psi = np.zeros(N, dtype=np.complex128) if ps["flags"] & 1 else psi
                psi[idx] = T
            else:
                w = np.abs(psi) ** 2
                tot = w.sum()
                for j in range(int(ex["nq"])):
                    q = int(ex["q"][j])
                    p1 = w[((x >> q) & 1) == 1].sum() / tot
                    if min(p1, 1 - p1) > mr_tol:
                        raise RuntimeError(f"non-deterministic measure-reset on qubit {q}")
                    b = 1 if p1 > 0.5 else 0
                    r = int(ex["idx"][j])
                    bits[r] = b
                    pb = p1 if b else 1 - p1
                    norms[r] = 1.0 / np.sqrt(pb * tot) if j == 0 else 1.0 / np.sqrt(pb)
        states.append(psi / np.linalg.norm(psi) if normalise else psi)
        allbits.append([bits[r] for r in sorted(bits)])
    return states, allbits


def run_adjoint(fwd, adj, dot_param, n, B, n_params, odiag, weights, back_tol=1e-9):
    """E and gradient from the forward tables and the reverse-sweep tables: every
    non-DOT op is applied to both psi and lambda tiles; a DOT op adds
    Im<lambda|P|psi> over the pass's tiles to its gradient term."""
    states, _ = run_program(fwd, n, B, normalise=False)
    E = 0.0
    grad = np.zeros(n_params)
    for t in range(B):
        psi = states[t].copy()
        E += weights[t] * float(np.sum(np.abs(psi) ** 2 * odiag))
        lam = odiag * psi
        for ex in adj["exec"]:
            p = int(ex["pass"])
            ps, k, idx, slot = _geometry(adj, p, t, n)
            assert not ps["flags"] & 1
            Tp, Tl = psi[idx].copy(), lam[idx].copy()
            reg = set(range(k - 4, k)) if k >= 6 else None
            for op in adj["ops"][ps["op_begin"]:ps["op_begin"] + ps["n_ops"]]:
                if int(op["type"]) == DOT:
                    if reg is not None:
                        assert int(op["a"]) in reg, "gradient term outside the register bits"
                    a, gen = int(op["a"]), int(op["b"])
                    d = int(op["slots"][0]) | (int(op["slots"][1]) << 16)
                    vp = Tp.reshape(Tp.shape[0], -1, 2, 1 << a)
                    vl = Tl.reshape(Tl.shape[0], -1, 2, 1 << a)
                    p0, p1, l0, l1 = vp[:, :, 0], vp[:, :, 1], vl[:, :, 0], vl[:, :, 1]
                    if gen == 3:
                        z = np.vdot(l0, p0) - np.vdot(l1, p1)
                    elif gen == 1:
                        z = np.vdot(l0, p1) + np.vdot(l1, p0)
                    else:
                        z = -1j * np.vdot(l0, p1) + 1j * np.vdot(l1, p0)
                    grad[int(dot_param[d])] += weights[t] * z.imag
                else:
                    r0 = reg
                    reg = _apply_op(Tp, op, slot, adj["pool"], idx, k, r0, {}, {})
                    _apply_op(Tl, op, slot, adj["pool"], idx, k, r0, {}, {})
            psi[idx] = Tp
            lam[idx] = Tl
        # the sweep un-applies the whole circuit: psi is back at |0>
        assert abs(psi[0]) > 1 - back_tol and float(np.sum(np.abs(psi[1:]) ** 2)) < back_tol
    return E, grad
