"""Expansion of a circuit and its noise model into an ordered step list.

Algorithm 1 of Sec. 2.2 walks the operator sequence and looks up the noise
channel attached to each operator; Algorithm 2 (Sec. 3.1) iterates over the
flattened list of (Kraus set, probabilities) of the noisy circuit.  This module
produces that flattened order ("noise sites"), which every sampler and every
simulator below shares.

Site order (the paper leaves it open; reading used): walk the ops in order.
Before a measure-reset op, one site per ``before_measure`` rule (rule order).
An explicit ``noise`` op is a site at its own position.  After a gate or
parametrised gate, one site per ``after_tag`` rule whose tag matches.  At the
end, for each ``before_readout`` rule, one site per listed qubit, ascending.

A channel on one or two qubits that is not a unitary mixture (amplitude
damping, any CPTP channel whose K^dagger K are not multiples of the identity)
is not pre-sampled: at each of its positions
the step list holds a ("gch", qubits, record index, channel, gch index) step,
decided when the state reaches it; its record index shares the counter of the
measure-resets.
"""

from .channels import kraus_ops, cptp_error, state_dependent, unitary_mixture


class NotCPTP(ValueError):
    pass


class Unsupported(ValueError):
    pass


def expand(circuit):
    """Return (steps, sites).

    steps: list of tuples
      ("gate", name, qubits, params) | ("param", gen, qubits, index) |
      ("site", site_id, qubits) | ("mr", qubits, mr_index) | ("p0", qubits)
    sites: list of dicts {"channel": c, "qubits": qs}
    """
    rules = circuit.get("rules", [])
    steps = []
    sites = []
    n_mr = 0
    n_g = 0
    general = [state_dependent(kraus_ops(ch)) for ch in circuit.get("channels", [])]

    def add_site(ch, qubits):
        nonlocal n_mr, n_g
        if circuit["channels"][ch]["nq"] != len(qubits):
            raise ValueError("channel arity does not match the site's qubits")
        if general[ch]:
            steps.append(("gch", tuple(qubits), n_mr, ch, n_g))
            n_mr += 1
            n_g += 1
            return
        sites.append({"channel": ch, "qubits": tuple(qubits)})
        steps.append(("site", len(sites) - 1, tuple(qubits)))

    for op in circuit["ops"]:
        kind = op["kind"]
        if kind == "measure_reset":
            for r in rules:
                if r["when"] == "before_measure":
                    add_site(r["channel"], op["qubits"])
            steps.append(("mr", tuple(op["qubits"]), n_mr))
            n_mr += 1
        elif kind == "project0":
            steps.append(("p0", tuple(op["qubits"])))
        elif kind == "noise":
            add_site(op["channel"], op["qubits"])
        elif kind in ("gate", "param"):
            if kind == "gate":
                steps.append(("gate", op["name"], tuple(op["qubits"]), tuple(op["params"])))
            else:
                steps.append(("param", op["gen"], tuple(op["qubits"]), op["index"]))
            for r in rules:
                if r["when"] == "after_tag" and r["tag"] == op["tag"]:
                    add_site(r["channel"], op["qubits"])
        else:
            raise ValueError(f"unknown op kind {kind}")
    for r in rules:
        if r["when"] == "before_readout":
            for q in sorted(r["qubits"]):
                add_site(r["channel"], (q,))
    return steps, sites


def site_channels(circuit):
    """Per channel: (probs, unitaries) after checking CPTP and the unitary-mixture form."""
    out = []
    for ch in circuit["channels"]:
        K = kraus_ops(ch)
        if cptp_error(K) > 1e-12:
            raise NotCPTP(ch.get("name", "kraus"))
        um = unitary_mixture(K)
        if um is None:
            if not state_dependent(K):
                raise Unsupported(f"{ch.get('name', 'kraus')} is not a unitary mixture")
            out.append(None)        # state-dependent: no pre-sampled probabilities
            continue
        out.append(um)
    return out


def site_probs(circuit):
    """List over sites of the probability vector p_{s,k}."""
    _, sites = expand(circuit)
    chans = site_channels(circuit)
    return [chans[s["channel"]][0] for s in sites]
