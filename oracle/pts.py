"""Pre-trajectory sampling (Sec. 3.1): choosing Kraus-operator sets and shot counts.

A *record* is the tuple of (site, k) pairs with k != 0 (index 0 is each
channel's no-error operator), sorted by site.  Equal records are one
trajectory (``uniqueKraus`` of Algorithm 2).  Trajectories are ordered by first
occurrence, except in most-likely-first mode where they are ordered by score.

Samplers:
* ``proportional``   -- one exact categorical draw per site per sample, so a
  record appears with its joint probability p_alpha (the proportional variant of
  Sec. 3.1).  index(r, {p}) of Algorithm 1 is read as the smallest k with
  r < p_0 + ... + p_k.
* ``alg2_literal``   -- Algorithm 2 as printed: for each (K, p) of the noisy
  circuit draw r and keep K if r <= p and it is compatible (no other
  non-identity operator chosen at the same site yet).
* ``most_likely``    -- the records of highest joint probability ("error
  combinations whose joint probability falls above a given cutoff").

Selection criteria (the checks Sec. 3.1 suggests adding where Algorithm 2
chooses each operator: gate type, parity, location): ``allow`` is a set of
(site, k) pairs; an operator outside it is never chosen (its site keeps
operator 0).  ``keep_record`` drops records by their number of errors (a
window and a parity); dropped draws do not count towards n_draws.

Allocations:
* ``multiplicity``   -- m_alpha = count_alpha * S / T, largest remainder.
* ``reweight``       -- m_alpha proportional to p'_alpha = p_alpha / sum over the
  selected set of p_beta (Sec. 3.1), largest remainder.
* ``uniform``        -- every kept record gets ``nshots`` (Algorithm 2).

Ensemble weights: the trajectories stand for the noisy channel in the
proportions their shots are allocated by, so an expectation over the set is
E = sum_alpha w_alpha <O>_alpha with w_alpha proportional to count_alpha
(multiplicity: the draw frequencies, an unbiased estimate of the channel),
p_alpha (reweight: the probability-weighted expectation over the selected
records, Sec. 3.1) or 1 (uniform), normalised over the set.

Probability band (Sec. 3.1: a Kraus operator set is only chosen if its joint
probability lies in [p_min, p_max]): applied to the records a sampler returns,
after the record-level criteria and before the allocation, which then runs
over the kept records and their kept draws.
"""

import itertools
import math

import numpy as np

from .rng import key1, uniforms

STREAM_PTS = 1


def _categorical(u, probs):
    """Smallest k with u < p_0 + ... + p_k (prefix sums in order), clamped to the last index."""
    c = np.cumsum(np.asarray(probs, dtype=np.float64))
    k = int(np.searchsorted(c, u, side="right"))
    return min(k, len(probs) - 1)


def proportional(site_probs, seed, cfg, n_draws, stream=STREAM_PTS, merge=True, allow=None):
    """Return (records, counts) for ``n_draws`` proportional draws.

    Draw t uses the stream [seed, key1(stream, cfg, t)]; word s is site s.  A
    drawn operator outside ``allow`` leaves its site at operator 0."""
    S = len(site_probs)
    index = {}
    records = []
    counts = []
    for t in range(n_draws):
        u = uniforms(seed, key1(stream, cfg, t), S) if S else np.zeros(0)
        rec = []
        for s in range(S):
            k = _categorical(u[s], site_probs[s])
            if k != 0 and (allow is None or (s, k) in allow):
                rec.append((s, k))
        rec = tuple(rec)
        if merge and rec in index:
            counts[index[rec]] += 1
        else:
            index[rec] = len(records)
            records.append(rec)
            counts.append(1)
    return records, counts


def alg2_draw(site_probs, seed, cfg, t, stream=STREAM_PTS, allow=None):
    """One sample of Algorithm 2 as printed.  Words of stream t are consumed one
    per (s, k >= 1) pair in circuit order; r <= p_{s,k} keeps K_{s,k} if it is
    compatible, i.e. site s has no operator yet (the first one kept wins), and
    it passes the selection (in ``allow``)."""
    n_pairs = sum(len(p) - 1 for p in site_probs)
    u = uniforms(seed, key1(stream, cfg, t), n_pairs) if n_pairs else np.zeros(0)
    j = 0
    rec = []
    for s, probs in enumerate(site_probs):
        chosen = False
        for k in range(1, len(probs)):
            r = u[j]
            j += 1
            if r <= probs[k] and not chosen and (allow is None or (s, k) in allow):
                rec.append((s, k))
                chosen = True
    return tuple(rec)


def alg2_literal(site_probs, seed, cfg, n_draws, nshots, stream=STREAM_PTS, allow=None):
    """Algorithm 2: ``n_draws`` samples, duplicates dropped (uniqueKraus), each kept
    record given ``nshots`` shots."""
    index = {}
    records = []
    for t in range(n_draws):
        rec = alg2_draw(site_probs, seed, cfg, t, stream, allow)
        if rec not in index:
            index[rec] = len(records)
            records.append(rec)
    return records, [int(nshots)] * len(records)


def joint_prob(record, site_probs):
    """p_alpha = product over all sites, in site order, of p_{s,k_s} (k_s = 0 off the record)."""
    ks = dict(record)
    p = 1.0
    for s, probs in enumerate(site_probs):
        p *= probs[ks.get(s, 0)]
    return p


def costs(site_probs):
    """c_{s,k} = -ln(p_{s,k} / p_{s,0}) for k >= 1 (math.log: the C library's log)."""
    out = {}
    for s, probs in enumerate(site_probs):
        for k in range(1, len(probs)):
            if probs[k] > 0:
                out[(s, k)] = -math.log(probs[k] / probs[0])
    return out


def score(record, cost):
    """Sum of the record's costs taken in ascending (c, s, k) order."""
    terms = sorted((cost[sk], sk[0], sk[1]) for sk in record)
    total = 0.0
    for c, _, _ in terms:
        total += c
    return total


def _records_dfs(e, items, bound):
    """All records of exactly ``e`` errors on distinct sites with score <= bound.

    ``items`` are (c, s, k) sorted ascending, so a record's score is the running
    sum in item order and the walk can stop as soon as the next item overshoots."""
    out = []

    def walk(start, chosen, used, partial):
        if len(chosen) == e:
            rec = tuple(sorted((s, k) for _, s, k in chosen))
            out.append((rec, partial))
            return
        for j in range(start, len(items)):
            c, s, k = items[j]
            if partial + c > bound:
                break
            if s in used:
                continue
            used.add(s)
            chosen.append(items[j])
            walk(j + 1, chosen, used, partial + c)
            chosen.pop()
            used.discard(s)

    walk(0, [], set(), 0.0)
    return out


def _pairs_numpy(items, bound, keep):
    """Two-error records with score <= bound, the ``keep`` best by (score, record)."""
    c = np.array([it[0] for it in items])
    s = np.array([it[1] for it in items], dtype=np.int64)
    k = np.array([it[2] for it in items], dtype=np.int64)
    i, j = np.triu_indices(len(items), 1)
    tot = c[i] + c[j]
    ok = (s[i] != s[j]) & (tot <= bound)
    i, j, tot = i[ok], j[ok], tot[ok]
    first = s[i] < s[j]
    sa = np.where(first, s[i], s[j]); ka = np.where(first, k[i], k[j])
    sb = np.where(first, s[j], s[i]); kb = np.where(first, k[j], k[i])
    order = np.lexsort((kb, sb, ka, sa, tot))[:keep]
    return [(((int(sa[o]), int(ka[o])), (int(sb[o]), int(kb[o]))), float(tot[o])) for o in order]


def keep_record(n_errors, min_errors=0, max_errors=0, parity=None):
    """Record-level selection: at least min_errors and (max_errors > 0) at most
    max_errors operators k >= 1, and their number even / odd if asked."""
    if n_errors < min_errors or (max_errors and n_errors > max_errors):
        return False
    if parity == "even" and n_errors % 2:
        return False
    if parity == "odd" and n_errors % 2 == 0:
        return False
    return True


def select_records(records, counts, **crit):
    """Drop the records (with their counts) that keep_record rejects."""
    kept = [(r, c) for r, c in zip(records, counts) if keep_record(len(r), **crit)]
    return [r for r, _ in kept], [c for _, c in kept]


def most_likely(site_probs, k_max, allow=None, **crit):
    """The ``k_max`` records of highest joint probability.

    Ranking: ascending score (= descending p_alpha / p_none), ties broken by the
    record's (s, k) list in lexicographic order.  Enumeration by number of
    errors e = 0, 1, 2, ...: each round adds every e-error record whose score
    does not exceed the current k_max-th score, and the search stops once the
    cheapest possible record with e errors scores above it.  With selection
    criteria only operators in ``allow`` are enumerated and only records that
    keep_record(**crit) accepts are ranked.  Returns (records, scores)."""
    cost = costs(site_probs)
    if allow is not None:
        cost = {sk: c for sk, c in cost.items() if sk in allow}
    max_e = crit.get("max_errors", 0)
    items = sorted((c, s, k) for (s, k), c in cost.items())
    per_site = {}
    for c, s, _ in items:
        per_site.setdefault(s, c)              # items ascending: first is the site's minimum
    site_min = sorted(per_site.values())
    cands = [((), 0.0)] if keep_record(0, **crit) else []
    e = 0
    while True:
        e += 1
        cands.sort(key=lambda rc: (rc[1], rc[0]))
        cands = cands[:k_max]
        bound = cands[-1][1] if len(cands) >= k_max else math.inf
        if e > len(site_min) or (max_e and e > max_e):
            break
        cheapest = 0.0
        for v in site_min[:e]:
            cheapest += v
        if cheapest > bound:
            break
        if not keep_record(e, **crit):
            continue
        if e == 2:
            cands.extend(_pairs_numpy(items, bound, k_max))
        else:
            cands.extend(_records_dfs(e, items, bound))
    cands.sort(key=lambda rc: (rc[1], rc[0]))
    top = cands[:k_max]
    return [r for r, _ in top], [sc for _, sc in top]


def most_likely_bruteforce(site_probs, k_max, allow=None, **crit):
    """Every record of the full product space, sorted by (score, record); tiny cases only."""
    cost = costs(site_probs)
    choices = [range(len(p)) for p in site_probs]
    allrec = []
    for ks in itertools.product(*choices):
        rec = tuple((s, k) for s, k in enumerate(ks) if k != 0)
        if (all(sk in cost for sk in rec) and (allow is None or all(sk in allow for sk in rec))
                and keep_record(len(rec), **crit)):
            allrec.append((rec, score(rec, cost)))
    allrec.sort(key=lambda rc: (rc[1], rc[0]))
    top = allrec[:k_max]
    return [r for r, _ in top], [sc for _, sc in top]


def probability_band(records, counts, site_probs, p_min, p_max):
    """Keep the records whose joint probability p_alpha lies in [p_min, p_max]
    (both ends included), with their draw counts, in their order.  Returns
    (records, counts, T) with T the number of kept draws."""
    kept_r, kept_c = [], []
    for rec, c in zip(records, counts):
        pa = joint_prob(rec, site_probs)
        if p_min <= pa <= p_max:
            kept_r.append(rec)
            kept_c.append(c)
    return kept_r, kept_c, sum(kept_c)


def allocate_multiplicity(counts, n_draws, total_shots):
    """m_alpha = floor(count_alpha * S / T) plus one for the largest remainders
    (ties to the lower alpha), so that sum m_alpha = S exactly."""
    base = [(c * total_shots) // n_draws for c in counts]
    rem = [(c * total_shots) % n_draws for c in counts]
    left = total_shots - sum(base)
    order = sorted(range(len(counts)), key=lambda a: (-rem[a], a))
    for a in order[:left]:
        base[a] += 1
    return base


def allocate_reweight(probs, total_shots):
    """m_alpha from p'_alpha = p_alpha / sum_beta p_beta (Sec. 3.1), largest remainder."""
    P = 0.0
    for p in probs:
        P += p
    x = [(p / P) * float(total_shots) for p in probs]
    base = [int(math.floor(v)) for v in x]
    frac = [v - b for v, b in zip(x, base)]
    left = total_shots - sum(base)
    order = sorted(range(len(probs)), key=lambda a: (-frac[a], a))
    for a in order[:left]:
        base[a] += 1
    return base


def _alg2_counts(site_probs, seed, cfg, n_draws, records):
    """How many of Algorithm 2's ``n_draws`` samples produced each unique record."""
    index = {r: a for a, r in enumerate(records)}
    counts = [0] * len(records)
    for t in range(n_draws):
        counts[index[alg2_draw(site_probs, seed, cfg, t)]] += 1
    return counts


def ensemble_weights(counts, probs, alloc):
    """w_alpha = b_alpha / sum_beta b_beta with b = counts (multiplicity),
    probs (reweight) or 1 (uniform), summed in trajectory order."""
    if alloc == "multiplicity":
        b = [float(c) for c in counts]
    elif alloc == "reweight":
        b = [float(p) for p in probs]
    elif alloc == "uniform":
        b = [1.0] * len(counts)
    else:
        raise ValueError(alloc)
    tot = 0.0
    for v in b:
        tot += v
    return [v / tot for v in b]


def sample_kraus(circuit_probs, pts, seed, cfg):
    """Run the PTS step described by a workload's ``pts`` options.

    ``pts["p_band"] = (p_min, p_max)`` keeps only the records in that band; the
    allocation then runs over the kept records (multiplicity: over their draws).
    Returns dict(records, m, p, counts, weights)."""
    mode = pts["mode"]
    if mode == "proportional":
        recs, counts = proportional(circuit_probs, seed, cfg, pts["n_draws"])
        T = pts["n_draws"]
    elif mode == "alg2_literal":
        recs, _ = alg2_literal(circuit_probs, seed, cfg, pts["n_draws"], pts.get("nshots", 1))
        counts = _alg2_counts(circuit_probs, seed, cfg, pts["n_draws"], recs)
        T = pts["n_draws"]
    elif mode == "most_likely":
        recs, _ = most_likely(circuit_probs, pts["k_max"])
        counts = [1] * len(recs)
        T = len(recs)
    else:
        raise ValueError(mode)
    if pts.get("p_band") is not None:
        recs, counts, T = probability_band(recs, counts, circuit_probs, *pts["p_band"])
        if not recs:
            raise ValueError("no record falls in the probability band")
    p = [joint_prob(r, circuit_probs) for r in recs]
    alloc = pts.get("alloc", "multiplicity")
    if alloc == "multiplicity":
        m = allocate_multiplicity(counts, T, pts["total_shots"])
    elif alloc == "reweight":
        m = allocate_reweight(p, pts["total_shots"])
    elif alloc == "uniform":
        m = [int(pts.get("nshots", 1))] * len(recs)
    else:
        raise ValueError(alloc)
    return {"records": recs, "m": m, "p": p, "counts": counts,
            "weights": ensemble_weights(counts, p, alloc)}
