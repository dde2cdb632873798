"""Brute-force k-medoids checks for tiny inputs (pure Python over a matrix).

Independent of the oracle: everything here recomputes the total deviation
TD(M) = sum_o min_{m in M} d(o, m) (Eq. td) from scratch for every medoid set
it considers, instead of using cached nearest/second distances or the change
formula.
"""
from itertools import combinations


def td_of(D, med):
    n = len(D)
    return sum(min(D[o][m] for m in med) for o in range(n))


def build_greedy(D, k, exclude_self=False):
    """Greedy BUILD by full TD recomputation.  Step 0: smallest distance sum.
    Later steps: the candidate whose addition lowers TD most (first on ties);
    with exclude_self the candidate's own drop to zero is not counted."""
    n = len(D)
    sums = [sum(D[o][c] for o in range(n) if o != c) for c in range(n)]
    best, m1 = None, None
    for c in range(n):
        if best is None or sums[c] < best:
            best, m1 = sums[c], c
    med = [m1]
    for _ in range(1, k):
        base = td_of(D, med)
        dn = [min(D[o][m] for m in med) for o in range(n)]
        best, bc = None, None
        for c in range(n):
            if c in med:
                continue
            ch = td_of(D, med + [c]) - base
            if exclude_self:
                ch += dn[c]
            if best is None or ch < best:
                best, bc = ch, c
        med.append(bc)
    return med


def all_swaps(D, med):
    """{(slot, cand): TD change} for every swap of a medoid slot with a non-medoid."""
    n = len(D)
    base = td_of(D, med)
    out = {}
    for i in range(len(med)):
        for c in range(n):
            if c in med:
                continue
            m2 = list(med)
            m2[i] = c
            out[(i, c)] = td_of(D, m2) - base
    return out


def best_swap(D, med):
    """Lexicographic minimum over (delta, slot, cand) among negative deltas, or None."""
    sw = all_swaps(D, med)
    best = None
    for (i, c), v in sw.items():
        if v < 0 and (best is None or (v, i, c) < best):
            best = (v, i, c)
    return best


def pam_swap(D, med, max_iter=1000):
    med = list(med)
    trace = []
    for _ in range(max_iter):
        b = best_swap(D, med)
        if b is None:
            break
        v, i, c = b
        med[i] = c
        trace.append((i, c, v))
    return med, trace


def fastpam2_swap(D, med, max_iter=1000):
    """Best swap per medoid, visited by (delta, slot), each re-checked by a
    full TD recomputation against the current medoids before it is applied."""
    n = len(D)
    med = list(med)
    trace = []
    for _ in range(max_iter):
        sw = all_swaps(D, med)
        per = []
        for i in range(len(med)):
            bv, bc = None, None
            for c in range(n):
                if (i, c) in sw and (bv is None or sw[(i, c)] < bv):
                    bv, bc = sw[(i, c)], c
            if bc is not None and bv < 0:
                per.append((bv, i, bc))
        if not per:
            break
        per.sort()
        for _, i, c in per:
            if c in med:
                continue
            m2 = list(med)
            m2[i] = c
            ch = td_of(D, m2) - td_of(D, med)
            if ch < 0:
                med = m2
                trace.append((i, c, ch))
    return med, trace


def global_optimum(D, k):
    n = len(D)
    return min(td_of(D, list(s)) for s in combinations(range(n), k))


def is_local_optimum(D, med):
    return all(v >= 0 for v in all_swaps(D, med).values())


def fasterpam_swap(D, med, max_passes=1000):
    """Alg. 4's scan with every change taken as a full TD recomputation.

    Positions 0, 1, ..., n-1, 0, ... are visited in turn; at a non-medoid c
    the TD change of putting c into each slot is computed and the smallest
    slot with the smallest change is swapped in at once if that change is
    negative.  The scan ends once n consecutive positions passed without a
    swap.  Returns (medoids, trace [(slot, cand, change)], passes begun)."""
    n = len(D)
    med = list(med)
    trace = []
    pos = visited = quiet = 0
    while quiet < n and visited < max_passes * n:
        c = pos
        pos = (pos + 1) % n
        visited += 1
        quiet += 1
        if c in med:
            continue
        base = td_of(D, med)
        ch = []
        for i in range(len(med)):
            m2 = list(med)
            m2[i] = c
            ch.append(td_of(D, m2) - base)
        i = min(range(len(med)), key=lambda j: (ch[j], j))
        if ch[i] < 0:
            med[i] = c
            trace.append((i, c, ch[i]))
            quiet = 0
    return med, trace, (visited + n - 1) // n


def lab_greedy(D, k, samples, exclude_self=False):
    """LAB by full recomputation: at step t the candidate of samples[t] (in
    listed order, medoids skipped, first strict minimum) that minimises the
    TD of the subsample, TD_S(M + [c]); step 0 uses TD_S([c]) (the first BUILD
    step on the subsample).  With exclude_self the candidate's own drop to
    distance zero is not counted."""
    n = len(D)
    med = []
    for t in range(k):
        S = list(samples[t])
        best, bc = None, None
        for c in S:
            if c in med:
                continue
            if t == 0:
                ch = sum(D[o][c] for o in S if o != c)
            else:
                dn = {o: min(D[o][m] for m in med) for o in S}
                ch = sum(min(dn[o], D[o][c]) for o in S) - sum(dn[o] for o in S)
                if exclude_self and c in dn:
                    ch += dn[c]
            if best is None or ch < best:
                best, bc = ch, c
        if bc is None:
            bc = min(o for o in range(n) if o not in med)
        med.append(bc)
    return med


def clarans_search(D, med, draws, maxneighbor):
    """One FastCLARANS local search by full TD recomputation: draws that are
    medoids are skipped; a drawn non-medoid takes its best slot (smallest on
    ties) and is swapped in when TD drops; maxneighbor consecutive failures
    end the search.  Returns (medoids, trace, evaluations, list exhausted)."""
    med = list(med)
    trace = []
    fails = evals = 0
    for c in draws:
        if fails >= maxneighbor:
            return med, trace, evals, False
        if c in med:
            continue
        evals += 1
        base = td_of(D, med)
        ch = []
        for i in range(len(med)):
            m2 = list(med)
            m2[i] = c
            ch.append(td_of(D, m2) - base)
        i = min(range(len(med)), key=lambda j: (ch[j], j))
        if ch[i] < 0:
            med[i] = c
            trace.append((i, c, ch[i]))
            fails = 0
        else:
            fails += 1
    return med, trace, evals, fails < maxneighbor


# ---- bichromatic medoids: D[consumer][location], medoids are locations
def rect_td_of(D, med):
    return sum(min(row[m] for m in med) for row in D)


def rect_build_greedy(D, k):
    """Location with the smallest distance sum to all consumers, then the
    location lowering TD most (first on ties), by full recomputation."""
    nl = len(D[0])
    med = []
    for _ in range(k):
        best, bc = None, None
        for c in range(nl):
            if c in med:
                continue
            v = rect_td_of(D, med + [c])
            if best is None or v < best:
                best, bc = v, c
        med.append(bc)
    return med


def rect_pam_swap(D, med, max_iter=1000):
    """Best-swap steepest descent over (change, slot, location) by full TD
    recomputation."""
    nl = len(D[0])
    med = list(med)
    trace = []
    for _ in range(max_iter):
        base = rect_td_of(D, med)
        best = None
        for i in range(len(med)):
            for c in range(nl):
                if c in med:
                    continue
                m2 = list(med)
                m2[i] = c
                v = rect_td_of(D, m2) - base
                if v < 0 and (best is None or (v, i, c) < best):
                    best = (v, i, c)
        if best is None:
            break
        v, i, c = best
        med[i] = c
        trace.append((i, c, v))
    return med, trace
