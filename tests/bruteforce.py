"""Brute-force checkers written from definitions, independent of oracle/.

* Distance-2 independence and maximality by breadth-first search (the
  problem statement, Section I).
* Luby's algorithm on G^2 (Section IV, Lemmas 1-2): each round every
  undecided vertex v draws a tuple; v leaves as OUT if an IN vertex chosen in
  an earlier round lies within distance 2, otherwise v joins as IN if its
  tuple is below that of every other undecided vertex within distance 2.
  Removal lags one round behind the IN decision, exactly as in Algorithm 1,
  where a neighbourhood sees an IN only in the next round's Refresh Column.
  Distances are computed on the explicit squared graph, not by two sweeps.
* Aggregation invariants of Algorithm 3 (Section III-B), Algorithm 2's
  aggregates from its statement, and the quotient graph by explicit pair
  sets.

Pure Python on small graphs only.
"""
MASK64 = (1 << 64) - 1


def xs64star(x):
    """xorshift64* from its published definition (Vigna, ACM TOMS 2016)."""
    x &= MASK64
    x ^= x >> 12
    x ^= (x << 25) & MASK64
    x ^= x >> 27
    return (x * 0x2545F4914F6CDD1D) & MASK64


def xs64(x):
    """xorshift64 as xorshift*'s first stage (shifts 12, 25, 27, no
    multiplication): the "Xor Hash" of Table I."""
    x &= MASK64
    x ^= x >> 12
    x ^= (x << 25) & MASK64
    x ^= x >> 27
    return x


def prio_hash(seed, it, v):
    """h(iter, v) = f(f(iter) xor f(v)) (Section V-A), iter offset by seed << 32."""
    return xs64star(xs64star(((seed << 32) ^ it) & MASK64) ^ xs64star(v))


def nbits(n):
    b = 0
    while 2 ** b < n + 2:
        b += 1
    return b


def tuple_of(prio, v, n):
    """The (priority, id) tuple as a pair compared lexicographically; the
    priority keeps the low 32 - b bits (Section V-C)."""
    b = nbits(n)
    pb = 32 - b
    return (prio & ((1 << pb) - 1) if pb > 0 else 0, v)


def adjacency(row_ptr, col):
    n = len(row_ptr) - 1
    return [set(int(c) for c in col[row_ptr[v]:row_ptr[v + 1]]) for v in range(n)]


def within2(adj, v, active=None):
    """Vertices at distance 1 or 2 from v (v excluded), through active
    vertices only when `active` is given (induced subgraph)."""
    ok = (lambda u: True) if active is None else (lambda u: active[u])
    d1 = {u for u in adj[v] if ok(u)}
    out = set(d1)
    for u in d1:
        out |= {w for w in adj[u] if ok(w)}
    out.discard(v)
    return out


def luby_g2(n, adj, prio_fn, active=None):
    """Returns (sorted IN list, rounds).  prio_fn(r, v) -> comparable tuple."""
    verts = [v for v in range(n) if active is None or active[v]]
    g2 = {v: within2(adj, v, active) for v in verts}
    und = set(verts)
    IN = set()
    r = 0
    while und:
        t = {v: prio_fn(r, v) for v in und}
        new_in, new_out = set(), set()
        for v in und:
            if g2[v] & IN:
                new_out.add(v)
            elif all(t[v] < t[u] for u in g2[v] if u in und):
                new_in.add(v)
        IN |= new_in
        und -= new_in | new_out
        r += 1
    return sorted(IN), r


def luby_g2_hashed(row_ptr, col, seed=0, active=None):
    n = len(row_ptr) - 1
    adj = adjacency(row_ptr, col)
    return luby_g2(n, adj, lambda r, v: tuple_of(prio_hash(seed, r, v), v, n), active)


def check_mis2(adj, members, active=None):
    """Distance-2 independence and maximality (on the induced subgraph when
    `active` is given).  Returns an error string or None."""
    n = len(adj)
    S = set(members)
    verts = [v for v in range(n) if active is None or active[v]]
    for v in S:
        if active is not None and not active[v]:
            return "member %d outside the subgraph" % v
        if within2(adj, v, active) & S:
            return "members within distance 2 of %d" % v
    for v in verts:
        if v not in S and not (within2(adj, v, active) & S):
            return "vertex %d could be added" % v
    return None


def check_aggregation(row_ptr, col, agg, n_agg, roots1, roots2):
    """Invariants of Algorithm 3.  roots1/roots2: phase-1 roots and accepted
    phase-2 roots.  Returns an error string or None."""
    n = len(row_ptr) - 1
    adj = adjacency(row_ptr, col)
    agg = [int(a) for a in agg]
    if sorted(set(agg)) != list(range(n_agg)):
        return "labels are not exactly 0..n_agg-1"
    if check_mis2(adj, roots1):
        return "phase-1 roots are not an MIS-2"
    # phase 1: closed neighbourhoods of the roots, disjoint, numbered by id
    lab1 = [-1] * n
    for k, r in enumerate(sorted(roots1)):
        for u in adj[r] | {r}:
            if lab1[u] != -1:
                return "phase-1 aggregates overlap"
            lab1[u] = k
    # phase 2: roots form an MIS-2 of the unaggregated subgraph
    active = [lab1[v] == -1 for v in range(n)]
    lab2 = list(lab1)
    for k, r in enumerate(sorted(roots2)):
        unagg = [u for u in adj[r] if lab1[u] == -1]
        if len(unagg) < 2 or not active[r]:
            return "phase-2 root %d has fewer than 2 unaggregated neighbours" % r
        for u in unagg + [r]:
            if lab2[u] != -1:
                return "phase-2 aggregates overlap"
            lab2[u] = len(roots1) + k
    for v in range(n):
        if lab2[v] != -1 and agg[v] != lab2[v]:
            return "vertex %d: label differs from phases 1-2" % v
    # phase 3: argmax coupling, then min aggsize, then min id, over frozen labels
    size = {}
    for v in range(n):
        if lab2[v] != -1:
            size[lab2[v]] = size.get(lab2[v], 0) + 1
    for v in range(n):
        if lab2[v] != -1:
            continue
        coup = {}
        for u in adj[v]:
            if lab2[u] != -1:
                coup[lab2[u]] = coup.get(lab2[u], 0) + 1
        if not coup:
            return "phase-3 vertex %d has no aggregated neighbour" % v
        best = min(coup, key=lambda a: (-coup[a], size[a], a))
        if agg[v] != best:
            return "vertex %d joined %d, expected %d" % (v, agg[v], best)
    # every aggregate is connected and holds exactly one root
    members = {}
    for v in range(n):
        members.setdefault(agg[v], []).append(v)
    rootset = set(roots1) | set(roots2)
    for a, mem in members.items():
        ms = set(mem)
        if len(ms & rootset) != 1:
            return "aggregate %d holds %d roots" % (a, len(ms & rootset))
        seen, stack = {mem[0]}, [mem[0]]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y in ms and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if seen != ms:
            return "aggregate %d is not connected" % a
    return None


def check_basic_coarsening(row_ptr, col, agg, n_agg, roots):
    """Algorithm 2 from its statement: the roots are an MIS-2; each root with
    its neighbours is one aggregate (numbered by increasing root id); every
    other vertex takes, among the aggregates that hold one of its
    neighbours, the one with the smallest id.  Returns an error string or
    None."""
    n = len(row_ptr) - 1
    adj = adjacency(row_ptr, col)
    agg = [int(a) for a in agg]
    roots = sorted(roots)
    if n_agg != len(roots):
        return "n_agg %d != %d roots" % (n_agg, len(roots))
    if check_mis2(adj, roots):
        return "roots are not an MIS-2"
    ball = {k: adj[r] | {r} for k, r in enumerate(roots)}  # the first loop's aggregates
    for k, b in ball.items():
        for u in b:
            if agg[u] != k:
                return "vertex %d of root %d's neighbourhood has label %d" % (u, roots[k], agg[u])
    covered = set().union(*ball.values()) if ball else set()
    for v in range(n):
        if v in covered:
            continue
        touching = [k for k, b in ball.items() if adj[v] & b]
        if not touching:
            return "leftover vertex %d touches no aggregate" % v
        if agg[v] != min(touching):
            return "leftover vertex %d joined %d, expected %d" % (v, agg[v], min(touching))
    members = {}
    for v in range(n):
        members.setdefault(agg[v], set()).add(v)
    if sorted(members) != list(range(n_agg)):
        return "labels are not exactly 0..n_agg-1"
    for k, ms in members.items():
        seen, stack = {roots[k]}, [roots[k]]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y in ms and y not in seen:
                    seen.add(y)
                    stack.append(y)
        if seen != ms:
            return "aggregate %d is not connected to its root" % k
    return None


def quotient_pairs(row_ptr, col, agg):
    n = len(row_ptr) - 1
    out = set()
    for u in range(n):
        for e in range(row_ptr[u], row_ptr[u + 1]):
            a, c = int(agg[u]), int(agg[col[e]])
            if a != c:
                out.add((a, c))
    return out
