"""Exhaustive schedule search for one level of Winograd's C = A*B (the pebble
game of Section 4), test infrastructure.

The graph is Section 2's: pre-additions S1..S4 / T1..T4, seven products and
the post-additions U1..U7 (U2 = P1 + P6, U3 = U2 + P7, U4 = U2 + P5,
U1 = P1 + P2, U5 = U4 + P3, U6 = U3 - P4, U7 = U3 + P5), with U1, U5, U6, U7
to be left in C11, C12, C21, C22.  Memory is the twelve quadrants of A, B and
C plus ``temps`` extra blocks of the same size.  A search state records which
values are computed and where the live ones sit; a move computes one value:

* an addition into a free block, or in place over one of its operands when
  that operand is not needed afterwards (the pebble rules 0-2: compute,
  free, compute in place);
* a product by a recursive call into a free block distinct from its operands.
  The call may destroy its operands as its kind says (a read-only call, the
  in-place call of Table 3 that destroys both, or a call destroying only the
  left or only the right operand); a destroyed operand must not be needed
  afterwards and must not be an input the schedule has to keep.

Inputs the schedule may not overwrite stay in place throughout.  Values that
nothing needs any more free their block.  Blocks outside C that hold no live
value are interchangeable, so the state keeps them as a multiset; the C
quadrants are kept by position because the results must land there.  The
search is a depth-first exploration with a memo of exhausted states, so a
"no schedule" answer covers every order and placement under these rules.
Copies (rule 4) and other bracketings of the post-additions are not explored.
"""
from functools import lru_cache

INPUTS = ["A11", "A12", "A21", "A22", "B11", "B12", "B21", "B22"]
# value: (kind, left, right, sign); kind "+" for additions, "*" for products
GRAPH = {
    "S1": ("+", "A21", "A22", 1), "S2": ("+", "S1", "A11", -1),
    "S3": ("+", "A11", "A21", -1), "S4": ("+", "A12", "S2", -1),
    "T1": ("+", "B12", "B11", -1), "T2": ("+", "B22", "T1", -1),
    "T3": ("+", "B22", "B12", -1), "T4": ("+", "T2", "B21", -1),
    "P1": ("*", "A11", "B11", 1), "P2": ("*", "A12", "B21", 1), "P3": ("*", "S4", "B22", 1),
    "P4": ("*", "A22", "T4", 1), "P5": ("*", "S1", "T1", 1), "P6": ("*", "S2", "T2", 1),
    "P7": ("*", "S3", "T3", 1),
    "U2": ("+", "P1", "P6", 1), "U3": ("+", "U2", "P7", 1), "U4": ("+", "U2", "P5", 1),
    "U1": ("+", "P1", "P2", 1), "U5": ("+", "U4", "P3", 1), "U6": ("+", "U3", "P4", -1),
    "U7": ("+", "U3", "P5", 1),
}
FINAL = {"U1": 0, "U5": 1, "U6": 2, "U7": 3}          # index into C11, C12, C21, C22
CNAMES = ["C11", "C12", "C21", "C22"]
NODES = list(GRAPH)
CONSUMERS = {v: [x for x, (_, l, r, _) in GRAPH.items() if v in (l, r)] for v in INPUTS + NODES}

# Kinds of recursive calls: which operands (left, right) a call destroys.
READ_ONLY, IN_PLACE, LEFT, RIGHT = (False, False), (True, True), (True, False), (False, True)


def search(temps, writable, calls):
    """Find a schedule, or prove there is none under the rules above.

    temps: number of extra blocks; writable: the input names the schedule
    may overwrite (a subset of INPUTS); calls: the allowed call kinds.
    Returns a list of moves (value, destination, call kind or None) or None.
    """
    kept = frozenset(v for v in INPUTS if v not in writable)
    order = {v: i for i, v in enumerate(INPUTS + NODES)}

    def needed(v, done):
        return v in kept or v in FINAL or any(x not in done for x in CONSUMERS[v])

    def normalise(done, pool, cslots):
        pool = tuple(sorted((x if x is not None and needed(x, done) else None for x in pool),
                            key=lambda x: -1 if x is None else order[x]))
        cslots = tuple(x if x is not None and needed(x, done) else None for x in cslots)
        return pool, cslots

    n_pool = len(writable) + temps
    pool0 = tuple(sorted(writable, key=order.get)) + (None,) * temps
    start = (frozenset(), pool0, (None,) * 4)

    def where(v, pool, cslots):
        if v in kept:
            return ("kept", None)
        if v in pool:
            return ("pool", pool.index(v))
        if v in cslots:
            return ("c", cslots.index(v))
        return None

    @lru_cache(maxsize=None)
    def dfs(done, pool, cslots):
        if len(done) == len(NODES):
            return ()
        for v in NODES:
            if v in done:
                continue
            kind, l, r, _ = GRAPH[v]
            wl, wr = where(l, pool, cslots), where(r, pool, cslots)
            if wl is None or wr is None:
                continue
            after = done | {v}
            dead_l, dead_r = not needed(l, after), not needed(r, after)
            dests = []
            if v in FINAL:
                ci = FINAL[v]
                if cslots[ci] is None:
                    dests.append(("c", ci))
                for w, dead in ((wl, dead_l), (wr, dead_r)):
                    if kind == "+" and dead and w == ("c", ci):
                        dests.append(w)
            else:
                if None in pool:
                    dests.append(("pool", pool.index(None)))
                dests += [("c", i) for i in range(4) if cslots[i] is None]
                if kind == "+":
                    for w, dead in ((wl, dead_l), (wr, dead_r)):
                        if dead and w[0] != "kept":
                            dests.append(w)
            if kind == "*":
                ok = [c for c in calls
                      if (not c[0] or (dead_l and wl[0] != "kept"))
                      and (not c[1] or (dead_r and wr[0] != "kept"))]
                if not ok:
                    continue
                call = ok[0]
                dests = [d for d in dests if d != wl and d != wr]
            else:
                call = None
            for d in dict.fromkeys(dests):
                p2, c2 = list(pool), list(cslots)
                if d[0] == "pool":
                    p2[d[1]] = v
                else:
                    c2[d[1]] = v
                np_, nc = normalise(after, p2, c2)
                rest = dfs(after, np_, nc)
                if rest is not None:
                    dest = CNAMES[d[1]] if d[0] == "c" else "pool"
                    return ((v, dest, call),) + rest
        return None

    pool, cslots = normalise(*start)
    found = dfs(start[0], pool, cslots)
    dfs.cache_clear()
    return None if found is None else list(found)


def replay_physical(moves, temps, writable, mul, add, inputs):
    """Run a found schedule on named physical blocks, independently of the
    search's bookkeeping: A11..B22 hold ``inputs``, X0.. are the extra
    blocks, C11..C22 the results.  A "pool" destination takes a free block
    among the writable inputs and the extra blocks (the block of an operand
    the addition consumes last, if there is one).  Every read checks that the
    block still holds the value it expects; a destroyed operand's block is
    marked junk.  Returns the values left in C11, C12, C21, C22 and the kept
    inputs' blocks."""
    mem = {v: (v, inputs[v]) for v in INPUTS}
    extra = ["X%d" % i for i in range(temps)]
    for b in extra + CNAMES:
        mem[b] = (None, None)
    home = {v: v for v in INPUTS}
    kept = [v for v in INPUTS if v not in writable]
    done = set()

    def live(v):
        return v in kept or v in FINAL or any(x not in done for x in CONSUMERS[v])

    def free(b):
        name = mem[b][0]
        return name is None or name == "junk" or not live(name)

    for v, dest, call in moves:
        kind, l, r, sign = GRAPH[v]
        for u in (l, r):
            assert mem[home[u]][0] == u, "%s read from a block that no longer holds it" % u
        x, y = mem[home[l]][1], mem[home[r]][1]
        val = mul(x, y) if kind == "*" else add(x, y, sign)
        done.add(v)
        if dest != "pool":
            block = dest
            assert free(block) or (kind == "+" and mem[block][0] in (l, r)), "occupied"
        else:
            spare = [home[u] for u in (l, r) if kind == "+" and not live(u)
                     and home[u] in list(writable) + extra]
            cands = spare or [b for b in list(writable) + extra if free(b)
                              and b not in (home[l], home[r])]
            assert cands, "no free block"
            block = cands[0]
        if call is not None:
            for u, destroys in zip((l, r), call):
                if destroys:
                    assert not live(u) and u not in kept, "destroyed a needed operand"
                    mem[home[u]] = ("junk", None)
        mem[block] = (v, val)
        home[v] = block
    for v in kept:
        assert mem[v][0] == v
    return [mem[c][1] if mem[c][0] in FINAL else None for c in CNAMES], {v: mem[v][1] for v in kept}
