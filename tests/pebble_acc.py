"""Exhaustive schedule search for one level of the accumulating product
C <- alpha*A*B + beta*C with A and B read-only: the pebble game of Section 4
on the computation graphs of the accumulating algorithms, test
infrastructure.

A graph fixes the values and how each is computed; the search chooses the
order and the memory placement, as Section 4's program does.  Values:

* ``pre``: a pre-addition S_i / T_i of Section 2 (x + sign*y over quadrants
  of A and B or other pre-additions).  A pre-addition may be formed again
  after its block was reused (as Table 9 forms T1 and T2 twice), up to
  ``max_recompute`` times;
* ``mul``: alpha * x * y by a read-only recursive call, into a block that
  holds neither operand;
* ``acc``: sign * alpha * x * y + s * v by a read-only accumulating recursive
  call, which lands in v's block (v is not needed afterwards);
* ``lin``: x + c * y, an addition row, c in {1, -1, beta, -beta}.

The quadrants C11..C22 hold the blocks of C at the start (values "C11" ..
"C22") and must hold the four results at the end; ``temps`` extra blocks of
the same size are available; A and B are never written.  Moves follow the
pebble rules: compute into a free block (rule 3), compute in place over an
operand that is not needed afterwards (rule 2), free a block whose value
nothing needs (rule 1); copies (rule 4) are not used.  Depth first with a
memo of exhausted states: "no schedule" covers every order and placement of
the graph under these rules.
"""
from functools import lru_cache

A_IN = ("A11", "A12", "A21", "A22", "B11", "B12", "B21", "B22")
C_IN = ("C11", "C12", "C21", "C22")
B = "beta"

# Section 2's pre-additions.
PRE = {
    "S1": ("pre", "A21", "A22", 1), "S2": ("pre", "S1", "A11", -1),
    "S3": ("pre", "A11", "A21", -1), "S4": ("pre", "A12", "S2", -1),
    "T1": ("pre", "B12", "B11", -1), "T2": ("pre", "B22", "T1", -1),
    "T3": ("pre", "B22", "B12", -1), "T4": ("pre", "T2", "B21", -1),
}

# Table 9's graph: Z-type combinations of C, accumulating calls with beta,
# one beta-scaled row, the post-additions.  Names give the value each node
# holds: Q5 = P5 + beta Z3, Q6 = P6 + beta C21, W1 = Q5 + beta Z1,
# Q3 = P3 + Q5, Q2 = P2 + beta C11, U3 = P7 + U2, U6 = U3 - P4.
ACC = dict(PRE, **{
    "Z1": ("lin", "C22", "C12", -1), "Z3": ("lin", "C12", "C21", -1),
    "Q5": ("acc", "S1", "T1", "Z3", B, 1), "Q6": ("acc", "S2", "T2", "C21", B, 1),
    "W1": ("lin", "Q5", "Z1", B), "Q3": ("acc", "S4", "B22", "Q5", 1, 1),
    "P1": ("mul", "A11", "B11"), "U2": ("lin", "Q6", "P1", 1),
    "Q2": ("acc", "A12", "B21", "C11", B, 1), "U1": ("lin", "P1", "Q2", 1),
    "U5": ("lin", "U2", "Q3", 1), "U3": ("acc", "S3", "T3", "U2", 1, 1),
    "U7": ("lin", "U3", "W1", 1), "U6": ("acc", "A22", "T4", "U3", 1, -1),
})

# Table 2's graph: P5 and P1 by plain calls, the beta terms by addition rows
# and accumulating calls.  V22 = P5 + beta C22, V12 = P5 + beta C12,
# V11 = P1 + beta C11, U2 = P6 + P1, U1 = P2 + V11, Q3 = P3 + V12,
# Q4 = P4 - beta C21, U5 = U2 + Q3, U3 = P7 + U2, U7 = U3 + V22, U6 = U3 - Q4.
HL = dict(PRE, **{
    "P5": ("mul", "S1", "T1"), "V22": ("lin", "P5", "C22", B),
    "V12": ("lin", "P5", "C12", B), "P1": ("mul", "A11", "B11"),
    "V11": ("lin", "P1", "C11", B), "U2": ("acc", "S2", "T2", "P1", 1, 1),
    "U1": ("acc", "A12", "B21", "V11", 1, 1), "Q3": ("acc", "S4", "B22", "V12", 1, 1),
    "U5": ("lin", "U2", "Q3", 1), "Q4": ("acc", "A22", "T4", "C21", "-beta", 1),
    "U3": ("acc", "S3", "T3", "U2", 1, 1), "U7": ("lin", "U3", "V22", 1),
    "U6": ("lin", "U3", "Q4", -1),
})

GRAPHS = {"table9": ACC, "table2": HL}
FINAL = {"U1": 0, "U5": 1, "U6": 2, "U7": 3}


def parents(g, v):
    op = g[v]
    if op[0] in ("pre", "lin", "mul"):
        return op[1:3]
    return op[1:4]


def _consumers(g):
    out = {}
    for v in g:
        for u in parents(g, v):
            out.setdefault(u, []).append(v)
    return out


def search(graph, temps, max_recompute=2, max_pre=None):
    """Return (moves, stats): the first schedule found, or None.

    ``max_pre`` caps the total number of pre-additions formed (8 when
    none is formed twice); ``least_additions`` raises it from 8 until a
    schedule appears.

    A move is (value, block): block is one of C11..C22, or "pool:<value>" for
    the extra block holding <value> (an operand overwritten in place, or a
    pre-addition taken over), "pool:None" for a free extra block."""
    g = GRAPHS[graph] if isinstance(graph, str) else graph
    pre = [v for v in g if g[v][0] == "pre"]
    main = [v for v in g if g[v][0] != "pre"]
    consumers = _consumers(g)
    order = {v: i for i, v in enumerate(list(C_IN) + list(g))}
    stats = {"states": 0}

    @lru_cache(maxsize=None)
    def needed(v, done):
        if v in FINAL:
            return True
        for x in consumers.get(v, ()):
            if g[x][0] == "pre":
                if needed(x, done):
                    return True
            elif x not in done:
                return True
        return False

    def norm(done, pool, cs):
        pool = tuple(sorted((x if x is not None and needed(x, done) else None for x in pool),
                            key=lambda x: -1 if x is None else order[x]))
        cs = tuple(x if x is not None and needed(x, done) else None for x in cs)
        return pool, cs

    def where(v, pool, cs):
        if v in A_IN:
            return ("in", None)
        if v in pool:
            return ("pool", pool.index(v))
        if v in cs:
            return ("c", cs.index(v))
        return None

    def dead_after(u, v, after, pool, cs):
        # u may be overwritten by v in place: nothing but v still needs it
        # (a pre-addition that uses u and is needed again but no longer
        # present would need u to form it)
        if u in FINAL:
            return False
        for x in consumers.get(u, ()):
            if x == v:
                continue
            if g[x][0] == "pre":
                if needed(x, after) and where(x, pool, cs) is None:
                    return False
            elif x not in after:
                return False
        return True

    @lru_cache(maxsize=None)
    def dfs(done, pool, cs, counts):
        stats["states"] += 1
        if len(done) == len(main):
            return ()
        for v in main + pre:
            if v in done:
                continue
            op = g[v]
            if op[0] == "pre":
                k = pre.index(v)
                if counts[k] >= max_recompute or where(v, pool, cs) or not needed(v, done):
                    continue
                if max_pre is not None and sum(counts) >= max_pre:
                    continue
            ps = parents(g, v)
            locs = [where(u, pool, cs) for u in ps]
            if any(l is None for l in locs):
                continue
            after = done | {v} if op[0] != "pre" else done
            if op[0] == "acc":
                lv = locs[2]
                if lv[0] == "in" or lv in locs[:2] or needed(ps[2], after):
                    continue
                if v in FINAL and lv != ("c", FINAL[v]):
                    continue
                dests = [lv]
            else:
                dests = []
                if v in FINAL:
                    if cs[FINAL[v]] is None:
                        dests.append(("c", FINAL[v]))
                else:
                    if None in pool:
                        dests.append(("pool", pool.index(None)))
                    dests += [("c", i) for i in range(4) if cs[i] is None]
                    # a block holding a pre-addition may be taken over: the
                    # pre-addition is formed again when it is needed
                    dests += [("pool", i) for i, x in enumerate(pool)
                              if x is not None and g[x][0] == "pre" and ("pool", i) not in locs]
                    dests += [("c", i) for i, x in enumerate(cs)
                              if x is not None and x in g and g[x][0] == "pre"
                              and ("c", i) not in locs]
                if op[0] == "mul":
                    dests = [d for d in dests if d not in locs]
                else:
                    for u, l in zip(ps, locs):
                        if l[0] == "in" or (v in FINAL and l != ("c", FINAL[v])):
                            continue
                        if dead_after(u, v, after, pool, cs):
                            dests.append(l)
            for d in dict.fromkeys(dests):
                p2, c2 = list(pool), list(cs)
                if d[0] == "pool":
                    p2[d[1]] = v
                else:
                    c2[d[1]] = v
                cnt = counts
                if op[0] == "pre":
                    k = pre.index(v)
                    cnt = counts[:k] + (counts[k] + 1,) + counts[k + 1:]
                np_, nc = norm(after, p2, c2)
                rest = dfs(after, np_, nc, cnt)
                if rest is not None:
                    where_to = C_IN[d[1]] if d[0] == "c" else "pool:%s" % (pool[d[1]],)
                    return ((v, where_to),) + rest
        return None

    p0, c0 = norm(frozenset(), (None,) * temps, C_IN)
    found = dfs(frozenset(), p0, c0, (0,) * len(pre))
    dfs.cache_clear()
    needed.cache_clear()
    return (None if found is None else list(found)), stats


def value_of(g, v, env, alpha, beta, mul):
    """The value of node v from its parents' values in env."""
    op = g[v]
    coef = {1: 1, -1: -1, B: beta, "-beta": -beta}
    if op[0] == "pre":
        return env[op[1]] + env[op[2]] * op[3]
    if op[0] == "lin":
        return env[op[1]] + env[op[2]] * coef[op[3]]
    if op[0] == "mul":
        return mul(env[op[1]], env[op[2]]) * alpha
    _, x, y, w, s, sign = op
    return mul(env[x], env[y]) * (alpha * sign) + env[w] * coef[s]


def to_rows(graph, moves, temps):
    """Physical rows of a found schedule: every value gets a block (C11..C22,
    X, Y, Z, ...); every read is checked against what its block holds at that
    point.  Returns [(value, op kind, destination, operand blocks)] in order."""
    g = GRAPHS[graph] if isinstance(graph, str) else graph
    extra = ["XYZW"[i] for i in range(temps)]
    holds = {c: c for c in C_IN}
    holds.update({x: None for x in extra})
    home = {c: c for c in C_IN}
    consumers = _consumers(g)
    done = set()

    def live(u):
        if u in FINAL:
            return True
        for x in consumers.get(u, ()):
            if g[x][0] == "pre":
                if live(x):
                    return True
            elif x not in done:
                return True
        return False

    rows = []
    for v, dest in moves:
        op = g[v]
        ps = parents(g, v)
        blocks = []
        for u in ps:
            if u in A_IN:
                blocks.append(u)
            else:
                assert u in home and holds[home[u]] == u, "%s read, its block holds %s" % (
                    u, holds.get(home.get(u)))
                blocks.append(home[u])
        if op[0] != "pre":
            done.add(v)
        if op[0] == "acc":
            block = home[ps[2]]
        elif not dest.startswith("pool:"):
            block = dest
        else:
            target = dest[5:]
            if target != "None":
                cands = [x for x in extra if holds[x] == target]
            else:
                cands = [x for x in extra if (holds[x] is None or not live(holds[x]))
                         and x not in blocks]
            assert cands, "no block for %s" % v
            block = cands[0]
        rows.append((v, op[0], block, tuple(blocks)))
        holds[block] = v
        home[v] = block
    for v, ci in FINAL.items():
        assert holds[C_IN[ci]] == v, "%s does not end in %s" % (v, C_IN[ci])
    return rows


def run_rows(graph, rows, A, B_, C, alpha, beta, p, mul):
    """Execute physical rows on blocks (numpy arrays reduced mod p, or formal
    symbols with p None).  A, B_ and C are lists of quadrants 11, 12, 21, 22;
    returns the final C quadrants."""
    g = GRAPHS[graph] if isinstance(graph, str) else graph
    mem = dict(zip(("A11", "A12", "A21", "A22"), A))
    mem.update(zip(("B11", "B12", "B21", "B22"), B_))
    mem.update(zip(C_IN, C))
    for v, kind, block, blocks in rows:
        env = {u: mem[b] for u, b in zip(parents(g, v), blocks)}
        val = value_of(g, v, env, alpha, beta, mul)
        mem[block] = val % p if p else val
    return [mem[c] for c in C_IN]


def least_additions(graph, temps, max_recompute=2):
    """The schedule with the fewest pre-additions under ``temps`` extra
    blocks (None if there is none at all), with that count."""
    g = GRAPHS[graph] if isinstance(graph, str) else graph
    npre = sum(1 for v in g if g[v][0] == "pre")
    for cap in range(npre, npre * max_recompute + 1):
        moves, _ = search(graph, temps, max_recompute, max_pre=cap)
        if moves is not None:
            return moves, cap
    return None, None



BLOCK_IDS = {"C11": 0, "C12": 1, "C21": 2, "C22": 3, "A11": 4, "A12": 5, "A21": 6, "A22": 7,
             "B11": 8, "B12": 9, "B21": 10, "B22": 11, "X": 12, "Y": 13, "Z": 14, "W": 15}
COEF_CODES = {1: 1, -1: 2, B: 3, "-beta": 4}        # the library's WS_COEF_* codes


def library_rows(graph, rows):
    """The physical rows as the library's row records:
    (op, dst, x, y, cx, cy, cs, sign) with op 0 = addition, 1 = product,
    2 = accumulating product."""
    g = GRAPHS[graph] if isinstance(graph, str) else graph
    out = []
    for v, kind, block, blocks in rows:
        op = g[v]
        ids = [BLOCK_IDS[b] for b in blocks]
        if kind == "pre":
            out.append((0, BLOCK_IDS[block], ids[0], ids[1], 1, COEF_CODES[op[3]], 0, 0))
        elif kind == "lin":
            out.append((0, BLOCK_IDS[block], ids[0], ids[1], 1, COEF_CODES[op[3]], 0, 0))
        elif kind == "mul":
            out.append((1, BLOCK_IDS[block], ids[0], ids[1], 0, 0, 0, 1))
        else:
            assert BLOCK_IDS[block] == ids[2]
            out.append((2, BLOCK_IDS[block], ids[0], ids[1], 0, 0, COEF_CODES[op[4]], op[5]))
    return out
