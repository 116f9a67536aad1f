"""Write tests/golden/acc_search.json: the schedules the accumulating search
(tests/pebble_acc.py, Section 4's pebble game on the graphs of Tables 9 and
2) finds with the fewest temporaries and, among those, the fewest
pre-additions, with the search's proofs that fewer do not exist.

Run from the repository root:  python -m tests.golden.make_acc_search
"""
import json
import os
import sys

from tests import pebble_acc as pa

sys.setrecursionlimit(10000)
HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    out = {"note": "written by tests/golden/make_acc_search.py from tests/pebble_acc.py"}
    for graph, temps in (("table9", 2), ("table2", 3)):
        fewer = {}
        for t in range(temps):
            moves, st = pa.search(graph, t)
            assert moves is None
            fewer[str(t)] = st["states"]
        moves, npre = pa.least_additions(graph, temps)
        fewer_pre = {}
        for cap in range(8, npre):
            m2, st = pa.search(graph, temps, max_pre=cap)
            assert m2 is None
            fewer_pre[str(cap)] = st["states"]
        rows = pa.to_rows(graph, moves, temps)
        out[graph] = {"temps": temps, "pre_additions": npre,
                      "no_schedule_with_temps": fewer, "no_schedule_with_pre_additions": fewer_pre,
                      "moves": [list(m) for m in moves],
                      "rows": [[v, kind, block, list(blocks)] for v, kind, block, blocks in rows],
                      "library_rows": pa.library_rows(graph, rows)}
        print(graph, temps, "temporaries,", npre, "pre-additions", flush=True)
    with open(os.path.join(HERE, "acc_search.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
