"""The schedule search of Section 4 (one level of C = A*B, tests/pebble.py).

* For the constraints of the paper's one-level schedules -- Table 1 (inputs
  kept, two temporaries, read-only calls), Table 3 (both inputs overwritten,
  no temporary, in-place calls), Table 4 (A overwritten, one temporary) and
  Table 5 (B overwritten, one temporary) -- the search finds a schedule, and
  each found schedule, run on named blocks holding formal symbols, leaves
  exactly the product in C and the kept inputs untouched.
* The claim of Section 5: no schedule overwrites only one of A and B without
  an extra temporary (its calls then being in-place ones or itself).
* With the inputs kept, one temporary is not enough either: two, as in
  Table 1, is the least.
"""
import pytest

from . import pebble as pb
from .test_oracle_symbolic import Sym

A = ["A11", "A12", "A21", "A22"]
B = ["B11", "B12", "B21", "B22"]


def _symbolic_inputs():
    out = {}
    for i, name in enumerate(A):
        out[name] = Sym.atom(("a", i // 2, i % 2))
    for i, name in enumerate(B):
        out[name] = Sym.atom(("b", i // 2, i % 2))
    return out


def _product(x):
    return [x["A11"] * x["B11"] + x["A12"] * x["B21"], x["A11"] * x["B12"] + x["A12"] * x["B22"],
            x["A21"] * x["B11"] + x["A22"] * x["B21"], x["A21"] * x["B12"] + x["A22"] * x["B22"]]


PAPER = [
    # (schedule, extra blocks, writable inputs, call kinds)
    ("Table 1", 2, [], [pb.READ_ONLY]),
    ("Table 3", 0, A + B, [pb.IN_PLACE]),
    ("Table 4", 1, A, [pb.IN_PLACE, pb.LEFT]),
    ("Table 5", 1, B, [pb.IN_PLACE, pb.RIGHT]),
]


@pytest.mark.parametrize("name,temps,writable,calls", PAPER)
def test_search_finds_the_papers_schedules(name, temps, writable, calls):
    moves = pb.search(temps, writable, calls)
    assert moves is not None, name
    assert sorted(v for v, _, _ in moves) == sorted(pb.NODES)       # each value once
    x = _symbolic_inputs()
    c, kept = pb.replay_physical(moves, temps, writable, lambda u, w: u * w,
                                 lambda u, w, s: u + w * s, x)
    assert all(got == want for got, want in zip(c, _product(x)))
    assert all(kept[v] == x[v] for v in kept)


@pytest.mark.parametrize("writable,calls", [(A, [pb.IN_PLACE, pb.LEFT]),
                                            (B, [pb.IN_PLACE, pb.RIGHT])])
def test_no_schedule_overwrites_one_input_without_a_temporary(writable, calls):
    assert pb.search(0, writable, calls) is None


def test_kept_inputs_need_two_temporaries():
    assert pb.search(0, [], [pb.READ_ONLY]) is None
    assert pb.search(1, [], [pb.READ_ONLY]) is None
    assert pb.search(2, [], [pb.READ_ONLY]) is not None


def test_replay_catches_a_dead_read():
    """The physical replay is a check of its own: a schedule whose moves are
    taken out of order reads a block that no longer holds its value."""
    moves = pb.search(0, A + B, [pb.IN_PLACE])
    # the first product destroys both operands; move a later reader of one of
    # them after it
    first = next(i for i, (v, _, _) in enumerate(moves) if pb.GRAPH[v][0] == "*")
    operands = pb.GRAPH[moves[first][0]][1:3]
    earlier = [i for i in range(first) if set(pb.GRAPH[moves[i][0]][1:3]) & set(operands)]
    if not earlier:
        pytest.skip("no reader of the destroyed operands before the first product")
    bad = list(moves)
    bad.insert(first + 1, bad.pop(earlier[-1]))
    with pytest.raises(AssertionError):
        pb.replay_physical(bad, 0, A + B, lambda u, w: u * w, lambda u, w, s: u + w * s,
                           _symbolic_inputs())
