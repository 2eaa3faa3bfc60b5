"""Readers of the paper's printed examples under tests/golden/ (test infrastructure)."""
import os

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(HERE, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def fig61_lists():
    """{(kind, box): [boxes]} in the paper's numbering (kind: child, nei, int)."""
    return {(row[0], int(row[1])): [int(v) for v in row[2:]] for row in _lines("fig61_lists.txt")}


def table1_ranks():
    """{eps: [P for each box side]} of Table 1."""
    eps = (1e-6, 1e-8, 1e-10, 1e-13)
    rows = _lines("table1_ranks.txt")
    return {e: [int(r[1 + k]) for r in rows] for k, e in enumerate(eps)}


def paper_number(level, x, y):
    """Box number of the Fig. 6.1 reading: levels in order from 1, Morton order (x bit lowest)."""
    m = 0
    for b in range(level):
        m |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
    return (4 ** level - 1) // 3 + 1 + m
