"""Readers for the text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def philox_kat():
    out = []
    for line in _lines("philox4x32_10_kat.txt"):
        w = [int(x, 16) for x in line.split()]
        out.append((w[0:4], w[4:6], w[6:10]))
    return out


def graver_closed_forms():
    out = []
    for line in _lines("graver_closed_forms.txt"):
        name, arows, R, elems = [s.strip() for s in line.split("|")]
        A = np.array([[int(x) for x in r.split()] for r in arows.split(";")], dtype=np.int64)
        G = [tuple(int(x) for x in e.split()) for e in elems.split(";")]
        out.append((name, A, int(R), G))
    return out


def tiny_graver_box6():
    """{seed: set of tuples} from tiny_graver_box6.txt."""
    out = {}
    cur = None
    for line in _lines("tiny_graver_box6.txt"):
        if line.startswith("seed"):
            parts = line.split()
            cur = int(parts[1])
            out[cur] = set()
        else:
            out[cur].add(tuple(int(x) for x in line.split()))
    return out


def augment_golden(name):
    """(inputs_sha256, best, rows) of an augmentation fixture; rows are
    (moves, f bits, x_end) per start."""
    rows = []
    head = None
    for line in _lines(name):
        w = line.split()
        if w[0] == "inputs":
            head = (w[1], int(w[9]))
            continue
        rows.append((int(w[1]), int(w[2], 16), np.array([int(v) for v in w[3:]], dtype=np.int64)))
    return head[0], head[1], rows
