"""Readers for the small text fixtures under tests/golden/ (values printed in the paper)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def matrices(name):
    """{name: {"rows": int ndarray, "rho": [...], "d": [...]}} from 'matrix' sections."""
    out, cur, extra = {}, None, {}
    for line in _lines(name):
        tok = line.split()
        if tok[0] == "matrix":
            cur, rows, extra = tok[1], [], {}
        elif tok[0] == "end":
            out[cur] = dict(extra, rows=np.array(rows, dtype=np.int64))
            cur = None
        elif cur is not None and tok[0] == "rho":
            extra["rho"] = [float(v) for v in tok[1:]]
        elif cur is not None and tok[0] == "d":
            extra["d"] = [int(v) for v in tok[1:]]
        elif cur is not None:
            rows.append([int(v) for v in tok])
        elif tok[0] == "adds":
            out.setdefault("_adds", {})[tok[1]] = int(tok[2])
    return out


def table(name):
    """Whitespace table -> list of token lists."""
    return [line.split() for line in _lines(name)]


def integers(name):
    vals = []
    for line in _lines(name):
        vals.extend(int(v) for v in line.split())
    return vals
