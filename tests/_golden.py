"""Readers for the fixtures under tests/golden/ (paper values with citations)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


def rational(name):
    """(p coefficients high->low, q coefficients high->low, bound, vmax) as strings."""
    p, q, meta = [], [], {}
    for parts in _lines(name):
        if parts[0] == "p":
            p.append(parts[1])
        elif parts[0] == "q":
            q.append(parts[1])
        else:
            meta[parts[0]] = parts[1]
    return p, q, float(meta["bound"]), float(meta["vmax"])


def keyed(name):
    """name -> list of string fields for 'key value...' fixtures."""
    out = {}
    for parts in _lines(name):
        out.setdefault(parts[0], []).append(parts[1:])
    return out
