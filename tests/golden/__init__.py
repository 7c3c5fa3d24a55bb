"""Stored values with their citations (paper or published generator)."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        return [l.split() for l in f if l.strip() and not l.startswith("#")]


def philox_kat():
    """(counters uint32[n,4], 64-bit seeds = key0 | key1 << 32, outputs uint32[n,4])."""
    r = [[int(v, 16) for v in row] for row in _rows("philox4x32_10_kat.txt")]
    a = np.array(r, dtype=np.uint64)
    seeds = [int(k0) | (int(k1) << 32) for k0, k1 in a[:, 4:6]]
    return a[:, :4].astype(np.uint32), seeds, a[:, 6:].astype(np.uint32)


def eq8_rows():
    """(lattice, T_C, eps, z, J) rows."""
    return [(l, float(t), float(e), int(z), float(j)) for l, t, e, z, j in _rows("eq8_exchange_from_tc.txt")]
