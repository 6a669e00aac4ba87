"""Reader for the text fixtures in tests/golden (hexadecimal floats)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    mats = {}
    with open(os.path.join(GOLDEN, name)) as f:
        lines = [ln for ln in f.read().splitlines() if ln and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        key, r, c = lines[i].split()
        r, c = int(r), int(c)
        rows = [[float.fromhex(t) for t in lines[i + 1 + j].split()] for j in range(r)]
        mats[key] = np.array(rows, dtype=np.float64).reshape(r, c)
        i += 1 + r
    return mats
