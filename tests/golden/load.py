"""Reader for the small hand-worked fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """Return {'n': n, '<Name>': (n, n) array, ...} from a fixture file."""
    out, cur, rows = {}, None, []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "n":
                out["n"] = int(tok[1])
            elif tok[0].isalpha():
                if cur is not None:
                    out[cur] = np.array(rows, dtype=np.float64)
                cur, rows = tok[0], []
            else:
                rows.append([float(t) for t in tok])
    if cur is not None:
        out[cur] = np.array(rows, dtype=np.float64)
    return out
