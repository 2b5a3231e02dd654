"""Parser of tests/golden/threshold_pairs.txt (hand-derived fixtures)."""
import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "threshold_pairs.txt")
CLASSES = {"none": 0, "safe": 1, "pb": 2, "pc": 3}


def load():
    cases, cur = [], None
    with open(PATH) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "case":
                cur = dict(name=tok[1], points=[], pairs={}, active={})
            elif tok[0] == "end":
                cur["points"] = np.ascontiguousarray(np.array(cur["points"], dtype=np.float32).T)
                cases.append(cur)
                cur = None
            elif tok[0] in ("b", "xi"):
                cur[tok[0]] = float(tok[1])
            elif tok[0] == "box":
                cur["box"] = tuple(float(v) for v in tok[1:4])
            elif tok[0] == "point":
                cur["points"].append([float(v) for v in tok[1:4]])
            elif tok[0] == "pair":
                cur["pairs"][(int(tok[1]), int(tok[2]))] = CLASSES[tok[3]]
            elif tok[0] in ("fof", "safe"):
                cur[tok[0]] = np.array([int(v) for v in tok[1:]], dtype=np.int32)
            elif tok[0] == "active":
                v = [int(x) for x in tok[2:]]
                cur["active"][tok[1]] = sorted(zip(v[0::2], v[1::2]))
    return cases
