"""Reader of the hand-derived golden fixtures in this folder."""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """(R, S, pairs, tiles): float32 rectangles, the expected sorted (r, s)
    pairs and the reporting tile (tx, ty) of each pair."""
    R, S, P = {}, {}, []
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            if line[0] in "RS":
                (R if line[0] == "R" else S)[int(line[1])] = [float(v) for v in line[2:6]]
            elif line[0] == "P":
                P.append([int(v) for v in line[1:5]])
    Ra = np.array([R[i] for i in sorted(R)], np.float32)
    Sa = np.array([S[i] for i in sorted(S)], np.float32)
    P = np.array(sorted(P), np.int64)
    return Ra, Sa, P[:, :2].astype(np.int32), P[:, 2:]
