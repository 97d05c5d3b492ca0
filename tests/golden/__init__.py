import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def paper_values() -> dict:
    out = {}
    with open(os.path.join(_HERE, "paper_values.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (s.strip() for s in line.split("="))
                out[k] = float(v)
    return out


def mrt_matrix() -> np.ndarray:
    return np.loadtxt(os.path.join(_HERE, "mrt_matrix.txt"))
