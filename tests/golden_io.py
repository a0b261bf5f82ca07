"""Reader of the oracle fixture in tests/golden/ (see make_golden.py there)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_icosphere3_64rays.txt")


def load(path=GOLDEN):
    """Returns (inputs, outputs): inputs f, b, v, W (float32 values, K = 1);
    outputs f, status, n_cross, hash, p, b, v, W, min_vdist (float64)."""
    rows = [ln.split("|") for ln in open(path) if ln.strip() and not ln.startswith("#")]
    a = [ln[0].split() for ln in rows]
    z = [ln[1].split() for ln in rows]
    n = len(rows)
    ins = dict(f=np.array([int(x[0]) for x in a], np.int32),
               b=np.array([[float(t) for t in x[1:4]] for x in a], np.float32),
               v=np.array([[float(t) for t in x[4:7]] for x in a], np.float32),
               W=np.array([[float(t) for t in x[7:10]] for x in a], np.float32).reshape(n, 1, 3))
    outs = dict(f=np.array([int(x[0]) for x in z], np.int32), status=np.array([int(x[1]) for x in z], np.int32),
                n_cross=np.array([int(x[2]) for x in z], np.int64), hash=np.array([int(x[3]) for x in z], np.uint64),
                p=np.array([[float(t) for t in x[4:7]] for x in z]), b=np.array([[float(t) for t in x[7:10]] for x in z]),
                v=np.array([[float(t) for t in x[10:13]] for x in z]),
                W=np.array([[float(t) for t in x[13:16]] for x in z]).reshape(n, 1, 3),
                min_vdist=np.array([float(x[16]) for x in z]))
    return ins, outs
