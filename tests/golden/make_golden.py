"""Writes oracle_icosphere3_64rays.txt: 64 rays of the 1,280-face icosphere
(the first rays of the config-1 batch: |v| ~ U[0, pi/2], one transported
vector) and the float64 oracle's answers for them.

The paper prints no worked example with reproducible inputs (its accuracy
table is measured on meshes it does not give), so this fixture holds the
oracle's own outputs.  It freezes them: a later change to the oracle's
arithmetic shows up in tests/test_golden.py and must regenerate this file
in a commit that names the passage, or the reading of it, that justifies
the change.  Calls only oracle/ and the seeded input generators.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle                                  # noqa: E402
from workloads import configs as CF            # noqa: E402

N = 64
OUT = os.path.join(HERE, "oracle_icosphere3_64rays.txt")
COLUMNS = ("f b0 b1 b2 v0 v1 v2 w0 w1 w2 | f_out status n_cross hash p0 p1 p2 bo0 bo1 bo2 "
           "vo0 vo1 vo2 wo0 wo1 wo2 min_vdist")


def main():
    X, F = CF.mesh_config(1)
    r = CF.rays_config(1, X, F)
    f, b, v, W = r["f"][:N], r["b"][:N], r["v"][:N], r["W"][:N]
    o = oracle.Mesh(X, F).exp(f, b, v, W)
    with open(OUT, "w") as fh:
        fh.write("# float64 oracle on the 1,280-face icosphere (config 1 mesh), first 64 config-1 rays, K = 1\n")
        fh.write("# written by tests/golden/make_golden.py; inputs are the float32 values, given exactly\n")
        fh.write("# columns: " + COLUMNS + "\n")
        for i in range(N):
            ins = [str(int(f[i]))] + [repr(float(x)) for x in (*b[i], *v[i], *W[i, 0])]
            outs = [str(int(o["f"][i])), str(int(o["status"][i])), str(int(o["n_cross"][i])), str(int(o["hash"][i]))]
            outs += ["%.17g" % x for x in (*o["p"][i], *o["b"][i], *o["v"][i], *o["W"][i, 0], o["min_vdist"][i])]
            fh.write(" ".join(ins) + " | " + " ".join(outs) + "\n")
    print(OUT)


if __name__ == "__main__":
    main()
