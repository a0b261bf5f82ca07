"""The oracle against its stored outputs in tests/golden/ (a drift check).

The paper prints no worked example with reproducible inputs, so the fixture
holds the float64 oracle's own answers for 64 rays on the 1,280-face
icosphere, written by tests/golden/make_golden.py.  This test pins the oracle
to that earlier state, not to the mathematics (the pins in test_oracle_pins.py
do that): a change to the oracle's arithmetic fails here until the fixture is
regenerated in a commit that names the passage that justifies it.  The GPU
path is compared with the same fixture in test_gpu_forward.py.
"""
import numpy as np

import oracle
from golden_io import load
from workloads import configs as CF


def test_oracle_matches_fixture():
    ins, ref = load()
    assert ins["f"].shape[0] == 64
    X, F = CF.mesh_config(1)
    o = oracle.Mesh(X, F).exp(ins["f"], ins["b"], ins["v"], ins["W"])
    for k in ("f", "status", "n_cross"):
        assert np.array_equal(o[k].astype(np.int64), ref[k].astype(np.int64)), k
    assert np.array_equal(o["hash"], ref["hash"])
    for k in ("p", "b", "v", "W", "min_vdist"):
        assert np.allclose(o[k], ref[k], rtol=1e-14, atol=1e-15), (k, np.abs(o[k] - ref[k]).max())


def test_fixture_inputs_are_the_config1_rays():
    """The stored inputs are the first config-1 rays (float32 values kept exactly)."""
    ins, _ = load()
    X, F = CF.mesh_config(1)
    r = CF.rays_config(1, X, F)
    assert np.array_equal(ins["f"], r["f"][:64])
    for k in ("b", "v", "W"):
        assert np.array_equal(ins[k], r[k][:64]), k
