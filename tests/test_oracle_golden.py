"""The oracle reproduces the stored golden vectors (written by
tests/golden/make_golden.py from the oracle alone).  Any change to the hash,
gradient maps or octave sum shows up here."""
import json
import os

import numpy as np

import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lattice_fbm.json")


def _doc():
    with open(GOLD) as fh:
        return json.load(fh)


def test_golden_keys_and_gradients():
    d = _doc()
    for e in d["keys2"]:
        k = O.key2(e["ix"], e["iy"], e["octave"], e["seed"])
        assert k == e["key"]
        np.testing.assert_allclose(O.grad2(k), e["grad"], rtol=0, atol=1e-15)
    for e in d["keys3"]:
        k = O.key3(e["ix"], e["iy"], e["iz"], e["octave"], e["seed"])
        assert k == e["key"]
        assert O.key3_second(k) == e["key_second"]
        np.testing.assert_allclose(O.grad3(k), e["grad"], rtol=0, atol=1e-15)


def test_golden_fbm_samples():
    for e in _doc()["fbm"]:
        if e["dim"] == 2:
            v = O.fbm_points_2d(e["smooth"], e["octaves"], e["persistence"], e["lacunarity"], e["base_freq"],
                                e["seed"], [e["x"]], [e["y"]])[0]
        else:
            v = O.fbm_points_3d(e["smooth"], e["octaves"], e["persistence"], e["lacunarity"], e["base_freq"],
                                e["seed"], [e["x"]], [e["y"]], [e["z"]])[0]
        assert abs(v - e["value"]) < 1e-15
