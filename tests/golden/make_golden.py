"""Write the golden vectors under tests/golden/ from the FP64 oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The stored values pin the stated lattice hash, gradient maps and a few fBm samples
so that any later change to the oracle's arithmetic shows up as a diff here.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

NODES = [
    (0, 0, 0, 1), (1, 0, 0, 1), (0, 1, 0, 1), (-1, -1, 3, 2), (2 ** 33 + 5, -(3 * 2 ** 20 + 7), 9, 3),
    (-(2 ** 46), 2 ** 46 - 1, 11, 0xDEADBEEF), (123456789, -987654321, 15, 0xFFFFFFFF),
    ((2 ** 24 - 3) * 512 // 512, -(2 ** 24 - 5), 0, 1),
]


def main():
    keys2 = []
    for ix, iy, o, s in NODES:
        k = O.key2(ix, iy, o, s)
        keys2.append({"ix": ix, "iy": iy, "octave": o, "seed": s, "key": k,
                      "grad": [float(v) for v in O.grad2(k)]})
    keys3 = []
    for ix, iy, o, s in NODES:
        iz = (ix ^ iy) % 1000 - 500
        k = O.key3(ix, iy, iz, o, s)
        keys3.append({"ix": ix, "iy": iy, "iz": iz, "octave": o, "seed": s, "key": k,
                      "key_second": O.key3_second(k), "grad": [float(v) for v in O.grad3(k)]})
    fbm = []
    for smooth in (1, 2):
        for (x, y) in [(0, 0), (17, 201), (-3 * 2 ** 20 - 7, 2 ** 33 + 5)]:
            v = O.fbm_points_2d(smooth, 4, 0.5, 2.0, 8 / 256, 1, [x], [y])[0]
            fbm.append({"dim": 2, "smooth": smooth, "octaves": 4, "persistence": 0.5, "lacunarity": 2.0,
                        "base_freq": 8 / 256, "seed": 1, "x": x, "y": y, "value": float(v)})
    for smooth in (1, 2):
        v = O.fbm_points_3d(smooth, 6, 0.5, 2.0, 8 / 512, 1, [3], [77], [401])[0]
        fbm.append({"dim": 3, "smooth": smooth, "octaves": 6, "persistence": 0.5, "lacunarity": 2.0,
                    "base_freq": 8 / 512, "seed": 1, "x": 3, "y": 77, "z": 401, "value": float(v)})
    doc = {"source": "tests/golden/make_golden.py (FP64 oracle)", "keys2": keys2, "keys3": keys3, "fbm": fbm}
    with open(os.path.join(HERE, "lattice_fbm.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
