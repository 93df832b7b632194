"""Write the oracle regression fixture `oracle_paths.json`.

The paper prints no per-path values for a worked example, so this fixture is
not a pin of the oracle: it is the oracle's own output on a few seeded points
(f, p, score and path record) for three small scenes, stored so that any later
change to the oracle's arithmetic shows up as a failing CPU test, and so that
the device can be checked against stored oracle values without running the
oracle.  It calls only `oracle/` (and the seeded input generators).

    python tests/golden/make_golden.py     (from the repository root)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402
from paper_2605_08916_amd import inputs  # noqa: E402

# (case name, scene factory name, path length L, points, point seed, film window)
CASES = [
    ("tiny_L4", "cornell_tiny", 4, 16, 101, 1.0),
    ("specular_box_L8", "specular_box", 8, 24, 102, 1.0),
    ("mirror_plane_L3", "mirror_plane", 3, 8, 103, 0.15),  # film block near the centre: the light's image
]


def points(d, n, seed, window):
    """Seeded points; the film block scaled into the central `window` of the film."""
    u = inputs.random_points(d, n, seed).astype(np.float64)
    u[:, :2] = 0.5 + (u[:, :2] - 0.5) * window
    return u


def compute():
    out = {"note": "oracle output (FP64) on seeded points; regression fixture written by make_golden.py",
           "eps": 1e-8, "cases": []}
    for name, factory, L, n, seed, window in CASES:
        sc = getattr(inputs, factory)()
        u = points(4 * (L - 1), n, seed, window)
        f, p, score, rec = orc.Scene(sc).path_eval(L, u, eps=1e-8)
        out["cases"].append({
            "name": name, "scene": factory, "L": L, "seed": seed, "n": n, "window": window,
            "u": u.tolist(), "f": f.tolist(), "p": p.tolist(), "score": score.tolist(),
            "rec": rec.astype(np.int64).tolist(),
        })
    return out


def main():
    path = os.path.join(HERE, "oracle_paths.json")
    with open(path, "w") as fh:
        json.dump(compute(), fh, indent=None, separators=(",", ":"))
        fh.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
