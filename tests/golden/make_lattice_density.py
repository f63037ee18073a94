"""Writes lattice_density.json: D = m sum_k W(|k| dx) on an infinite cubic lattice, m = dx^3.

Uses the Wendland functions in their standard support-radius form (support H = 2h):
  C2: W = 21/(2 pi H^3) (1-s)^4 (1+4s),           s = r/H
  C4: W = 495/(32 pi H^3) (1-s)^6 (1+6s+35 s^2/3)
Independent of the oracle (no import of it).
"""
import json
import math
import os

import numpy as np


def lattice_density(kind, eta):
    dx = 1.0
    H = 2.0 * eta * dx
    R = int(math.ceil(H / dx)) + 1
    g = np.arange(-R, R + 1)
    k = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(float)
    r = np.sqrt((k**2).sum(1)) * dx
    s = r[r < H] / H
    if kind == "WC2":
        W = 21.0 / (2 * math.pi * H**3) * (1 - s) ** 4 * (1 + 4 * s)
    else:
        W = 495.0 / (32 * math.pi * H**3) * (1 - s) ** 6 * (1 + 6 * s + 35.0 / 3.0 * s * s)
    return float(dx**3 * W.sum()), int(s.size)


if __name__ == "__main__":
    eta100 = (3.0 * 100.0 / (32.0 * math.pi)) ** (1.0 / 3.0)
    out = {"_source": __doc__.strip().splitlines()[0] + " Written by tests/golden/make_lattice_density.py.",
           "eta100": eta100}
    for name, kind, eta in (("WC2_eta1.3", "WC2", 1.3), ("WC4_eta1.3", "WC4", 1.3),
                            ("WC4_eta100", "WC4", eta100)):
        D, cnt = lattice_density(kind, eta)
        out[name] = {"D": D, "neighbours_incl_self": cnt}
    path = os.path.join(os.path.dirname(__file__), "lattice_density.json")
    json.dump(out, open(path, "w"), indent=2)
    print(json.dumps(out, indent=2))
