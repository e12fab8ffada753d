"""Writes tests/golden/tiny16_oracle.json: residual and Jacobian rows of the
16x16x16 workload (seed 1) at fixed cells, computed by the oracle only.
It is a regression fixture for the oracle's arithmetic: a change to it must
name, in its commit message, the passage of the paper that justifies it.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import geomodel  # noqa: E402
import oracle  # noqa: E402

CELLS = [0, 1, 15, 16, 255, 256, 1000, 2047, 2048, 3000, 4080, 4095]


def main():
    geo = geomodel.tiny16()
    p = oracle.pressure(geo)
    r, J, s = oracle.rows(geo.grid, geo.fluid, geo.kx, p, np.array(CELLS), ry=geo.ry,
                          rz=geo.rz, seal=geo.seal)
    pref = oracle.hydrostatic(geo.grid, geo.fluid)
    doc = {
        "workload": "16x16x16, sigma 1, isotropic, no seals, seed 1 (geomodel.tiny16)",
        "source": "oracle only (tests/golden/make_golden.py)",
        "cells": CELLS,
        "r": [float.hex(float(v)) for v in r],
        "J": [[float.hex(float(v)) for v in row] for row in J],
        "scale": [[float.hex(float(v)) for v in row] for row in s],
        "pref": [float.hex(float(v)) for v in pref],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny16_oracle.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
