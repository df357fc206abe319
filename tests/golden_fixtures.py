"""Readers of the cited fixtures under tests/golden/ (values the paper prints)."""

import os

import numpy as np


def load_model1():
    """The paper's printed Model 1 (tests/golden/model1_vti.txt): (C0 in Pa, rho, printed background c11, c44 in Pa)."""
    vals = {}
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "model1_vti.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *nums = line.split()
        if key.startswith("C_row"):
            rows.append([float(v) for v in nums])
        else:
            vals[key] = float(nums[0])
    C = np.zeros((6, 6))
    for i, r in enumerate(rows):
        C[i, i:] = r
    C = (C + C.T - np.diag(np.diag(C))) * 1e9
    return C, vals["density_kg_m3"], vals["background_c11"] * 1e9, vals["background_c44"] * 1e9
