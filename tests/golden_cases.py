"""Loader for the hand-worked fixtures under tests/golden/."""
import json
import os

import numpy as np

import mspgen

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _csr(d):
    vals = None if "values" not in d else np.asarray(d["values"], np.float64)
    return mspgen.CSR(d["nrows"], d["ncols"], np.asarray(d["rowptr"], np.int64),
                      np.asarray(d["colidx"], np.int32), vals)


def hand_example():
    with open(os.path.join(HERE, "hand_example.json")) as f:
        g = json.load(f)
    return _csr(g["A"]), _csr(g["B"]), _csr(g["M"]), g["expect"]
