"""Shared helpers for the GPU tests (comparison metrics and run drivers)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def rel(a, b):
    """max|a - b| / max|b| (per-field relative error against the reference b)."""
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / den) if den > 0 else float(np.abs(a - b).max())


def fp64_spread():
    with open(os.path.join(HERE, "golden", "fp64_spread.json")) as fh:
        return json.load(fh)["spread"]


def oracle_params(orc, p):
    return orc.params(**p.as_dict())


def say(*a):
    print(*a, flush=True)
