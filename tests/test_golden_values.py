"""The stored oracle values under tests/golden belong to the current workloads and oracle:
the momenta digest matches, and a few events recomputed by the oracle agree exactly."""
import importlib.util
import os

import numpy as np

import oracle
from workloads import configs

_spec = importlib.util.spec_from_file_location(
    "make_oracle_values", os.path.join(os.path.dirname(__file__), "golden", "make_oracle_values.py"))
mov = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(mov)


def test_stored_oracle_values_are_current(card):
    for name, (key, n) in mov.SETS.items():
        w = configs.WORKLOADS[key]
        p = w.momenta(n)
        vals = mov.load(name, p)
        assert vals.shape == (n,) and np.all(vals > 0)
        idx = np.array([0, 1, n // 2, n - 1])
        again = oracle.me2(w.process, p[idx], card, mov.ALPHA_S)
        assert np.array_equal(again, vals[idx]), name
