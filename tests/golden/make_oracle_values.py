"""Write FP64 oracle values for workloads whose oracle evaluation is too slow to repeat in a
GPU test (gg -> ttbar ggg: a few events per second per core).

Calls only the CPU oracle and the seeded input generators.  Each stored value comes with a
checksum of its event's momenta (the sum of the absolute values of its components); the test
recomputes the momenta on its own machine and requires every checksum to agree to 1e-12
relative before it uses the values (the extended-precision generator need not give the same
last bits on every CPU, and such differences move |M|^2 by far less than the tolerances the
stored values serve).

    python tests/golden/make_oracle_values.py [name ...]
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import configs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
ALPHA_S = 0.118

# name -> (workload, number of leading events)
SETS = {"ggttggg_2048": ("ggttggg", 2048)}


def momenta_checksums(p: np.ndarray) -> np.ndarray:
    return np.abs(np.asarray(p, dtype=np.float64)).reshape(len(p), -1).sum(axis=1)


def path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.txt")


def load(name: str, p: np.ndarray) -> np.ndarray:
    """The stored values for `name`, after checking they were computed on these momenta."""
    data = np.loadtxt(path(name), dtype=np.float64, comments="#")
    vals, sums = data[:, 0], data[:, 1]
    here = momenta_checksums(p)
    if len(vals) != len(p) or not np.all(np.abs(here / sums - 1) <= 1e-12):
        raise ValueError(f"{name}: stored values belong to other momenta")
    return vals


def write(name: str) -> None:
    key, n = SETS[name]
    w = configs.WORKLOADS[key]
    p = w.momenta(n)
    card = configs.card_array()
    vals = oracle.me2(w.process, p, card, ALPHA_S)
    with open(path(name), "w") as f:
        f.write(f"# FP64 oracle |M|^2, {configs.PROCESS_NAMES[w.process]}, first {n} events of the "
                f"{key} workload (sqrt(s) = {w.sqrt_s} GeV, seed {w.seed}), alpha_s = {ALPHA_S}\n")
        f.write("# columns: |M|^2, sum of |components| of the event's momenta (a checksum of the input)\n")
        f.write("# written by tests/golden/make_oracle_values.py (oracle only)\n")
        for v, c in zip(vals, momenta_checksums(p)):
            f.write(f"{v:.17e} {c:.17e}\n")


if __name__ == "__main__":
    for name in sys.argv[1:] or SETS:
        write(name)
        print("wrote", path(name))
