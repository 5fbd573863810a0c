"""Write the stored expected values of the GPU parity tests.

Calls only the oracle (oracle/rtcc3.py) and the seeded input generators.
Run: python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rtcc3 as orc  # noqa: E402
from paper_2407_18947_amd.inputs import CONFIGS, config_field, initial_state, make_system  # noqa: E402


def monomer(steps=None):
    c = CONFIGS["monomer"]
    steps = c["steps"] if steps is None else steps
    s = make_system(c["o"], c["v"], seed=c["seed"])
    m = orc.Model.from_system(s)
    f = config_field("monomer", steps)
    t0 = time.time()
    y, mu = orc.propagate(m, initial_state(s), c["dt"], f, triples="loop")
    print(f"monomer: {steps} steps in {time.time() - t0:.1f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "monomer_20steps.npz"), mu=mu.numpy(), y=y.numpy(),
                        steps=steps, dt=c["dt"], seed=c["seed"])


if __name__ == "__main__":
    torch.set_num_threads(os.cpu_count() or 8)
    monomer()
