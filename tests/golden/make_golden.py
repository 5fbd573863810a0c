"""Write the stored expected values of the GPU parity tests.

Calls only the oracle (oracle/rtcc3.py) and the seeded input generators
(paper_2407_18947_amd/inputs.py).  The cases that would take the oracle more
than a minute are stored here instead of being recomputed by each test run.

Run: python tests/golden/make_golden.py [case ...]
cases: monomer, dimer, trimer_terms, o17v24_terms, o16v66_terms, pentamer_sampled (default: all)
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import rtcc3 as orc  # noqa: E402
from paper_2407_18947_amd.inputs import (CONFIGS, config_field, initial_state, make_system,  # noqa: E402
                                         random_state)

# Right-hand-side terms at full workload sizes: seeded random states (scale 0.02)
# at a static field.
TERMS_FIELD = np.array([0.001, -0.002, 0.002])
TERMS_CASES = {
    "trimer_terms": dict(o=15, v=57, seed=3, state_seed=8, scale=0.02),
    "o17v24_terms": dict(o=17, v=24, seed=12, state_seed=4, scale=0.1),
    # o > 15 with v > 64: the separate sweep over blocks wider than one wave
    "o16v66_terms": dict(o=16, v=66, seed=13, state_seed=5, scale=0.05),
}
PENTAMER = dict(o=25, v=95, seed=5, state_seed=9, scale=0.02)
# doubles rows (i, j) stored for the trimer: X2[i,j,:,:] and Y2[i,j,:,:]
TRIMER_ROWS = [(0, 0), (3, 7), (14, 2)]
DIMER_STEPS = 30


def _save(name, **arrays):
    np.savez_compressed(os.path.join(HERE, name + ".npz"), **arrays)


def monomer(steps=None):
    c = CONFIGS["monomer"]
    steps = c["steps"] if steps is None else steps
    s = make_system(c["o"], c["v"], seed=c["seed"])
    m = orc.Model.from_system(s)
    f = config_field("monomer", steps)
    t0 = time.time()
    y, mu = orc.propagate(m, initial_state(s), c["dt"], f, triples="loop")
    print(f"monomer: {steps} steps in {time.time() - t0:.1f} s", flush=True)
    _save("monomer_20steps", mu=mu.numpy(), y=y.numpy(), steps=steps, dt=c["dt"], seed=c["seed"])


def dimer(steps=DIMER_STEPS):
    """Dimer workload (o=10, v=38, seed 2, sine field under a Gaussian envelope along z),
    the first `steps` RK4 steps of dt = 0.05 in FP64."""
    c = CONFIGS["dimer"]
    s = make_system(c["o"], c["v"], seed=c["seed"])
    m = orc.Model.from_system(s)
    f = config_field("dimer", steps)
    t0 = time.time()

    def cb(n, y):
        print(f"  dimer step {n + 1}/{steps} ({time.time() - t0:.0f} s)", flush=True)

    y, mu = orc.propagate(m, initial_state(s), c["dt"], f, triples="loop", callback=cb)
    print(f"dimer: {steps} steps in {time.time() - t0:.1f} s", flush=True)
    _save(f"dimer_{steps}steps", mu=mu.numpy(), y=y.numpy(), steps=steps, dt=c["dt"], seed=c["seed"])


def terms(name):
    """Every term of the right-hand side (oracle's loop over all blocks, with the
    density) at a seeded random state: X1, Y1, D, mu in full, doubles rows of X2, Y2."""
    c = TERMS_CASES[name]
    o, v = c["o"], c["v"]
    s = make_system(o, v, seed=c["seed"])
    m = orc.Model.from_system(s)
    y = random_state(o, v, c["state_seed"], c["scale"])
    t0 = time.time()
    r = orc.rhs_terms(m, y, TERMS_FIELD, triples="loop")
    print(f"{name}: all terms in {time.time() - t0:.1f} s", flush=True)
    rows = TRIMER_ROWS if name == "trimer_terms" else [(0, 0), (o - 1, 2)]
    out = {k: r[k].numpy() for k in ("X1", "Y1", "D", "mu", "R1", "G1")}
    out["rows"] = np.array(rows)
    for k in ("X2", "Y2", "R2", "G2"):
        out[k + "_rows"] = np.stack([r[k][i, j].numpy() for i, j in rows])
    _save(name, field=TERMS_FIELD, **out)


def pentamer_sampled():
    """o=25, v=95 (seed 5): X1[0] (blocks with first occupied index 0), X2[0,0] and
    Y2[0,0] (blocks with second index 0), and the CCSD parts R1, G1, R2[0,0], G2[0,0]."""
    c = PENTAMER
    o, v = c["o"], c["v"]
    s = make_system(o, v, seed=c["seed"])
    m = orc.Model.from_system(s)
    y = random_state(o, v, c["state_seed"], c["scale"])
    t0 = time.time()
    ccsd = orc.rhs_terms(m, y, TERMS_FIELD, with_triples=False, with_density=False)
    print(f"pentamer: CCSD part in {time.time() - t0:.1f} s", flush=True)
    with torch.no_grad():
        t1, t2, l1, l2 = orc.unpack(m, y)
        ti = orc.TriplesIntegrals(orc.Dressed(m, t1, m.h(TERMS_FIELD)))
        part = orc.triples_loop(m, ti, t2, l1, l2, only=lambda i, j, k: i == 0 or j == 0)
    print(f"pentamer: sampled triples in {time.time() - t0:.1f} s", flush=True)
    _save("pentamer_sampled", field=TERMS_FIELD, X1_0=part["X1"][0].numpy(), X2_00=part["X2"][0, 0].numpy(),
          Y2_00=part["Y2"][0, 0].numpy(), R1=ccsd["R1"].numpy(), G1=ccsd["G1"].numpy(),
          R2_00=ccsd["R2"][0, 0].numpy(), G2_00=ccsd["G2"][0, 0].numpy())


CASES = {
    "monomer": monomer,
    "dimer": dimer,
    "trimer_terms": lambda: terms("trimer_terms"),
    "o17v24_terms": lambda: terms("o17v24_terms"),
    "o16v66_terms": lambda: terms("o16v66_terms"),
    "pentamer_sampled": pentamer_sampled,
}

if __name__ == "__main__":
    torch.set_num_threads(int(os.environ.get("GOLDEN_THREADS", os.cpu_count() or 8)))
    for name in sys.argv[1:] or list(CASES):
        CASES[name]()
