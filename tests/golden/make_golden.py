"""Writes the stored expected values under tests/golden/.

Calls only the seeded generator (``synth``) and the CPU oracle (``oracle/``):
* synth_hashes.json   - SHA-256 digests of generated inputs (determinism pin)
* oracle_sphere16.json - digests and counters of the oracle's sphere_16 run in
  each form (a regression pin of the oracle itself)

Run from the repository root:  python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import oracle  # noqa: E402
from helpers import problem_of  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE = 4096


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def synth_hashes() -> dict:
    out = {}
    for name, make in synth.WORKLOADS.items():
        w = make()
        entry = {}
        for s in range(len(w.species)):
            entry[f"species{s}_first{SAMPLE}"] = digest(*synth.particles(w, s, 0, SAMPLE))
            last = w.species[s].count - SAMPLE
            entry[f"species{s}_last{SAMPLE}"] = digest(*synth.particles(w, s, last, SAMPLE))
        if w.nodes <= 400_000:
            entry["node_E"] = digest(*synth.node_E(w))
        out[name] = entry
    return out


def oracle_sphere16() -> dict:
    w = synth.sphere_16()
    sp, x, v = synth.all_particles(w)
    E = synth.node_E(w)
    out = {}
    for form in ("fp64", "fp32_abs", "fp32_cell"):
        r = oracle.run(problem_of(w, form), sp, x, v, E, w.steps)
        alive = r.fate == 0
        out[form] = {
            "steps": w.steps,
            "alive": [int((alive & (sp == s)).sum()) for s in range(2)],
            "absorbed": r.tally.sum(0).tolist(),
            "escaped": r.escaped.tolist(),
            "rho_fixed_sum": int(r.rho_fixed.sum()),
            "rho_fixed_sha256": digest(r.rho_fixed),
            "state_sha256": digest(r.x, r.v, r.fate, r.where, r.when),
        }
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "synth_hashes.json"), "w") as f:
        json.dump(synth_hashes(), f, indent=1, sort_keys=True)
    with open(os.path.join(HERE, "oracle_sphere16.json"), "w") as f:
        json.dump(oracle_sphere16(), f, indent=1, sort_keys=True)
    print("written")
