"""Write grid_golden.json: expected flow values and minimal-cut hashes for the
full-size grid workloads, computed by the CPU oracle (FIFO push-relabel) only.

Run from the repository root: python tests/golden/make_grid_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def record(inst):
    v, side = oracle.grid_maxflow(inst, "fifo")
    return {"name": inst.name, "H": inst.H, "W": inst.W, "flow": int(v),
            "source_side_sha256": hashlib.sha256(side.tobytes()).hexdigest(),
            "source_side_count": int(side.sum())}


def main():
    out = {"generator": "synth.grid_batch(seed=0) and synth.grid_blobs(1024, 1024, seed)",
           "oracle": "oracle.grid_maxflow(inst, 'fifo')",
           "batch_seed0": [record(g) for g in synth.grid_batch(seed=0)],
           "blobs1024": [record(synth.grid_blobs(1024, 1024, seed=s)) for s in range(3)]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_golden.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
