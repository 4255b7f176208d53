"""Writes grid3d6_464_oracle.json: the oracle's result on the 464^3 workload
(synthetic blob grid, 6-connected, seed 4): the maximum flow value and SHA-256
digests of the two extremal minimum cuts as row-major uint8 source-side
indicators (the minimal source side, and the maximal one = the paper's
(T-bar, T)).  The oracle's single-thread solve of 10^8 vertices takes minutes
and tens of GB, so its result is stored once; the GPU tests and the bench
compare against it.  Calls only the oracle and the input generator.

    python tests/golden/make_grid3d6_464.py
"""
import hashlib
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    oracle.build(force=False)
    inst = synth.config(4)
    t0 = time.perf_counter()
    ref = oracle.solve_grid(inst, method="pr")
    secs = time.perf_counter() - t0
    smin = np.ascontiguousarray(ref["smin"], np.uint8)
    smax = np.ascontiguousarray(ref["smax"], np.uint8)
    out = {
        "workload": "464^3 3D 6-connected blob grid, 256 blobs, seed 4 (synth.config(4))",
        "n": int(inst.n),
        "flow": int(ref["flow"]),
        "smin_sha256": hashlib.sha256(smin.tobytes()).hexdigest(),
        "smax_sha256": hashlib.sha256(smax.tobytes()).hexdigest(),
        "smin_count": int(smin.sum()),
        "smax_count": int(smax.sum()),
        "oracle": "highest-label push-relabel, 1 thread",
        "oracle_seconds": round(secs, 1),
        "host": platform.processor() or platform.machine(),
    }
    with open(os.path.join(HERE, "grid3d6_464_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
