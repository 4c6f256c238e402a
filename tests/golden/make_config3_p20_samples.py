"""Writes config3_p20_samples.json: the oracle's two-level solution of the 4x4x4-box,
p = 20 problem (configuration 3's second case), sampled at seeded interior and
interface nodes, plus the l2 norms of the full solution vectors.

Uses only oracle/ and workloads/ (FP64 NumPy/SciPy, dense LAPACK for the 46,656-unknown
interface system; about 10 minutes and 25 GB on 8 cores):

    python tests/golden/make_config3_p20_samples.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import interface as oi  # noqa: E402

N_INTERIOR, N_FACE, SEED = 512, 256, 20


def main():
    prob = W.config3_p20()
    ref = oi.solve(prob, keep_boxes=False, dense=True, progress=lambda msg: print(msg, flush=True))
    rng = np.random.default_rng(SEED)
    nbox, n_i = ref.u_i.shape
    flat = rng.choice(nbox * n_i, size=N_INTERIOR, replace=False)
    fidx = rng.choice(ref.u_face.size, size=N_FACE, replace=False)
    out = {
        "problem": prob.name, "nboxes": list(prob.nboxes), "p": prob.p, "kappa": prob.kappa,
        "source": "oracle.interface.solve (FP64), written by tests/golden/make_config3_p20_samples.py",
        "interior_box": (flat // n_i).tolist(), "interior_node": (flat % n_i).tolist(),
        "interior_value": ref.u_i.reshape(-1)[flat].tolist(),
        "face_index": fidx.tolist(), "face_value": ref.u_face[fidx].tolist(),
        "norm_u_i": float(np.linalg.norm(ref.u_i)), "norm_u_face": float(np.linalg.norm(ref.u_face)),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_p20_samples.json"), "w") as fh:
        json.dump(out, fh, indent=None)
        fh.write("\n")


if __name__ == "__main__":
    main()
