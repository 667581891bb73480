"""Write spectra.json: the eigenvalues around the gap (HOMO, LUMO) and the
spectral range of the synthetic workloads, from a dense symmetric
eigensolver.  These are inputs of the purification (the tolerance schedule
needs bounds of the gap) and of the accuracy checks; they come from the
workload definition alone.

    python tests/golden/make_spectra.py [name ...]
"""
import json
import os
import sys
import time

import numpy as np
import scipy.linalg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

WORKLOADS = {
    "sys3d_n16384_s2_b64": lambda: synth.sys3d(16384, 2, 64),
    "sys3d_n4096_s6_b64": lambda: synth.sys3d(4096, 6, 64),
    "chain1d_n1024_s1_b32": lambda: synth.chain1d(1024, 1, 32),
}


def main(names):
    path = os.path.join(HERE, "spectra.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        t = time.time()
        M = WORKLOADS[name]()
        D = M.to_dense()
        n = D.shape[0]
        h = n // 2
        w = scipy.linalg.eigh(D, eigvals_only=True, subset_by_index=[h - 2, h + 1], overwrite_a=True,
                              driver="evr")
        ends = scipy.linalg.eigh(M.to_dense(), eigvals_only=True, subset_by_index=[0, 0], driver="evr")
        top = scipy.linalg.eigh(M.to_dense(), eigvals_only=True, subset_by_index=[n - 1, n - 1], driver="evr")
        out[name] = {"n": n, "n_occ": h, "homo": float(w[1]), "lumo": float(w[2]),
                     "around_gap": [float(x) for x in w], "lmin": float(ends[0]), "lmax": float(top[0]),
                     "seconds": round(time.time() - t, 1)}
        print(name, out[name], flush=True)
        json.dump(out, open(path, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
