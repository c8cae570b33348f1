"""Writes tests/golden/kappa_c.json: kappa_c of the 8^4 gradient-check field (links exp(0.5 i Q),
seed 104) and its rightmost eigenvalues of the hopping matrix, computed by the oracle alone
(restarted Arnoldi via ARPACK on H; several minutes of CPU time).

    python tests/golden/make_kappa_c.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import kappa as K  # noqa: E402
from oracle import wilson as W  # noqa: E402

FIELDS = [dict(name="c4_8x8x8x8", L=(8, 8, 8, 8), c=0.5, seed=104)]


def main():
    out = {"source": "oracle.kappa.kappa_c (scipy ARPACK, which='LR', tol 1e-12) on the synth "
                     "gauge fields below; kappa_c = 1 / max Re lambda(H)", "fields": []}
    for f in FIELDS:
        lat = W.Lattice(f["L"])
        U = synth.gauge_field(f["L"], f["c"], f["seed"])
        t = time.time()
        kc, vals, res = K.kappa_c(U, lat, nev=3, tol=1e-12)
        out["fields"].append(dict(f, L=list(f["L"]), kappa_c=kc,
                                  lambda_re=[float(v.real) for v in vals],
                                  lambda_im=[float(v.imag) for v in vals],
                                  eigen_residual=float(res), seconds=round(time.time() - t, 1)))
        print(out["fields"][-1], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "kappa_c.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
