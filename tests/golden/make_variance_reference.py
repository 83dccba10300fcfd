"""Write variance_reference.json: the deterministic long-range SOG pressure
P^F (Theorem 1: the full k-space sum over every mode, M = 10, Table 1 row 2
scaled to the cutoff) of the seeded disordered ionic systems of the
benchmark's estimator study, so that the benchmark can report each sampler's bias and
mean squared error against it.  Calls the oracle only.

usage: python tests/golden/make_variance_reference.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2602_23582_amd import workloads as W  # noqa: E402

SIZES = (2000, 16000)


def main():
    out = {"note": "P^F of W.ionic_melt(n, seed=11) by the oracle's full k-space SOG sum "
                   "(sog_kspace_full), Table 1 row 2 at M = 10, Gaussian units; row-major 3x3",
           "systems": {}}
    for n in SIZES:
        d = W.ionic_melt(n, seed=11)
        p = orc.sog(d["rc"], row=2, M=10)
        _, PF, UF = orc.sog_kspace_full(d["q"], d["pos"], d["L"], p, forces=False)
        out["systems"][str(n)] = {"L": d["L"].tolist(), "rc": d["rc"], "PF": PF.ravel().tolist(), "UF": UF}
        print(n, PF.ravel(), flush=True)
    with open(os.path.join(HERE, "variance_reference.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
