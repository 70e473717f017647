"""Writes fullsize_d6.json: oracle facts about the benchmark workload (d=6,
2000 support vectors, degree 3, scale 0.06, batch triangulation with k=4)
that the oracle computes in under a minute although it cannot trace the
whole fine set: the number of coarse intersecting edges and of coarse
n-simplices (Sec. V-B).

Run from the repository root:  python tests/golden/make_fullsize.py
It calls only the oracle and the seeded input generators."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2406_04795_amd import inputs as I  # noqa: E402


def main():
    O.build(force=False)
    wl = I.config_c3(eps=2e-5, k=4)
    cv, cm = O.trace_direct(wl, coarse_k=wl.k)
    sig = O.batch_sigma(wl)
    out = {
        "workload": wl.name,
        "recipe": "paper_2406_04795_amd.inputs.config_c3(eps=2e-5, k=4)",
        "coarse_edges": int(len(cv)),
        "coarse_simplices": int(len(sig)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_d6.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(out)


if __name__ == "__main__":
    main()
