"""Writes c3_scene.json: the collision share of the d=6 workload's scene on
cells of that workload, for the scene streams 200..215, and the stream the
workload uses (inputs.C3_SCENE_STREAM).

The cells: for every seed, the batch trace (same f, scale and k) inside the
sub-box of half-width 0.12 around it, up to 1500 of its cells, their
intersection points and the verdicts at those points, all from the oracle.
The share of a stream is the fraction of those points in collision.

Run from the repository root:  python tests/golden/make_c3_scene.py
It calls only the oracle and the seeded input generators."""
import copy
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2406_04795_amd import inputs as I  # noqa: E402


def cell_points(wl, half=0.12, n_max=1500):
    out = []
    for i, s in enumerate(wl.seeds):
        sub = copy.copy(wl)
        sub.dom = I.Domain(lo=np.maximum(wl.dom.lo, s - half), hi=np.minimum(wl.dom.hi, s + half))
        sub.seeds = wl.seeds[i:i + 1]
        v, m, _ = O.trace_batch(sub)
        if len(v) == 0:
            continue
        idx = np.random.default_rng(i).choice(len(v), min(n_max, len(v)), replace=False)
        pts, _ = O.points(sub, v[idx], m[idx])
        out.append(pts)
    return out


def main():
    O.build(force=False)
    wl = I.config_c3(eps=2e-5, k=4)
    P = cell_points(wl)
    Q = np.concatenate(P)
    scan = {}
    for stream in range(200, 216):
        sc = I.spatial_arm_scene(np.random.default_rng(stream), 6, spheres_per_link=3, sphere_r=0.05,
                                 n_osph=8, n_obox=8, obst_ball=I.C3_OBST_BALL)
        scan[stream] = {"share": float(O.check(sc, Q).mean()),
                        "per_seed": [round(float(O.check(sc, p).mean()), 3) for p in P]}
    chosen = scan[I.C3_SCENE_STREAM]
    assert 0.3 <= chosen["share"] <= 0.8, chosen
    assert O.check(wl.scene, Q).mean() == chosen["share"]
    out = {"workload": wl.name, "recipe": "paper_2406_04795_amd.inputs.config_c3(eps=2e-5, k=4)",
           "obstacle_ball": I.C3_OBST_BALL, "stream": I.C3_SCENE_STREAM, "sample_points": int(len(Q)),
           "share": chosen["share"], "scan": scan}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_scene.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print({k: out[k] for k in ("stream", "share", "sample_points")})


if __name__ == "__main__":
    main()
