"""Writes oracle_small.json: the oracle's output on a tiny seeded case, kept
as a regression fixture. Every stored value comes from `oracle/` (and the
seeded input generators); nothing comes from the GPU path. Rerun only when
the oracle's arithmetic changes on purpose, and name the passage of the paper
(or the reading of it) that justifies the change in the commit that updates
the fixture.

    python tests/golden/make_oracle_fixture.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc                                   # noqa: E402
from paper_2309_03717_amd import workloads as W        # noqa: E402

N_TRACKS = 12


def case():
    """The first 12 tracks of the 160-antenna star workload on 4 of its
    antennas (two heights), 4096 bins of 0.1 ns, in the uniform and the
    exponential medium."""
    w = W.config(1)
    tr = w.tracks(N_TRACKS)
    idx = np.array([0, 19, 87, 150])
    arr = W.AntennaArray(w.array.x[idx], w.array.y[idx], w.array.z[idx] + np.array([0, 0, 40.0, 0]),
                         w.array.t_start[idx], w.array.dt, w.array.n_bins)
    media = {"uniform": W.Medium("uniform", 2.92e-4, 8000.0), "exponential": w.medium}
    return tr, arr, media


def compute():
    tr, arr, media = case()
    out = {}
    for name, md in media.items():
        t, u, b = orc.propagate(tr, arr, md)
        entry = {"bins": b.tolist(), "t": [float(x) for x in t.ravel()]}
        for f in ("endpoint", "zhs"):
            tr_ = orc.traces(f, tr, arr, md)
            nz = np.nonzero(tr_)
            entry[f] = {"index": [list(map(int, v)) for v in nz],
                        "value": [float(x) for x in tr_[nz]]}
        out[name] = entry
    return out


if __name__ == "__main__":
    data = {"what": "oracle output, first 12 tracks of the star workload, 4 antennas, "
                    "uniform and exponential media; bins, arrival times and nonzero trace values",
            "n_tracks": N_TRACKS, "cases": compute()}
    with open(os.path.join(HERE, "oracle_small.json"), "w") as fh:
        json.dump(data, fh, separators=(",", ":"))
        fh.write("\n")
    print("wrote", os.path.join(HERE, "oracle_small.json"))
