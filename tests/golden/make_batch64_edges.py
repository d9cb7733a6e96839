"""Write d3q19_batch64_edges.json: the cubic edge of each of the 64 replicas
of the batched workload as drawn by flb_workloads.batch_edges (uniform over
{32, 48, 64, 80, 96}, numpy PCG64 seed 2024), with the total site count.

Run from the repository root:  python tests/golden/make_batch64_edges.py
"""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import flb_workloads as W  # noqa: E402


def main():
    wl = W.WORKLOADS["d3q19_batch64"]
    edges = W.batch_edges(wl["replicas"], wl["edges"], wl["size_seed"])
    out = dict(workload="d3q19_batch64", seeds=list(range(wl["replicas"])), edges=edges,
               sites=int(sum(e ** 3 for e in edges)),
               count_by_edge={str(e): edges.count(e) for e in wl["edges"]})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "d3q19_batch64_edges.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path, out["sites"], out["count_by_edge"])


if __name__ == "__main__":
    main()
