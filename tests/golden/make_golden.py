"""Writes tests/golden/sizes.json by calling only the oracle package.

Sizes of the paper-problem meshes: the paper's own Nx = 200 / 300 and the
20^3, 64^3, 128^3, 256^3 workloads.  nnz comes from running the oracle's
neighbour-loop count where that is quick; the stored values are then
checked in tests against the closed forms (3n-2)^3 and n(3n-2)^2.
nns (segments) is stored for the meshes the oracle assembles quickly.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402

meshes = {}
for N in (20, 64, 128, 200, 256, 300):
    m = oracle.num_rows(N, N, N)
    nnz = oracle.count_nnz(N, N, N)
    row = dict(N=[N, N, N], m=m, nnz=nnz)
    if N <= 64:  # segment count from the oracle's BCRS build (Sec. 3.1)
        row["nns"] = len(oracle.bcrsvar(oracle.assemble(N, N, N, apply_bc=False))[0])
    meshes[f"{N}^3"] = row
with open(os.path.join(HERE, "sizes.json"), "w") as f:
    json.dump(dict(source="oracle.num_rows / oracle.count_nnz (Fig 3.6 neighbour loop); "
                          "nns from oracle.bcrsvar (Sec. 3.1)",
                   meshes=meshes), f, indent=1)
print("wrote sizes.json")
