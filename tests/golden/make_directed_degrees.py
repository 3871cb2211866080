"""Writes directed_degrees.json: closed forms worked by hand for a 4-node directed,
weighted graph under the Laplacian of Table 1 with the two degree readings.

The paper's options paragraph (Section 2) and Table 1's Laplacian row write
D^-1/2 A D^-1/2 with "D the degree matrix" and name no side for a directed graph. The
fixture pins both readings: row sums on both sides (the default) and out-degrees (row
sums) on the left with in-degrees (column sums) on the right. The expressions were derived
on paper; this script only evaluates them. It calls neither the oracle nor the GPU path.
Run: python tests/golden/make_directed_degrees.py
"""
import json
import math
import os

r2, r3, r6 = math.sqrt(2), math.sqrt(3), math.sqrt(6)

fx = {
    "citation": "Section 2 options paragraph and Table 1 (Laplacian row: A replaced by D^-1/2 A D^-1/2, "
                "D the degree matrix); Section 2 definition of W (rows 1/n_k) and Eq. 1 (Z = A W). "
                "Worked by hand; the paper prints no values.",
    "graph": {"N": 4, "K": 2, "labels": [0, 1, 1, 0],
              "directed_rows": [[0, 1, 1.0], [0, 2, 2.0], [1, 2, 1.0], [2, 0, 1.0], [3, 0, 2.0]]},
    "derivation": {
        "A": "A[0,1] = 1, A[0,2] = 2, A[1,2] = 1, A[2,0] = 1, A[3,0] = 2; n_0 = 2 (nodes 0, 3), n_1 = 2",
        "lap_rowsum": "row sums d = (3, 1, 1, 2) on both sides: v_ij = A_ij / sqrt(d_i d_j); "
                      "Z[0] = (0, (1/sqrt3 + 2/sqrt3)/2), Z[1] = (0, 1/2), Z[2] = (1/(2 sqrt3), 0), "
                      "Z[3] = (2/sqrt6/2, 0)",
        "lap_inout": "out-degrees (3, 1, 1, 2), in-degrees (3, 1, 3, 0): v_ij = A_ij / sqrt(dout_i din_j); "
                     "v01 = 1/sqrt3, v02 = 2/3, v12 = 1/sqrt3, v20 = 1/sqrt3, v30 = 2/sqrt6; "
                     "Z[0] = (0, 1/(2 sqrt3) + 1/3), Z[1] = (0, 1/(2 sqrt3)), Z[2] = (1/(2 sqrt3), 0), "
                     "Z[3] = (1/sqrt6, 0)",
        "diag_lap_inout": "A + I: out-degrees (4, 2, 2, 3), in-degrees (4, 2, 4, 1); v00 = 1/4, "
                          "v01 = 1/(2 sqrt2), v02 = 1/2, v11 = 1/2, v12 = 1/(2 sqrt2), v20 = 1/(2 sqrt2), "
                          "v22 = 1/(2 sqrt2), v30 = 1/sqrt3, v33 = 1/sqrt3; Z[0] = (1/8, (1/(2 sqrt2) + 1/2)/2), "
                          "Z[1] = (0, (1/2 + 1/(2 sqrt2))/2), Z[2] = (1/(4 sqrt2), 1/(4 sqrt2)), "
                          "Z[3] = (1/sqrt3, 0)",
        "degrees": "in-degrees without augmentation (3, 1, 3, 0); with it (4, 2, 4, 1)",
    },
    "expect": {
        "lap_rowsum": [[0, r3 / 2], [0, 0.5], [1 / (2 * r3), 0], [1 / r6, 0]],
        "lap_inout": [[0, 1 / (2 * r3) + 1 / 3], [0, 1 / (2 * r3)], [1 / (2 * r3), 0], [1 / r6, 0]],
        "diag_lap_inout": [[1 / 8, (1 / (2 * r2) + 0.5) / 2], [0, (0.5 + 1 / (2 * r2)) / 2],
                           [1 / (4 * r2), 1 / (4 * r2)], [1 / r3, 0]],
        "in_degrees": [3, 1, 3, 0],
        "in_degrees_diag": [4, 2, 4, 1],
    },
}

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "directed_degrees.json")
    with open(out, "w") as f:
        json.dump(fx, f, indent=1)
