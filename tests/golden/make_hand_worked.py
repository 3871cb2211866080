"""Writes hand_worked_small.json: closed forms worked by hand for a 5-node graph.

The expressions below were derived on paper from Section 2 (W rows 1/n_k, Eq. 1 and
the Z_i^k sum over class-k neighbours) and Table 1 (A + I, D^-1/2 A D^-1/2, row
2-norm); this script only evaluates them. It calls neither the oracle nor the GPU path.
Run: python tests/golden/make_hand_worked.py
"""
import json
import math
import os

r2, r3, r6, r19 = math.sqrt(2), math.sqrt(3), math.sqrt(6), math.sqrt(19)


def nrm(r):
    n = math.sqrt(sum(x * x for x in r))
    return [x / n if n > 0 else 0 for x in r]


off = [[1 / 2, 1 / 2], [1 / 2, 1 / 2], [1, 1 / 2], [0, 1 / 2], [0, 1 / 2]]
diag = [[1, 1 / 2], [1, 1 / 2], [1, 1], [0, 1], [0, 1 / 2]]
lap = [[1 / 4, 1 / (2 * r6)], [1 / 4, 1 / (2 * r6)], [1 / r6, 1 / (2 * r6)], [0, 1 / (2 * r6)],
       [0, 1 / (2 * r2)]]
cor = [nrm(r) for r in off]
allon = [[4 / r19, r3 / r19], [4 / r19, r3 / r19], nrm([1 / (2 * r3), (1 / r3 + 1 / 2) / 4]), [0, 1], [0, 1]]

fx = {
    "citation": "Worked by hand from Section 2 (W rows 1/n_k, Z = A W of Eq. 1, the Z_i^k sum over "
                "class-k neighbours) and the option formulas of Table 1 (A + I, D^-1/2 A D^-1/2, row "
                "2-norm). The paper prints no embedding values; these are closed forms derived by hand "
                "and evaluated by tests/golden/make_hand_worked.py.",
    "graph": {"N": 5, "K": 2, "labels": [0, 0, 1, 1, -1],
              "undirected_edges": [[0, 1], [0, 2], [1, 2], [2, 3], [3, 4]]},
    "derivation": {
        "class_sizes": "n_0 = 2 (nodes 0,1), n_1 = 2 (nodes 2,3); node 4 is unknown and counts in no class",
        "off": "Z[i,k] = (#class-k neighbours of i)/2",
        "diag": "off plus 1/n_{y_i} at column y_i for labelled i",
        "lap": "degrees (2,2,3,2,1); Z[i,k] = sum_j d_i^-1/2 d_j^-1/2 / n_k over class-k neighbours",
        "cor": "off with every row divided by its 2-norm",
        "all": "degrees of A+I are (3,3,4,3,2); Z[i,k] = d_i^-1/2 sum over j in N(i) + {i} with y_j = k "
               "of d_j^-1/2 / n_k, then each row divided by its 2-norm; row 0 = (1/3, 1/(4 sqrt 3)) -> "
               "(4, sqrt 3)/sqrt 19; row 2 = (1/(2 sqrt 3), (1/sqrt 3 + 1/2)/4) normalised",
    },
    "expect": {"off": off, "diag": diag, "lap": lap, "cor": cor, "all": allon},
    "directed": {
        "graph": {"N": 3, "K": 2, "labels": [0, 1, 1], "directed_rows": [[0, 1], [1, 2]]},
        "derivation": "Without symmetrization each row is the single entry A[s,d]. n_1 = 2. Options off: "
                      "Z[0] = (0, 1/2), Z[1] = (0, 1/2), Z[2] = 0. Laplacian with row-sum degrees (1, 1, 0) "
                      "and d^-1/2 = 0 for degree 0: Z[0] = (0, 1*1/2), Z[1] = (0, 1*0/2) = 0, Z[2] = 0.",
        "expect": {"off": [[0, 0.5], [0, 0.5], [0, 0]], "lap": [[0, 0.5], [0, 0], [0, 0]]},
    },
}

if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hand_worked_small.json")
    with open(out, "w") as f:
        json.dump(fx, f, indent=1)
