"""Write the stored oracle values used by the parity tests.

Calls only the FP64 oracle and the seeded input generator.  Run from the
repository root:  python tests/golden/make_golden.py
The paper prints no numerical (T) example, so every stored value here is
the oracle's, for the seeded inputs named beside it.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import spinorb_t_energy, t_energy  # noqa: E402
from synth import make_inputs  # noqa: E402

CASES = [
    # (nocc, nvir, naux, seed): the small workload over ten seeds
    *[(6, 30, 120, s) for s in range(10)],
    # ragged shapes: virtual counts that are not multiples of any tile size
    (2, 17, 40, 5), (5, 37, 100, 3), (7, 45, 150, 2), (3, 1, 12, 4), (1, 9, 20, 6),
    (9, 20, 60, 8), (4, 64, 160, 1),
]
TINY = [(2, 3, 8, 7), (3, 4, 10, 1), (3, 5, 12, 11), (4, 6, 16, 8)]


def main():
    out = {"generator": "synth.make_inputs", "cases": [], "spin_orbital": []}
    for (o, v, naux, seed) in CASES:
        x = make_inputs(o, v, naux, seed)
        e, terms = t_energy(*x.arrays(), return_triples=True)
        rec = {"nocc": o, "nvir": v, "naux": naux, "seed": seed, "E_T": e}
        if (o, v, naux, seed) == (6, 30, 120, 0):
            rec["triples"] = terms
        out["cases"].append(rec)
    for (o, v, naux, seed) in TINY:
        x = make_inputs(o, v, naux, seed)
        out["spin_orbital"].append({"nocc": o, "nvir": v, "naux": naux, "seed": seed,
                                    "E_T": spinorb_t_energy(*x.arrays())})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
