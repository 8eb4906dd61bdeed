"""Write the FP64 oracle's whole solve of a workload too large for a test.

Calls only the FP64 oracle (``oracle.closed_shell.triple_energy``, one call
per unique occupied triple, exactly as ``oracle.t_energy`` makes them) and
the seeded input generator.  The triples are spread over worker processes
(each with one BLAS thread); the per-triple energies are collected in
unique-triple order and summed with math.fsum, as ``oracle.t_energy`` does.

Workloads: large_fragment, nocc = 32, nvir = 300, naux = 1000, seed 0
(5952 unique triples, 6.4e14 flops; about two hours on eight host cores),
and precision_sweep, nocc = 24, nvir = 240, naux = 800, seed 0 (2576
triples, 1.1e14 flops).  Output: tests/golden/<workload>_seed0.json with
E_T, every per-triple energy and a summary of the generated inputs
(synth.input_summary).
Run from the repository root:

    python tests/golden/make_golden_large.py [--workload NAME] [--workers N]

With --summary-only, an existing file keeps its oracle values and gets the
input summary of freshly generated inputs (the summary replaced an exact
hash of the inputs, which differs between machines in the last bits of the
BLAS products).
"""
import argparse
import json
import math
import os
import sys
import time

# one BLAS thread per worker process (set before numpy loads its BLAS)
for _k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_k] = "1"

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import multiprocessing as mp  # noqa: E402

from oracle.closed_shell import triple_energy, triple_table  # noqa: E402
from synth import input_summary, make_inputs  # noqa: E402

SHAPES = {"large_fragment": (32, 300, 1000, 0), "precision_sweep": (24, 240, 800, 0)}
HERE = os.path.dirname(os.path.abspath(__file__))

_X = None  # inputs, inherited by the forked workers


def _one(args):
    idx, (i, j, k, m) = args
    return idx, triple_energy(i, j, k, m, *_X.arrays())


def main():
    global _X
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    ap.add_argument("--workload", default="large_fragment", choices=sorted(SHAPES))
    ap.add_argument("--summary-only", action="store_true")
    a = ap.parse_args()
    o, v, naux, seed = SHAPES[a.workload]
    out_path = os.path.join(HERE, f"{a.workload}_seed{seed}.json")
    t0 = time.time()
    _X = make_inputs(o, v, naux, seed)
    if a.summary_only:
        rec = json.load(open(out_path))
        rec.pop("input_fingerprint", None)
        rec = {**{k: rec[k] for k in ("nocc", "nvir", "naux", "seed", "generator", "oracle")},
               "input_summary": input_summary(_X), "E_T": rec["E_T"], "triples": rec["triples"]}
        with open(out_path, "w") as f:
            json.dump(rec, f)
            f.write("\n")
        print(f"summary of {out_path} rewritten", flush=True)
        return
    table = triple_table(o)
    print(f"inputs in {time.time() - t0:.0f} s; {len(table)} triples on {a.workers} workers", flush=True)
    terms = [None] * len(table)
    ctx = mp.get_context("fork")
    done = 0
    with ctx.Pool(a.workers) as pool:
        for idx, e in pool.imap_unordered(_one, list(enumerate(table)), chunksize=1):
            terms[idx] = e
            done += 1
            if done % 100 == 0 or done == len(table):
                el = time.time() - t0
                print(f"{done}/{len(table)} triples at {el:.0f} s "
                      f"(eta {el / done * (len(table) - done):.0f} s)", flush=True)
    e_t = math.fsum(terms)
    rec = {"nocc": o, "nvir": v, "naux": naux, "seed": seed, "generator": "synth.make_inputs",
           "oracle": "oracle.closed_shell.triple_energy per unique triple, math.fsum over triples",
           "input_summary": input_summary(_X), "E_T": e_t, "triples": terms}
    with open(out_path, "w") as f:
        json.dump(rec, f)
        f.write("\n")
    print(f"E_T = {e_t!r}; wrote {out_path} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
