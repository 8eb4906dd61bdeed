"""Parity at the benchmarked sizes (nocc=32, nvir=300, naux=1000, seed 0, and
the precision-sweep workload nocc=24, nvir=240, naux=800, seed 0).

The oracle's whole solve of each workload is stored
(tests/golden/<workload>_seed0.json, written by
tests/golden/make_golden_large.py, which calls only the oracle and the
generator): the GPU's FP64 per-triple energies are compared with it triple
by triple and in total, and the mixed-precision totals with its total, in
the launch configuration the benchmark times.  A seeded sample of triples
is also recomputed by the oracle at test time.
"""
import json
import os

import numpy as np
import pytest

from oracle.closed_shell import triple_energy, triple_table
from synth import CONFIGS, make_inputs, summary_matches

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "large_fragment_seed0.json")


def _golden(x):
    if not os.path.exists(GOLDEN):
        pytest.skip("the oracle's whole solve of the large fragment has not been stored")
    rec = json.load(open(GOLDEN))
    assert summary_matches(rec["input_summary"], x), "the generator no longer makes the stored inputs"
    return rec


@pytest.fixture(scope="module")
def large():
    import torch

    import paper_2502_17963_amd as bqc
    bqc.lib()
    o, v, naux, seed = CONFIGS["large_fragment"]
    print(f"case large_fragment o={o} v={v} naux={naux} seed={seed}", flush=True)
    x = make_inputs(o, v, naux, seed)
    dev = [torch.from_numpy(a).to("cuda:0") for a in x.arrays()]
    torch.cuda.synchronize()
    e64, ex = bqc.t_energy(o, v, *dev, precision="fp64", triple_energies=True)
    torch.cuda.synchronize()
    return bqc, x, dev, e64, ex["triples"]


def test_fp64_sampled_triples_match_oracle(large):
    bqc, x, dev, e64, trip = large
    table = triple_table(x.nocc)
    assert len(trip) == len(table)
    rng = np.random.default_rng(2025)
    picks = sorted(set([0, 1, len(table) - 1] + list(rng.choice(len(table), 3, replace=False))))
    for n in picks:
        i, j, k, m = table[n]
        ref = triple_energy(i, j, k, m, *x.arrays())
        print(f"triple {n} ({i},{j},{k}) gpu={trip[n]:.15e} oracle={ref:.15e}", flush=True)
        assert abs(trip[n] - ref) <= 1e-10 * abs(ref)
    assert abs(float(np.sum(trip)) - e64) <= 1e-12 * abs(e64)


def test_fp64_every_triple_matches_stored_oracle(large):
    """Every one of the 5952 per-triple energies at 1e-10 relative (of the
    largest), and E_T at 1e-10 relative, against the oracle's whole solve."""
    bqc, x, dev, e64, trip = large
    rec = _golden(x)
    ref = np.array(rec["triples"])
    assert ref.shape == trip.shape
    worst = np.max(np.abs(trip - ref)) / np.max(np.abs(ref))
    rel = abs(e64 - rec["E_T"]) / abs(rec["E_T"])
    print(f"stored oracle E_T={rec['E_T']:.15e} gpu={e64:.15e} rel={rel:.3e} worst triple {worst:.3e}", flush=True)
    assert worst <= 1e-10
    assert rel <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_totals_against_stored_oracle(large, prec):
    import torch
    bqc, x, dev, e64, _ = large
    rec = _golden(x)
    e = bqc.t_energy(x.nocc, x.nvir, *dev, precision=prec)
    torch.cuda.synchronize()
    rel = abs(e - rec["E_T"]) / abs(rec["E_T"])
    print(f"{prec}: E={e:.12e} oracle={rec['E_T']:.12e} rel={rel:.3e} dE={abs(e - rec['E_T']) * 1e6:.3e} uEh",
          flush=True)
    assert rel <= 1e-6


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_totals_against_fp64(large, prec):
    import torch
    bqc, x, dev, e64, _ = large
    e = bqc.t_energy(x.nocc, x.nvir, *dev, precision=prec)
    torch.cuda.synchronize()
    rel = abs(e - e64) / abs(e64)
    print(f"{prec}: E={e:.12e} fp64={e64:.12e} rel={rel:.3e} dE={abs(e - e64) * 1e6:.3e} uEh", flush=True)
    assert rel <= 1e-6


def test_df_bf16x3_matches_ovvv_input(large):
    """Density-fitting entry at the benchmarked size: (ia|bc) formed on the
    device from B (draw of the same seed) gives the energy of the solve that
    takes (ia|bc) as an input, to the mixed-precision gate."""
    import torch

    from synth import draw_factors
    bqc, x, dev, e64, _ = large
    o, v = x.nocc, x.nvir
    b = draw_factors(o, v, 1000, 0)[0]
    b_ov = torch.from_numpy(np.ascontiguousarray(b[:, :o, o:])).to("cuda:0")
    b_vv = torch.from_numpy(np.ascontiguousarray(b[:, o:, o:])).to("cuda:0")
    del b
    eps_o, eps_v, t1, t2, _ovvv, ooov, ovov = dev
    e_df = bqc.t_energy_df(o, v, 1000, eps_o, eps_v, t1, t2, b_ov, b_vv, ooov, ovov, precision="bf16x3")
    e_in = bqc.t_energy(o, v, *dev, precision="bf16x3")
    torch.cuda.synchronize()
    print(f"df bf16x3 E={e_df:.12e} ovvv-input E={e_in:.12e} fp64 {e64:.12e}", flush=True)
    assert abs(e_df - e_in) <= 1e-7 * abs(e_in)
    assert abs(e_df - e64) <= 1e-6 * abs(e64)


def test_virtual_formulation_sampled_triples_and_total(large):
    """The loop over virtual triples at the benchmarked size: its per-virtual-
    triple energies on a seeded sample against the oracle's (loop over
    virtual triples, one at a time), its FP64 total against the occupied
    loop's, and its split-BF16x3 total against FP64 at the mixed gate."""
    import torch

    from oracle.virtual_loop import virtual_triple_energy, virtual_triple_table
    bqc, x, dev, e64, _ = large
    o, v = x.nocc, x.nvir
    e_v, ex = bqc.t_energy(o, v, *dev, precision="fp64", triple_energies=True, formulation="virtual")
    torch.cuda.synchronize()
    trip = ex["triples"]
    table = virtual_triple_table(v)
    assert len(trip) == len(table)
    rng = np.random.default_rng(7)
    picks = sorted(set([0, 1, len(table) - 1] + list(rng.choice(len(table), 4, replace=False))))
    for n in picks:
        a, b, c, m = table[n]
        ref = virtual_triple_energy(a, b, c, m, *x.arrays())
        print(f"virtual triple {n} ({a},{b},{c}) gpu={trip[n]:.15e} oracle={ref:.15e}", flush=True)
        assert abs(trip[n] - ref) <= 1e-10 * max(abs(ref), 1e-300)
    print(f"virtual fp64 E={e_v:.12e} occupied fp64 E={e64:.12e}", flush=True)
    assert abs(e_v - e64) <= 1e-12 * abs(e64)
    e_b = bqc.t_energy(o, v, *dev, precision="bf16x3", formulation="virtual")
    torch.cuda.synchronize()
    assert abs(e_b - e64) <= 1e-6 * abs(e64)


def test_precision_sweep_every_triple_matches_stored_oracle():
    """The precision-sweep workload (nocc=24, nvir=240, naux=800, seed 0)
    against the oracle's stored whole solve
    (tests/golden/precision_sweep_seed0.json): every per-triple energy and
    E_T at 1e-10 in FP64, the FP32 and split-BF16x3 totals at 1e-6."""
    import torch

    import paper_2502_17963_amd as bqc
    path = os.path.join(os.path.dirname(__file__), "golden", "precision_sweep_seed0.json")
    if not os.path.exists(path):
        pytest.skip("the oracle's whole solve of the precision-sweep workload has not been stored")
    o, v, naux, seed = CONFIGS["precision_sweep"]
    print(f"case precision_sweep o={o} v={v} naux={naux} seed={seed}", flush=True)
    x = make_inputs(o, v, naux, seed)
    rec = json.load(open(path))
    assert summary_matches(rec["input_summary"], x), "the generator no longer makes the stored inputs"
    dev = [torch.from_numpy(a).to("cuda:0") for a in x.arrays()]
    e64, ex = bqc.t_energy(o, v, *dev, precision="fp64", triple_energies=True)
    ref = np.array(rec["triples"])
    worst = np.max(np.abs(ex["triples"] - ref)) / np.max(np.abs(ref))
    rel = abs(e64 - rec["E_T"]) / abs(rec["E_T"])
    print(f"fp64 E={e64:.15e} oracle={rec['E_T']:.15e} rel={rel:.3e} worst triple {worst:.3e}", flush=True)
    assert worst <= 1e-10 and rel <= 1e-10
    for prec in ("fp32", "bf16x3"):
        e = bqc.t_energy(o, v, *dev, precision=prec)
        rel = abs(e - rec["E_T"]) / abs(rec["E_T"])
        print(f"{prec} E={e:.12e} rel={rel:.3e} dE={abs(e - rec['E_T']) * 1e6:.3e} uEh", flush=True)
        assert rel <= 1e-6
    torch.cuda.synchronize()
