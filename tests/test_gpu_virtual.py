"""Parity of the virtual-triple formulation (loop over a <= b <= c with
tensors over the occupied indices) with the FP64 oracles, through the C ABI.

The energy is the one of the occupied-triple loop, so the stored oracle
values of tests/golden apply; per-virtual-triple energies are compared with
oracle/virtual_loop.py computed here.  Gates as in test_gpu_parity.py:
FP64 <= 1e-10 relative; FP32 and split-BF16x3 <= 1 uEh at the small
workload and <= 1e-6 relative elsewhere.
"""
import json
import os

import numpy as np
import pytest

import oracle.closed_shell as cs
import oracle.virtual_loop as vl
from synth import make_df_inputs, make_inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))
FP64_REL = 1e-10


def _bqc():
    import paper_2502_17963_amd as bqc
    bqc.lib()
    return bqc


def _golden(o, v, naux, seed):
    for c in GOLDEN["cases"]:
        if (c["nocc"], c["nvir"], c["naux"], c["seed"]) == (o, v, naux, seed):
            return c["E_T"]
    raise KeyError((o, v, naux, seed))


@pytest.mark.parametrize("seed", range(5))
def test_small_fp64(seed):
    bqc = _bqc()
    print(f"case virtual small seed={seed}", flush=True)
    x = make_inputs(6, 30, 120, seed)
    ref = _golden(6, 30, 120, seed)
    e = bqc.t_energy(6, 30, *x.arrays(), formulation="virtual")
    assert abs(e - ref) <= FP64_REL * abs(ref), (e, ref)


def test_per_virtual_triple_energies():
    bqc = _bqc()
    print("case virtual per-triple (6, 30)", flush=True)
    x = make_inputs(6, 30, 120, 0)
    e_ref, terms = vl.t_energy_virtual_loop(*x.arrays(), return_triples=True)
    e, ex = bqc.t_energy(6, 30, *x.arrays(), formulation="virtual", triple_energies=True)
    got = ex["triples"]
    ref = np.array(terms)
    assert got.shape == ref.shape == (bqc.num_triples(30),)
    assert np.max(np.abs(got - ref)) <= FP64_REL * np.max(np.abs(ref))
    assert abs(e - e_ref) <= FP64_REL * abs(e_ref)


# occupied spaces of one 16-block, of two (ragged), and of three (two tiles
# of the 2 x 2 wave grid); tiny and degenerate spaces
RAGGED = [(2, 17, 40, 5), (5, 37, 100, 3), (9, 20, 60, 8), (4, 64, 160, 1), (1, 9, 20, 6), (3, 1, 12, 4),
          (17, 11, 50, 2), (20, 13, 60, 7), (33, 9, 60, 3), (40, 6, 50, 9)]


@pytest.mark.parametrize("o,v,naux,seed", RAGGED)
def test_ragged_fp64(o, v, naux, seed):
    bqc = _bqc()
    print(f"case virtual ragged o={o} v={v} seed={seed}", flush=True)
    x = make_inputs(o, v, naux, seed)
    ref = cs.t_energy(*x.arrays())
    e = bqc.t_energy(o, v, *x.arrays(), formulation="virtual")
    if o == 1 or v == 1:
        # every element of every remaining term is one where the numerator
        # operator cancels V exactly (up to rounding)
        scale = np.max(np.abs(x.ovvv)) ** 2 * np.max(np.abs(x.t2)) ** 2 * max(o, v) ** 3
        assert abs(e) <= 1e-12 * scale and abs(ref) <= 1e-12 * scale
    else:
        assert abs(e - ref) <= FP64_REL * abs(ref), (e, ref)


def test_equals_occupied_formulation_on_device_inputs():
    import torch
    bqc = _bqc()
    o, v, naux, seed = 7, 45, 150, 2
    print(f"case virtual vs occupied o={o} v={v}", flush=True)
    x = make_inputs(o, v, naux, seed)
    dev = [torch.from_numpy(a).to("cuda:0") for a in x.arrays()]
    e_occ = bqc.t_energy(o, v, *dev)
    e_vir = bqc.t_energy(o, v, *dev, formulation="virtual")
    e_host = bqc.t_energy(o, v, *x.arrays(), formulation="virtual")
    torch.cuda.synchronize()
    assert e_vir == e_host
    assert abs(e_vir - e_occ) <= 1e-12 * abs(e_occ)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision(prec):
    bqc = _bqc()
    for (o, v, naux, seed) in [(6, 30, 120, 0), (5, 37, 100, 3), (20, 13, 60, 7), (33, 9, 60, 3)]:
        x = make_inputs(o, v, naux, seed)
        ref = _golden(o, v, naux, seed) if (o, v) in [(6, 30), (5, 37)] else cs.t_energy(*x.arrays())
        e = bqc.t_energy(o, v, *x.arrays(), precision=prec, formulation="virtual")
        print(f"virtual {prec} o={o} v={v} dE={abs(e - ref) * 1e6:.3e} uEh rel={abs(e - ref) / abs(ref):.3e}",
              flush=True)
        if (o, v) == (6, 30):
            assert abs(e - ref) <= 1e-6
        else:
            assert abs(e - ref) <= 1e-6 * abs(ref), (o, v, e, ref)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_fock_term(prec):
    bqc = _bqc()
    o, v, naux, seed = 5, 37, 100, 3
    print(f"case virtual fock {prec}", flush=True)
    x = make_inputs(o, v, naux, seed)
    f = np.random.default_rng(1000 + seed).normal(0.0, 0.02, (o, v))
    ref = vl.t_energy_virtual_loop(*x.arrays(), fock_ov=f)
    e = bqc.t_energy(o, v, *x.arrays(), precision=prec, fock_ov=f, formulation="virtual")
    tol = FP64_REL if prec == "fp64" else 1e-6
    assert abs(e - ref) <= tol * abs(ref), (e, ref)
    assert abs(ref - cs.t_energy(*x.arrays())) > 1e-3 * abs(ref)  # the term matters here


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_density_fitted(prec):
    bqc = _bqc()
    o, v, naux, seed = 6, 30, 120, 1
    print(f"case virtual DF {prec}", flush=True)
    eps_o, eps_v, t1, t2, b_ov, b_vv, ooov, ovov = make_df_inputs(o, v, naux, seed)
    ref = _golden(o, v, naux, seed)
    e = bqc.t_energy_df(o, v, naux, eps_o, eps_v, t1, t2, b_ov, b_vv, ooov, ovov, precision=prec,
                        formulation="virtual")
    tol = 1e-10 * abs(ref) if prec == "fp64" else 1e-6
    assert abs(e - ref) <= tol, (e, ref)


def test_triple_shares_add_up_to_the_solve():
    import torch
    bqc = _bqc()
    o, v, naux, seed = 6, 30, 120, 0
    print("case virtual triple shares", flush=True)
    x = make_inputs(o, v, naux, seed)
    dev = [torch.from_numpy(a).to("cuda:0") for a in x.arrays()]
    e_all, ex = bqc.t_energy(o, v, *dev, triple_energies=True, formulation="virtual")
    n = bqc.num_triples(v)
    parts = []
    for b, e in [(0, 1), (1, n // 3), (n // 3, n - 1), (n - 1, n)]:
        es, exs = bqc.t_energy(o, v, *dev, triple_energies=True, triple_range=(b, e), formulation="virtual")
        assert np.array_equal(exs["triples"][b:e], ex["triples"][b:e])
        assert np.all(exs["triples"][:b] == 0) and np.all(exs["triples"][e:] == 0)
        parts.append(es)
    torch.cuda.synchronize()
    assert abs(sum(parts) - e_all) <= 1e-13 * abs(e_all)


@pytest.mark.parametrize("o,v,naux,seed", [(70, 5, 30, 1), (66, 4, 30, 2)])
def test_many_occupied_fp64(o, v, naux, seed):
    """More than 64 occupied orbitals: the contraction runs on the general
    tile kernel instead of one plane per wave."""
    bqc = _bqc()
    print(f"case virtual many-occupied o={o} v={v} seed={seed}", flush=True)
    x = make_inputs(o, v, naux, seed)
    ref = vl.t_energy_virtual_loop(*x.arrays())
    for prec, tol in (("fp64", FP64_REL), ("bf16x3", 1e-6)):
        e = bqc.t_energy(o, v, *x.arrays(), precision=prec, formulation="virtual")
        assert abs(e - ref) <= tol * abs(ref), (prec, e, ref)


@pytest.mark.parametrize("form,fock", [("occupied", False), ("occupied", True), ("virtual", False), ("virtual", True)])
def test_footprint_bounds_the_solve(form, fock):
    """bqc_t_footprint_ex is an upper bound of what a host-input solve holds
    (its stats), within 1 %."""
    bqc = _bqc()
    o, v, naux, seed = 7, 45, 150, 2
    x = make_inputs(o, v, naux, seed)
    f = np.random.default_rng(5).normal(0.0, 0.02, (o, v)) if fock else None
    _, ex = bqc.t_energy(o, v, *x.arrays(), precision="bf16x3", stats=True, fock_ov=f, formulation=form)
    held = ex["stats"]["footprint_bytes"]
    bound = bqc.footprint(o, v, "bf16x3", formulation=form, fock=fock)
    print(f"footprint {form} fock={fock}: solve {held} bound {bound}", flush=True)
    assert held <= bound <= 1.01 * held


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_all_options_together(prec):
    """Loop over virtual triples with density fitting, an f_ov block, device
    inputs and a triple share at once: per-triple energies of the share
    against the oracle's."""
    import torch
    bqc = _bqc()
    o, v, naux, seed = 5, 23, 80, 6
    print(f"case virtual all options {prec}", flush=True)
    x = make_inputs(o, v, naux, seed)
    f = np.random.default_rng(1000 + seed).normal(0.0, 0.02, (o, v))
    e_ref, terms = vl.t_energy_virtual_loop(*x.arrays(), return_triples=True, fock_ov=f)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
           for a in make_df_inputs(o, v, naux, seed)]
    f_dev = torch.from_numpy(f).to("cuda:0")
    n = bqc.num_triples(v)
    b, e = n // 4, 3 * n // 4
    es, ex = bqc.t_energy_df(o, v, naux, *dev, precision=prec, triple_energies=True, triple_range=(b, e),
                             fock_ov=f_dev, formulation="virtual")
    torch.cuda.synchronize()
    got, ref = ex["triples"][b:e], np.array(terms[b:e])
    tol_triple, tol_sum = (1e-10, 1e-10) if prec == "fp64" else (1e-5, 1e-6)
    assert np.max(np.abs(got - ref)) <= tol_triple * np.max(np.abs(ref))
    assert abs(es - float(np.sum(ref))) <= tol_sum * abs(float(np.sum(ref)))
