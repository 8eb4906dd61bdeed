"""bqc_t_energy_noalloc (workspace in the library's fixed device array, no
device allocation) against bqc_t_energy_ex, through the C ABI.

Bar: bitwise equality of E_T and of every per-triple energy (same kernels,
same summation order; only the triples per launch may differ), plus the
FP64 result against the oracle's stored values at 1e-10 relative.  Two calls
in a row share the array, the second with a smaller input; the device's free
memory does not change across the calls.
"""
import json
import os

import numpy as np
import pytest

from synth import make_inputs

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


def _oracle(o, v, naux, seed):
    for c in GOLDEN["cases"]:
        if (c["nocc"], c["nvir"], c["naux"], c["seed"]) == (o, v, naux, seed):
            return c
    raise KeyError((o, v, naux, seed))


def _dev(x):
    import torch
    return [torch.from_numpy(a).to("cuda:0") for a in x.arrays()]


@pytest.mark.parametrize("prec,form", [("fp64", "occupied"), ("fp32", "occupied"), ("bf16x3", "occupied"),
                                       ("fp8", "occupied"), ("fp64", "virtual"), ("bf16x3", "virtual")])
def test_noalloc_equals_ex_two_calls(prec, form):
    import torch

    import paper_2502_17963_amd as bqc
    bqc.lib()
    print(f"case noalloc {prec} {form}", flush=True)
    shapes = [(6, 30, 120, 0), (5, 37, 100, 3)] if form == "occupied" else [(6, 30, 120, 0), (4, 17, 40, 1)]
    # the second input is smaller (fewer unique triples of the loop)
    nt = [bqc.num_triples(s[1] if form == "virtual" else s[0]) for s in shapes]
    assert nt[1] < nt[0]
    first = True
    for (o, v, naux, seed) in shapes:
        assert bqc.noalloc_batch(o, v, prec, form) >= 1
        dev = _dev(make_inputs(o, v, naux, seed))
        torch.cuda.synchronize()
        e_ref, ex_ref = bqc.t_energy(o, v, *dev, precision=prec, formulation=form, triple_energies=True)
        if first:
            bqc.t_energy_noalloc(o, v, *dev, precision=prec, formulation=form)  # first use of the array
            first = False
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        e, ex = bqc.t_energy_noalloc(o, v, *dev, precision=prec, formulation=form, triple_energies=True,
                                     stats=True)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0  # the call allocated no device memory
        assert e == e_ref, (o, v, e, e_ref)
        assert np.array_equal(ex["triples"], ex_ref["triples"])
        st = ex["stats"]
        assert st["n_triples"] == len(ex_ref["triples"]) and 0 < st["footprint_bytes"] <= 64 << 20
        if prec == "fp64" and form == "occupied" and (o, v, naux, seed) == (6, 30, 120, 0):
            ref = _oracle(o, v, naux, seed)["E_T"]
            assert abs(e - ref) <= 1e-10 * abs(ref)


def test_noalloc_share_and_fock():
    import torch

    import paper_2502_17963_amd as bqc
    bqc.lib()
    print("case noalloc share + f_ov", flush=True)
    o, v = 6, 30
    dev = _dev(make_inputs(o, v, 120, 2))
    f = torch.from_numpy(np.random.default_rng(7).normal(0.0, 0.02, (o, v))).to("cuda:0")
    torch.cuda.synchronize()
    for rng in [(3, 41), (0, 50), (49, 50)]:
        a = bqc.t_energy(o, v, *dev, precision="bf16x3", triple_range=rng, fock_ov=f)
        b = bqc.t_energy_noalloc(o, v, *dev, precision="bf16x3", triple_range=rng, fock_ov=f)
        assert a == b, (rng, a, b)


def test_noalloc_rejects_what_does_not_fit_and_host_inputs():
    import paper_2502_17963_amd as bqc
    from paper_2502_17963_amd.binding import BqcError
    bqc.lib()
    x = make_inputs(2, 5, 10, 0)
    with pytest.raises(ValueError):
        bqc.t_energy_noalloc(2, 5, *x.arrays())
    import torch
    big = [torch.zeros(n, dtype=torch.float64, device="cuda:0") for n in (32, 300, 32 * 300, 1, 1, 1, 1)]
    big[1] += 1.0
    big[0] -= 1.0
    with pytest.raises(BqcError) as ei:
        bqc.t_energy_noalloc(32, 300, *big, precision="bf16x3")
    assert ei.value.code == -2
