"""Non-canonical reference: the f_ov term of the disconnected triples
(paper Eqs. 5 and 7) on the GPU against the oracle (which is pinned to the
spin-orbital definition with f_IA t_JK^BC)."""
import numpy as np
import pytest

from oracle.closed_shell import t_energy as oracle_t_energy
from synth import make_df_inputs, make_inputs

pytestmark = pytest.mark.gpu


def _bqc():
    import paper_2502_17963_amd as bqc
    bqc.lib()
    return bqc


def _fock(o, v, seed):
    return np.random.default_rng(2000 + seed).normal(0.0, 0.02, (o, v))


@pytest.mark.parametrize("shape", [(6, 30, 120, 0), (6, 30, 120, 1), (2, 17, 40, 5), (5, 37, 100, 3),
                                   (4, 64, 160, 1)])
def test_fock_fp64_matches_oracle(shape):
    bqc = _bqc()
    o, v, naux, seed = shape
    print(f"case fock fp64 o={o} v={v} seed={seed}", flush=True)
    x = make_inputs(o, v, naux, seed)
    f = _fock(o, v, seed)
    ref, ref_trip = oracle_t_energy(*x.arrays(), return_triples=True, fock_ov=f)
    e, ex = bqc.t_energy(o, v, *x.arrays(), precision="fp64", triple_energies=True, fock_ov=f)
    assert abs(e - ref) <= 1e-10 * abs(ref), (e, ref)
    trip = np.array(ref_trip)
    assert np.max(np.abs(ex["triples"] - trip)) <= 1e-10 * np.max(np.abs(trip))
    e0 = bqc.t_energy(o, v, *x.arrays(), precision="fp64")
    assert abs(e - e0) > 1e-6 * abs(e0)  # the term changes the energy


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fock_mixed_matches_oracle(prec):
    bqc = _bqc()
    x = make_inputs(6, 30, 120, 0)
    f = _fock(6, 30, 0)
    ref = oracle_t_energy(*x.arrays(), fock_ov=f)
    e = bqc.t_energy(6, 30, *x.arrays(), precision=prec, fock_ov=f)
    print(f"{prec}: dE = {abs(e - ref) * 1e6:.3e} uEh", flush=True)
    assert abs(e - ref) <= 1e-6  # 1 uEh at the small workload


def test_zero_fock_equals_canonical_bitwise():
    bqc = _bqc()
    x = make_inputs(5, 37, 100, 3)
    e0 = bqc.t_energy(5, 37, *x.arrays(), precision="bf16x3")
    e1 = bqc.t_energy(5, 37, *x.arrays(), precision="bf16x3", fock_ov=np.zeros((5, 37)))
    assert e0 == e1


def test_fock_with_density_fitting_and_device_inputs():
    import torch
    bqc = _bqc()
    o, v, naux, seed = 7, 45, 150, 2
    x = make_inputs(o, v, naux, seed)
    a = make_df_inputs(o, v, naux, seed)
    f = _fock(o, v, seed)
    ref = oracle_t_energy(*x.arrays(), fock_ov=f)
    dev = [torch.from_numpy(np.ascontiguousarray(t)).to("cuda:0") for t in a]
    fd = torch.from_numpy(f).to("cuda:0")
    e = bqc.t_energy_df(o, v, naux, *dev, precision="fp64", fock_ov=fd)
    torch.cuda.synchronize()
    assert abs(e - ref) <= 1e-10 * abs(ref), (e, ref)
