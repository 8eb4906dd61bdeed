"""Density-fitted MP2 energy on the GPU (bqc_mp2_energy_df) against the FP64
oracle (pinned to the spin-orbital MP2 definition)."""
import numpy as np
import pytest

from oracle.mp2 import mp2_energy
from synth import draw_factors

pytestmark = pytest.mark.gpu


def _bqc():
    import paper_2502_17963_amd as bqc
    bqc.lib()
    return bqc


def _factors(o, v, naux, seed):
    b, eo, ev, _ = draw_factors(o, v, naux, seed)
    return eo, ev, np.ascontiguousarray(b[:, :o, o:])


# single tile, ragged tiles, one occupied orbital, naux not a multiple of the
# 16-step, several tile pairs, the benchmarked (T) fragment's shape
SHAPES = [(6, 30, 120, 0), (6, 30, 120, 1), (1, 9, 20, 6), (5, 37, 37, 3), (7, 100, 150, 2),
          (9, 130, 301, 4), (32, 300, 1000, 0)]


@pytest.mark.parametrize("shape", SHAPES)
def test_mp2_matches_oracle(shape):
    bqc = _bqc()
    o, v, naux, seed = shape
    print(f"case mp2 o={o} v={v} naux={naux} seed={seed}", flush=True)
    eo, ev, b = _factors(o, v, naux, seed)
    ref = mp2_energy(eo, ev, b)
    e = bqc.mp2_energy_df(o, v, naux, eo, ev, b)
    assert abs(e - ref) <= 1e-12 * abs(ref), (e, ref)


def test_mp2_device_inputs_and_determinism():
    import torch
    bqc = _bqc()
    eo, ev, b = _factors(8, 77, 200, 9)
    ref = mp2_energy(eo, ev, b)
    dev = [torch.from_numpy(a).to("cuda:0") for a in (eo, ev, b)]
    e1 = bqc.mp2_energy_df(8, 77, 200, *dev)
    e2 = bqc.mp2_energy_df(8, 77, 200, *dev)
    torch.cuda.synchronize()
    assert e1 == e2
    assert abs(e1 - ref) <= 1e-12 * abs(ref)


def test_mp2_no_gap_rejected():
    bqc = _bqc()
    eo, ev, b = _factors(3, 7, 20, 1)
    eo = eo.copy()
    eo[-1] = ev[0]
    with pytest.raises(bqc.BqcError) as err:
        bqc.mp2_energy_df(3, 7, 20, eo, ev, b)
    assert "gap" in str(err.value)


def test_mp2_device_inputs_right_after_torch_work():
    """Inputs written by torch on its default stream and passed at once (no
    caller synchronisation): the binding orders the solve after them."""
    import torch
    bqc = _bqc()
    o, v, naux = 24, 400, 1500
    g = torch.Generator(device="cuda:0")
    g.manual_seed(5)
    b = torch.randn((naux, o, v), generator=g, device="cuda:0", dtype=torch.float64) * 0.05
    eo = torch.sort(torch.rand(o, generator=g, device="cuda:0", dtype=torch.float64) * 1.7 - 2.0).values
    ev = torch.sort(torch.rand(v, generator=g, device="cuda:0", dtype=torch.float64) * 2.9 + 0.1).values
    e = bqc.mp2_energy_df(o, v, naux, eo, ev, b)
    ref = mp2_energy(eo.cpu().numpy(), ev.cpu().numpy(), b.cpu().numpy())
    assert abs(e - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("shape", [(6, 30, 120, 0), (9, 130, 301, 4)])
def test_mp2_pair_energies_match_oracle(shape):
    from oracle.mp2 import pair_energies
    bqc = _bqc()
    o, v, naux, seed = shape
    print(f"case mp2 pairs o={o} v={v} naux={naux} seed={seed}", flush=True)
    eo, ev, b = _factors(o, v, naux, seed)
    ref = np.array([e for _, e in pair_energies(eo, ev, b)])
    e, ex = bqc.mp2_energy_df(o, v, naux, eo, ev, b, pair_energies=True)
    got = ex["pairs"]
    assert got.shape == (o * (o + 1) // 2,)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert abs(e - float(np.sum(got))) <= 1e-13 * abs(e)
