"""Parity at the largest single-GPU shape (nocc=48, nvir=480, naux=1600).

The inputs (51 GB in FP64) are generated on the GPU.  Sampled unique
triples are solved alone in FP64 (a one-triple share of the solve, in the
launch configuration of the full solve) and compared with the oracle's
energy of that triple, computed on the host from copies of the slices it
reads; the same for sampled virtual triples of the virtual-triple loop.
"""
import numpy as np
import pytest

from oracle.closed_shell import triple_energy, triple_table
from oracle.virtual_loop import virtual_triple_energy, virtual_triple_table
from synth import CONFIGS


class _DeviceSlices:
    """(ia|bc) left on the device; indexing copies the requested slice to
    the host (ovvv[p] for the occupied loop, ovvv[:, a, b, :] for the
    virtual one)."""

    def __init__(self, t):
        self.t = t
        self.cache = {}

    def __getitem__(self, key):
        k = repr(key)
        if k not in self.cache:
            self.cache[k] = self.t[key].cpu().numpy()
        return self.cache[k]


@pytest.fixture(scope="module")
def largest():
    import torch

    import paper_2502_17963_amd as bqc
    from synth import make_inputs_device
    bqc.lib()
    o, v, naux, seed = CONFIGS["largest_fragment"]
    print(f"case largest_fragment o={o} v={v} naux={naux} seed={seed}", flush=True)
    dev = make_inputs_device(o, v, naux, seed)
    torch.cuda.synchronize()
    eps_o, eps_v, t1, t2, ovvv, ooov, ovov = dev
    host = [a.cpu().numpy() for a in (eps_o, eps_v, t1, t2)]
    host += [_DeviceSlices(ovvv), ooov.cpu().numpy(), ovov.cpu().numpy()]
    return bqc, o, v, dev, host


@pytest.mark.gpu
@pytest.mark.slow
def test_occupied_loop_sampled_triples(largest):
    bqc, o, v, dev, host = largest
    table = triple_table(o)
    rng = np.random.default_rng(48)
    picks = sorted(set([0, len(table) - 1] + list(rng.choice(len(table), 2, replace=False))))
    for n in picks:
        i, j, k, m = table[n]
        _, ex = bqc.t_energy(o, v, *dev, precision="fp64", triple_energies=True, triple_range=(n, n + 1))
        gpu = ex["triples"][n]
        ref = triple_energy(i, j, k, m, *host)
        print(f"triple {n} ({i},{j},{k}) gpu={gpu:.15e} oracle={ref:.15e}", flush=True)
        assert abs(gpu - ref) <= 1e-10 * abs(ref)


def _vir_index(a, b, c, v):
    """Position of the virtual triple a <= b <= c (not all equal) in the
    lexicographic unique-triple order with a = b = c skipped."""
    before = sum((v - x) * (v - x + 1) // 2 for x in range(a)) + sum(v - y for y in range(a, b)) + (c - b)
    return before - (a + 1)  # the diagonal triples (x, x, x) for x <= a precede it


def test_virtual_index_formula():
    for v in (1, 2, 5, 9):
        for n, (a, b, c, m) in enumerate(virtual_triple_table(v)):
            assert _vir_index(a, b, c, v) == n


@pytest.mark.gpu
@pytest.mark.slow
def test_virtual_loop_sampled_triples(largest):
    bqc, o, v, dev, host = largest
    rng = np.random.default_rng(480)
    trips = [(0, 0, 1), (v - 2, v - 1, v - 1)] + [tuple(sorted(rng.choice(v, 3, replace=False))) for _ in range(2)]
    for (a, b, c) in trips:
        m = 6 if a < b < c else 3
        n = _vir_index(a, b, c, v)
        _, ex = bqc.t_energy(o, v, *dev, precision="fp64", triple_energies=True, triple_range=(n, n + 1),
                             formulation="virtual")
        gpu = ex["triples"][n]
        ref = virtual_triple_energy(a, b, c, m, *host)
        print(f"virtual triple {n} ({a},{b},{c}) gpu={gpu:.15e} oracle={ref:.15e}", flush=True)
        assert abs(gpu - ref) <= 1e-10 * abs(ref)


@pytest.mark.gpu
@pytest.mark.slow
def test_host_inputs_at_full_size(largest):
    """The host-pointer form of the entry point at the largest shape: the
    library uploads the 51 GB of FP64 inputs itself and the energy of a
    sampled triple equals the device-input solve's bit for bit, in FP64 and
    in split-BF16x3."""
    bqc, o, v, dev, host = largest
    hin = [a.cpu().numpy() for a in dev]
    nbytes = sum(a.nbytes for a in hin)
    n = len(triple_table(o)) // 2
    for prec in ("bf16x3", "fp64"):
        e_dev, ex_d = bqc.t_energy(o, v, *dev, precision=prec, triple_energies=True, triple_range=(n, n + 1))
        e_host, ex_h = bqc.t_energy(o, v, *hin, precision=prec, triple_energies=True, triple_range=(n, n + 1),
                                    stats=True)
        up = ex_h["stats"]["upload_s"]
        print(f"{prec} triple {n}: device inputs {e_dev!r}, host inputs {e_host!r}; "
              f"upload {nbytes / 1e9:.1f} GB in {up:.2f} s ({nbytes / up / 1e9:.1f} GB/s)", flush=True)
        assert e_host == e_dev
        assert ex_h["triples"][n] == ex_d["triples"][n]
