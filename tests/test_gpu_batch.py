"""Batched solve of several fragments (bqc_t_energy_batch): every
fragment's energy bitwise equal to its solve alone (bqc_t_energy_ex with the
same options), in every precision, with host and device inputs, mixed wave
tiles in one batch, several rounds of triple batches; FP64 against the
oracle."""
import numpy as np
import pytest

from synth import make_inputs

pytestmark = pytest.mark.gpu

SHAPES = [(3, 20, 40, 401), (6, 30, 120, 402), (1, 9, 20, 403), (4, 45, 90, 404), (8, 24, 80, 405),
          (5, 37, 100, 406), (2, 50, 60, 407), (7, 33, 100, 408), (9, 18, 60, 409), (4, 64, 160, 410)]


def _bqc():
    import paper_2502_17963_amd as bqc
    bqc.lib()
    return bqc


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp8"])
def test_batch_equals_alone_host_inputs(prec):
    bqc = _bqc()
    print(f"case batch host inputs {prec}", flush=True)
    xs = [make_inputs(*s) for s in SHAPES]
    alone = [bqc.t_energy(s[0], s[1], *x.arrays(), precision=prec) for s, x in zip(SHAPES, xs)]
    got, st = bqc.t_energy_batch([(s[0], s[1], *x.arrays()) for s, x in zip(SHAPES, xs)], precision=prec,
                                 stats=True)
    assert got == alone, [(a, b) for a, b in zip(got, alone) if a != b]
    assert st["n_triples"] == sum(bqc.num_triples(s[0]) for s in SHAPES)
    assert st["gemm_launches"] >= 1 and st["epilogue_launches"] >= 1


def test_batch_device_inputs_and_oracle():
    import torch

    from oracle import t_energy as oracle_t_energy
    bqc = _bqc()
    print("case batch device inputs fp64", flush=True)
    xs = [make_inputs(*s) for s in SHAPES]
    devs = [[torch.from_numpy(a).to("cuda:0") for a in x.arrays()] for x in xs]
    torch.cuda.synchronize()
    got = bqc.t_energy_batch([(s[0], s[1], *d) for s, d in zip(SHAPES, devs)], precision="fp64")
    alone = [bqc.t_energy(s[0], s[1], *d, precision="fp64") for s, d in zip(SHAPES, devs)]
    torch.cuda.synchronize()
    assert got == alone
    for k in (1, 3, 9):
        ref = oracle_t_energy(*xs[k].arrays())
        assert abs(got[k] - ref) <= 1e-10 * abs(ref), (SHAPES[k], got[k], ref)
    assert got[2] == 0.0  # one occupied orbital: no unique triple


def test_batch_several_rounds_and_wave_tiles():
    """Three fragments whose H buffers together exceed the batch's budget
    (several rounds of triple batches; wave tiles 4 x 4) with small ones
    (2 x 2 and 3 x 3 tiles) in the same batch, split-BF16x3."""
    import torch
    bqc = _bqc()
    print("case batch rounds", flush=True)
    shapes = [(12, 120, 400, 501), (12, 118, 400, 502), (11, 120, 400, 503), (6, 30, 120, 504), (5, 75, 200, 505)]
    devs = []
    for s in shapes:
        x = make_inputs(*s)
        devs.append([torch.from_numpy(a).to("cuda:0") for a in x.arrays()])
        del x
    torch.cuda.synchronize()
    got, st = bqc.t_energy_batch([(s[0], s[1], *d) for s, d in zip(shapes, devs)], precision="bf16x3", stats=True)
    alone = [bqc.t_energy(s[0], s[1], *d, precision="bf16x3") for s, d in zip(shapes, devs)]
    torch.cuda.synchronize()
    print(f"  grouped contraction launches {st['gemm_launches']}, epilogue launches {st['epilogue_launches']}",
          flush=True)
    assert got == alone
    assert st["epilogue_launches"] > 1  # more than one round
