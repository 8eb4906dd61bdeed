"""Serving: continuous batching of independent fragment solves.

Each result must be bitwise identical alone (bqc_t_energy_ex) and in the
mix, and within 1e-10 of the FP64 oracle; admission under a small memory
budget, oversize rejection, failure isolation and ticket life cycle.
"""
import numpy as np
import pytest

from oracle import t_energy as oracle_t_energy
from synth import make_inputs

pytestmark = pytest.mark.gpu

SHAPES = [(3, 20, 40, 101), (6, 30, 120, 102), (4, 45, 90, 103), (8, 24, 80, 104),
          (5, 37, 100, 105), (2, 50, 60, 106), (7, 33, 100, 107), (9, 18, 60, 108)]


def _bqc():
    import paper_2502_17963_amd as bqc
    bqc.lib()
    return bqc


def test_each_result_same_alone_and_in_the_mix():
    bqc = _bqc()
    xs = [make_inputs(*s) for s in SHAPES]
    alone = [bqc.t_energy(s[0], s[1], *x.arrays()) for s, x in zip(SHAPES, xs)]
    with bqc.Server(precision="fp64", max_inflight=3, mem_budget_bytes=1 << 30) as srv:
        tickets = [srv.submit(s[0], s[1], *x.arrays()) for s, x in zip(SHAPES, xs)]
        # poll out of order
        res = {}
        for t in reversed(tickets):
            res[t] = srv.wait(t)
        for t in tickets:
            with pytest.raises(bqc.BqcError) as ei:
                srv.poll(t)
            assert ei.value.code == -4  # consumed
    for k, t in enumerate(tickets):
        e, st = res[t]
        assert e == alone[k], (SHAPES[k], e, alone[k])
        ref = oracle_t_energy(*xs[k].arrays())
        assert abs(e - ref) <= 1e-10 * abs(ref)
        assert st["n_triples"] == bqc.num_triples(SHAPES[k][0])
        assert st["total_s"] >= st["queue_s"] >= 0.0


def test_small_budget_admission_and_oversize_rejection():
    bqc = _bqc()
    big = (8, 60, 100, 201)
    small = [(3, 20, 40, 202), (4, 25, 50, 203), (3, 30, 40, 204), (5, 22, 60, 205)]
    need = max(bqc.footprint(s[0], s[1]) for s in small)
    budget = int(need * 1.5)  # one small request at a time, at most
    assert bqc.footprint(big[0], big[1]) > budget
    with bqc.Server(precision="fp64", max_inflight=4, mem_budget_bytes=budget) as srv:
        xb = make_inputs(*big)
        with pytest.raises(bqc.BqcError) as ei:
            srv.submit(big[0], big[1], *xb.arrays())
        assert ei.value.code == -2
        xs = [make_inputs(*s) for s in small]
        ts = [srv.submit(s[0], s[1], *x.arrays()) for s, x in zip(small, xs)]
        out = [srv.wait(t)[0] for t in ts]
    for s, x, e in zip(small, xs, out):
        assert e == bqc.t_energy(s[0], s[1], *x.arrays())


def test_invalid_request_rejected_others_complete():
    bqc = _bqc()
    good = make_inputs(4, 20, 40, 301)
    bad = make_inputs(4, 20, 40, 302)
    bad.eps_o[-1] = bad.eps_v[0] + 1.0
    with bqc.Server(precision="fp64", max_inflight=2, mem_budget_bytes=1 << 28) as srv:
        t1 = srv.submit(4, 20, *good.arrays())
        with pytest.raises(bqc.BqcError) as ei:
            srv.submit(4, 20, *bad.arrays())
        assert ei.value.code == -1
        t2 = srv.submit(4, 20, *good.arrays())
        e1, _ = srv.wait(t1)
        e2, _ = srv.wait(t2)
    assert e1 == e2
    with pytest.raises(bqc.BqcError):
        srv.poll(12345)


def test_fp32_serving_matches_fp32_alone():
    bqc = _bqc()
    xs = [make_inputs(*s) for s in SHAPES[:4]]
    with bqc.Server(precision="fp32", max_inflight=4, mem_budget_bytes=1 << 30) as srv:
        ts = [srv.submit(s[0], s[1], *x.arrays()) for s, x in zip(SHAPES, xs)]
        got = [srv.wait(t)[0] for t in ts]
    for s, x, e in zip(SHAPES, xs, got):
        assert e == bqc.t_energy(s[0], s[1], *x.arrays(), precision="fp32")


def test_device_resident_submit():
    """Fragments generated on the GPU and submitted as device pointers."""
    import torch

    from synth import make_inputs_device
    bqc = _bqc()
    shapes = [(3, 20, 40, 401), (5, 33, 80, 402), (4, 27, 60, 403)]
    xs = [make_inputs_device(*s) for s in shapes]
    with bqc.Server(precision="fp64", max_inflight=2, mem_budget_bytes=1 << 29) as srv:
        ts = [srv.submit(s[0], s[1], *x) for s, x in zip(shapes, xs)]
        got = [srv.wait(t)[0] for t in ts]
    for s, x, e in zip(shapes, xs, got):
        assert e == bqc.t_energy(s[0], s[1], *x)
        torch.cuda.synchronize()
        ref = oracle_t_energy(*[a.cpu().numpy() for a in x])
        assert abs(e - ref) <= 1e-10 * abs(ref)


def test_graph_and_direct_launch_agree():
    bqc = _bqc()
    xs = [make_inputs(*s) for s in SHAPES[:5]]
    out = {}
    for graphs in (True, False):
        with bqc.Server(precision="fp64", max_inflight=3, mem_budget_bytes=1 << 30, graphs=graphs) as srv:
            ts = [srv.submit(s[0], s[1], *x.arrays()) for s, x in zip(SHAPES, xs)]
            out[graphs] = [srv.wait(t)[0] for t in ts]
    assert out[True] == out[False]


def test_request_of_many_graphs_matches_direct_solve():
    """A request whose triple batches span several hipGraphs (210 triples in
    70 batches of three; a graph holds at most 64 batches) gives bitwise the
    energy of the stream-launched single solve."""
    import torch

    import paper_2502_17963_amd as bqc
    from synth import make_inputs_device
    o, v, naux = 10, 304, 600
    print(f"case many-graph request o={o} v={v}", flush=True)
    x = make_inputs_device(o, v, naux, 77)
    torch.cuda.synchronize()
    e_direct = bqc.t_energy(o, v, *x, precision="bf16x3")
    torch.cuda.synchronize()
    with bqc.Server(precision="bf16x3", max_inflight=2, mem_budget_bytes=int(8e9)) as srv:
        t = srv.submit(o, v, *x)
        e_srv, st = srv.wait(t)
    assert e_srv == e_direct


def test_cancel_queued_request():
    """One slot: the requests behind the first are queued; cancelling one of
    them removes it (its terminal poll is BQC_ECANCELED) and every other
    request's energy is the one it has alone."""
    bqc = _bqc()
    shapes = [(6, 30, 120, 301), (5, 24, 80, 302), (4, 20, 60, 303), (6, 28, 100, 304)]
    xs = [make_inputs(*s) for s in shapes]
    alone = [bqc.t_energy(s[0], s[1], *x.arrays(), precision="bf16x3") for s, x in zip(shapes, xs)]
    print("case serving cancel", flush=True)
    with bqc.Server(precision="bf16x3", max_inflight=1, mem_budget_bytes=1 << 30) as srv:
        tickets = [srv.submit(s[0], s[1], *x.arrays()) for s, x in zip(shapes, xs)]
        cancelled = srv.cancel(tickets[3])
        for k, t in enumerate(tickets):
            if k == 3 and cancelled:
                try:
                    e, _ = srv.wait(t)  # it had finished before the cancel
                except bqc.BqcError as err:
                    assert err.code == -6
                    continue
            else:
                e, _ = srv.wait(t)
            assert e == alone[k], (shapes[k], e, alone[k])
        with pytest.raises(bqc.BqcError) as ei:
            srv.cancel(tickets[0])
        assert ei.value.code == -4


@pytest.mark.parametrize("grouping", [True, False])
def test_small_requests_grouped_into_batches(grouping):
    """One slot and a queue of small requests: with grouping the slot admits
    several at once and runs them as one batch (grouped launches); every
    result is bitwise the request's alone either way."""
    bqc = _bqc()
    print(f"case serving grouping={grouping}", flush=True)
    shapes = [(3, 20, 40, 601), (4, 25, 50, 602), (2, 30, 40, 603), (5, 22, 60, 604), (6, 30, 120, 605),
              (3, 17, 30, 606), (4, 45, 90, 607), (7, 33, 100, 608), (1, 9, 20, 609), (8, 24, 80, 610),
              (5, 37, 100, 611), (2, 50, 60, 612)]
    xs = [make_inputs(*s) for s in shapes]
    alone = [bqc.t_energy(s[0], s[1], *x.arrays(), precision="bf16x3") for s, x in zip(shapes, xs)]
    with bqc.Server(precision="bf16x3", max_inflight=1, mem_budget_bytes=4 << 30, grouping=grouping) as srv:
        tickets = [srv.submit(s[0], s[1], *x.arrays()) for s, x in zip(shapes, xs)]
        res = [srv.wait(t) for t in tickets]
    grouped = 0
    for k, (e, st) in enumerate(res):
        assert e == alone[k], (shapes[k], e, alone[k])
        grouped += st["gemm_launches"] > 0  # set for requests that ran in a batch
    print(f"  {grouped} of {len(shapes)} requests ran in batches", flush=True)
    if grouping:
        assert grouped >= 2
    else:
        assert grouped == 0
