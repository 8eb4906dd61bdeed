"""Invariants of the (T) energy checked on the GPU path, in every precision
and both loops (the same facts pin the oracle in test_oracle_pins.py).

Power-of-two scalings commute with every rounding of the path (the BF16
hi/lo split and the FP8 block exponents included), so they hold bit for
bit: integrals x4 => E x16; orbital energies x2 => E / 2; zero amplitudes
=> E = 0.  Orbital relabelling and the separability of non-interacting
fragments hold to rounding.
"""
import numpy as np
import pytest

from synth import direct_sum_inputs, make_inputs

pytestmark = pytest.mark.gpu

CASES = [(p, f) for f in ("occupied", "virtual") for p in ("fp64", "fp32", "bf16x3", "fp8")
         if not (f == "virtual" and p == "fp8")]


def _bqc():
    import paper_2502_17963_amd as bqc
    bqc.lib()
    return bqc


@pytest.mark.parametrize("prec,form", CASES)
def test_power_of_two_scalings_and_zero_amplitudes_bit_exact(prec, form):
    bqc = _bqc()
    print(f"case invariants {prec} {form}", flush=True)
    o, v = 6, 30
    x = make_inputs(o, v, 120, 3)
    E = lambda *a: bqc.t_energy(o, v, *a, precision=prec, formulation=form)  # noqa: E731
    e0 = E(*x.arrays())
    assert E(x.eps_o, x.eps_v, x.t1, x.t2, 4 * x.ovvv, 4 * x.ooov, 4 * x.ovov) == 16.0 * e0
    assert E(2 * x.eps_o, 2 * x.eps_v, *x.arrays()[2:]) == 0.5 * e0
    assert E(x.eps_o, x.eps_v, 0 * x.t1, 0 * x.t2, x.ovvv, x.ooov, x.ovov) == 0.0


@pytest.mark.parametrize("form", ["occupied", "virtual"])
def test_orbital_relabelling(form):
    bqc = _bqc()
    o, v = 7, 37
    x = make_inputs(o, v, 100, 12)
    rng = np.random.default_rng(77)
    po, pv = rng.permutation(o), rng.permutation(v)
    e0 = bqc.t_energy(o, v, *x.arrays(), formulation=form)
    e1 = bqc.t_energy(o, v, x.eps_o[po], x.eps_v[pv], x.t1[np.ix_(po, pv)],
                      np.ascontiguousarray(x.t2[np.ix_(po, po, pv, pv)]),
                      np.ascontiguousarray(x.ovvv[np.ix_(po, pv, pv, pv)]),
                      np.ascontiguousarray(x.ooov[np.ix_(po, po, po, pv)]),
                      np.ascontiguousarray(x.ovov[np.ix_(po, pv, po, pv)]), formulation=form)
    assert abs(e1 - e0) <= 1e-12 * abs(e0)


@pytest.mark.parametrize("prec,form,tol", [("fp64", "occupied", 1e-12), ("fp64", "virtual", 1e-12),
                                           ("bf16x3", "occupied", 1e-6), ("bf16x3", "virtual", 1e-6)])
def test_non_interacting_fragments_add(prec, form, tol):
    bqc = _bqc()
    shapes = [(4, 21, 60, 31), (5, 26, 70, 32)]
    es = [bqc.t_energy(o, v, *make_inputs(o, v, q, s).arrays(), precision=prec, formulation=form)
          for (o, v, q, s) in shapes]
    no, nv = sum(s[0] for s in shapes), sum(s[1] for s in shapes)
    eab = bqc.t_energy(no, nv, *direct_sum_inputs(shapes), precision=prec, formulation=form)
    assert abs(eab - sum(es)) <= tol * abs(sum(es))
