"""Pins of the virtual-triple-loop oracle (oracle/virtual_loop.py).

* The spin-orbital textbook definition, brute-forced on tiny systems (with
  and without an f_ov block).
* The occupied-triple-loop oracle: the same energy summed in the other
  order, through different contractions (X over virtuals at fixed i, j, k
  there; X over occupied indices at fixed a, b, c here).
* Exact special cases: a = b = c contributes nothing; nvir = 1 gives zero.
* Planted mistakes in this loop must break the spin-orbital pin.
"""
import numpy as np
import pytest

import oracle.virtual_loop as vl
from oracle import spinorb_t_energy, t_energy
from synth import make_inputs


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


TINY = [(2, 3, 8, 7), (2, 5, 9, 2), (3, 4, 10, 1), (3, 6, 12, 5), (4, 3, 12, 4), (4, 5, 14, 9)]


@pytest.mark.parametrize("o,v,naux,seed", TINY)
def test_virtual_loop_equals_spin_orbital(o, v, naux, seed):
    x = make_inputs(o, v, naux, seed)
    e = vl.t_energy_virtual_loop(*x.arrays())
    es = spinorb_t_energy(*x.arrays())
    assert _rel(e, es) <= 1e-12


@pytest.mark.parametrize("o,v,naux,seed", [(2, 5, 9, 2), (3, 4, 10, 1), (4, 3, 12, 4)])
def test_virtual_loop_fock_equals_spin_orbital(o, v, naux, seed):
    x = make_inputs(o, v, naux, seed)
    f = np.random.default_rng(1000 + seed).normal(0.0, 0.02, (o, v))
    e = vl.t_energy_virtual_loop(*x.arrays(), fock_ov=f)
    es = spinorb_t_energy(*x.arrays(), fock_ov=f)
    assert _rel(e, es) <= 1e-12


@pytest.mark.parametrize("o,v,naux,seed", [(6, 30, 120, 0), (5, 37, 100, 3), (7, 9, 30, 4)])
def test_virtual_loop_equals_occupied_loop(o, v, naux, seed):
    x = make_inputs(o, v, naux, seed)
    e_v, terms = vl.t_energy_virtual_loop(*x.arrays(), return_triples=True)
    e_o = t_energy(*x.arrays())
    assert len(terms) == v * (v + 1) * (v + 2) // 6 - v
    assert _rel(e_v, e_o) <= 1e-12


def test_equal_virtuals_contribute_nothing():
    x = make_inputs(4, 5, 12, 3)
    e_aaa = vl.virtual_triple_energy(2, 2, 2, 1, *x.arrays())
    scale = abs(vl.virtual_triple_energy(0, 2, 4, 6, *x.arrays()))
    assert abs(e_aaa) <= 1e-13 * scale


def test_single_virtual_gives_zero():
    x = make_inputs(4, 1, 10, 2)
    assert vl.t_energy_virtual_loop(*x.arrays()) == 0.0  # no unique virtual triple exists


@pytest.mark.parametrize("kind", ["hole_sign", "transposed_t2", "dropped_perm", "weight", "z_sign"])
def test_planted_mistakes_break_the_pin(monkeypatch, kind):
    x = make_inputs(3, 4, 10, 1)
    ref = spinorb_t_energy(*x.arrays())
    if kind in ("hole_sign", "transposed_t2"):
        def x_bad(p, q, r, t2, ovvv, ooov):
            tz = t2[:, :, r, :]
            if kind == "transposed_t2":
                tz = t2.transpose(1, 0, 2, 3)[:, :, r, :]
            part = np.tensordot(ovvv[:, p, q, :], tz, axes=([1], [2])).transpose(0, 2, 1)
            hole = np.tensordot(ooov[:, :, :, p], t2[:, :, q, r], axes=([1], [0])).transpose(1, 0, 2)
            return part + hole if kind == "hole_sign" else part - hole
        monkeypatch.setattr(vl, "x_term_fixed_virtuals", x_bad)
    elif kind == "dropped_perm":
        orig = vl.x_term_fixed_virtuals

        def w_bad(a, b, c, t2, ovvv, ooov):
            w = orig(a, b, c, t2, ovvv, ooov).copy()
            w += orig(a, c, b, t2, ovvv, ooov).transpose(0, 2, 1)
            w += orig(b, a, c, t2, ovvv, ooov).transpose(1, 0, 2)
            w += np.einsum("jki->ijk", orig(b, c, a, t2, ovvv, ooov))
            w += np.einsum("kij->ijk", orig(c, a, b, t2, ovvv, ooov))
            return w
        monkeypatch.setattr(vl, "w_occ_tensor", w_bad)
    elif kind == "weight":
        orig_table = vl.virtual_triple_table
        monkeypatch.setattr(vl, "virtual_triple_table", lambda n: [(a, b, c, 6) for (a, b, c, m) in orig_table(n)])
    else:
        def z_bad(a, b, c, v, eps_o, eps_v):
            num = (4.0 * v + np.einsum("jki->ijk", v) + np.einsum("kij->ijk", v)
                   + 2.0 * np.einsum("ikj->ijk", v) - 2.0 * np.einsum("jik->ijk", v)
                   - 2.0 * np.einsum("kji->ijk", v))
            d = (eps_o[:, None, None] + eps_o[None, :, None] + eps_o[None, None, :]
                 - eps_v[a] - eps_v[b] - eps_v[c])
            return num / d
        monkeypatch.setattr(vl, "z_occ_tensor", z_bad)
    assert _rel(vl.t_energy_virtual_loop(*x.arrays()), ref) > 1e-6
