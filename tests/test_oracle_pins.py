"""Pins of the FP64 oracle against facts other than itself.

* The spin-orbital textbook definition, brute-forced on tiny systems.
* Invariants that hold exactly: permutational symmetry of W, vanishing cases,
  power-of-two homogeneity (bit-exact), orbital relabelling, size
  extensivity of two non-interacting fragments.
* Planted mistakes: each plausible error in the closed-shell loop (dropped
  term, wrong sign, transposed operand, wrong weight) must break a pin.
"""
import itertools
import math

import numpy as np
import pytest

import oracle.closed_shell as cs
from oracle import spinorb_t_energy, t_energy, w_tensor
from synth import direct_sum_inputs, make_inputs


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


TINY = [(1, 3, 6, 0), (2, 1, 5, 3), (2, 3, 8, 7), (2, 5, 9, 2), (3, 4, 10, 1), (3, 5, 12, 11),
        (3, 6, 12, 5), (4, 3, 12, 4), (4, 5, 14, 9), (4, 6, 16, 8)]


@pytest.mark.parametrize("o,v,naux,seed", TINY)
def test_closed_shell_equals_spin_orbital(o, v, naux, seed):
    x = make_inputs(o, v, naux, seed)
    e = t_energy(*x.arrays())
    es = spinorb_t_energy(*x.arrays())
    assert abs(e - es) <= 1e-12 * max(abs(es), 1e-20) + 1e-24


@pytest.mark.parametrize("o,v,naux,seed", TINY[2:7])
def test_fourth_order_part_equals_spin_orbital(o, v, naux, seed):
    """t1 = 0: only the connected triples remain (E_T[4] with MP1 t2)."""
    x = make_inputs(o, v, naux, seed)
    x.t1[:] = 0.0
    e = t_energy(*x.arrays())
    es = spinorb_t_energy(*x.arrays())
    assert e < 0.0
    assert _rel(e, es) <= 1e-12


def test_w_permutational_symmetry():
    o, v = 3, 5
    x = make_inputs(o, v, 12, 3)
    i, j, k = 0, 1, 2
    w = w_tensor(i, j, k, x.t2, x.ovvv, x.ooov)
    occ = (i, j, k)
    for perm in itertools.permutations(range(3)):
        wp = w_tensor(*(occ[p] for p in perm), x.t2, x.ovvv, x.ooov)
        # W_{pi(ijk)}^{pi(abc)} = W_ijk^abc
        letters = "abc"
        spec = "".join(letters[p] for p in perm) + "->abc"
        assert np.max(np.abs(np.einsum(spec, wp) - w)) <= 1e-15 * np.max(np.abs(w))


def test_single_occupied_gives_zero():
    x = make_inputs(1, 6, 10, 2)
    assert t_energy(*x.arrays()) == 0.0  # no unique triple exists
    # the skipped i = j = k triple really contributes nothing: the numerator
    # operator's coefficients sum to zero and V is symmetric in abc there
    y = make_inputs(3, 6, 10, 2)
    e_iii = cs.triple_energy(1, 1, 1, 1, *y.arrays())
    scale = abs(cs.triple_energy(0, 1, 2, 6, *y.arrays()))
    assert abs(e_iii) <= 1e-13 * scale


def test_single_virtual_gives_zero():
    x = make_inputs(4, 1, 10, 2)
    e = t_energy(*x.arrays())
    # every element is a=b=c, where the numerator operator annihilates V
    scale = np.max(np.abs(x.ovvv)) ** 2 * np.max(np.abs(x.t2)) ** 2
    assert abs(e) <= 1e-12 * scale


def test_zero_amplitudes():
    x = make_inputs(3, 5, 12, 4)
    x.t1[:] = 0.0
    x.t2[:] = 0.0
    assert t_energy(*x.arrays()) == 0.0
    y = make_inputs(3, 5, 12, 4)
    y.t2[:] = 0.0  # W = 0, so every term W*Z vanishes whatever t1 is
    assert t_energy(*y.arrays()) == 0.0


def test_homogeneity_power_of_two_bit_exact():
    x = make_inputs(3, 5, 12, 6)
    e0 = t_energy(*x.arrays())
    # integrals x4 (B -> 2B), amplitudes fixed: E -> 16 E exactly
    e1 = t_energy(x.eps_o, x.eps_v, x.t1, x.t2, 4 * x.ovvv, 4 * x.ooov, 4 * x.ovov)
    assert e1 == 16.0 * e0
    # B -> 2B with t2 regenerated (x4) and t1 -> 4 t1: E -> 256 E exactly
    e2 = t_energy(x.eps_o, x.eps_v, 4 * x.t1, 4 * x.t2, 4 * x.ovvv, 4 * x.ooov, 4 * x.ovov)
    assert e2 == 256.0 * e0
    # eps -> 2 eps with amplitudes fixed: E -> E / 2 exactly
    e3 = t_energy(2 * x.eps_o, 2 * x.eps_v, *x.arrays()[2:])
    assert e3 == 0.5 * e0


def test_energy_scale_inverse_in_eps():
    x = make_inputs(3, 4, 10, 8)
    e0 = t_energy(*x.arrays())
    lam = 1.7
    e1 = t_energy(lam * x.eps_o, lam * x.eps_v, *x.arrays()[2:])
    assert _rel(e1 * lam, e0) < 1e-13


def test_orbital_relabelling_invariance():
    o, v = 4, 5
    x = make_inputs(o, v, 14, 12)
    e0 = t_energy(*x.arrays())
    po = np.array([2, 0, 3, 1])
    pv = np.array([4, 1, 0, 3, 2])
    e1 = t_energy(x.eps_o[po], x.eps_v[pv], x.t1[np.ix_(po, pv)],
                  x.t2[np.ix_(po, po, pv, pv)], x.ovvv[np.ix_(po, pv, pv, pv)],
                  x.ooov[np.ix_(po, po, po, pv)], x.ovov[np.ix_(po, pv, po, pv)])
    assert _rel(e1, e0) < 1e-13


def test_size_extensivity_two_fragments():
    ea = t_energy(*make_inputs(2, 4, 8, 21).arrays())
    eb = t_energy(*make_inputs(3, 5, 9, 22).arrays())
    eab = t_energy(*direct_sum_inputs([(2, 4, 8, 21), (3, 5, 9, 22)]))
    assert _rel(eab, ea + eb) < 1e-12


# ------------------------------------------------- non-canonical Fock term (f_ov)

FOCK = [(2, 3, 8, 7), (3, 5, 12, 0), (2, 6, 14, 1), (4, 4, 10, 2), (3, 6, 16, 3)]


def _fock(o, v, seed):
    return np.random.default_rng(1000 + seed).normal(0.0, 0.02, (o, v))


@pytest.mark.parametrize("o,v,naux,seed", FOCK)
def test_fock_term_equals_spin_orbital(o, v, naux, seed):
    """With f_ov != 0 the disconnected triples gain f_IA t_JK^BC (spin-orbital
    definition); the closed-shell loop folds f_ia t_jk^bc + f_jb t_ik^ac +
    f_kc t_ij^ab into V."""
    x = make_inputs(o, v, naux, seed)
    f = _fock(o, v, seed)
    e = t_energy(*x.arrays(), fock_ov=f)
    es = spinorb_t_energy(*x.arrays(), fock_ov=f)
    assert _rel(e, es) <= 1e-12
    assert _rel(e, t_energy(*x.arrays())) > 1e-3  # the term is not negligible here


def test_zero_fock_is_the_canonical_energy():
    x = make_inputs(3, 5, 12, 0)
    assert t_energy(*x.arrays(), fock_ov=np.zeros((3, 5))) == t_energy(*x.arrays())


@pytest.mark.parametrize("kind", ["transposed", "sign", "one_term"])
def test_planted_fock_mistakes_break_the_pin(monkeypatch, kind):
    x = make_inputs(3, 5, 12, 0)
    f = _fock(3, 5, 0)
    ref = spinorb_t_energy(*x.arrays(), fock_ov=f)
    orig_v = cs.v_tensor

    def v_bad(i, j, k, w, t1, ovov, t2=None, fock_ov=None):
        v = orig_v(i, j, k, w, t1, ovov)
        s = -1.0 if kind == "sign" else 1.0
        tjk = t2[j, k].T if kind == "transposed" else t2[j, k]
        v += s * fock_ov[i][:, None, None] * tjk[None, :, :]
        if kind != "one_term":
            v += s * fock_ov[j][None, :, None] * t2[i, k][:, None, :]
            v += s * fock_ov[k][None, None, :] * t2[i, j][:, :, None]
        return v
    monkeypatch.setattr(cs, "v_tensor", v_bad)
    assert _rel(cs.t_energy(*x.arrays(), fock_ov=f), ref) > 1e-6


# ---------------------------------------------------------------- planted mistakes

def _mutant_x(kind):
    def x_term(p, q, r, t2, ovvv, ooov):
        nvir = t2.shape[2]
        b = t2[r, q].T
        if kind == "transposed_t2":
            b = t2[q, r].T
        part = (ovvv[p].reshape(nvir * nvir, nvir) @ b).reshape(nvir, nvir, nvir)
        if kind == "hole_index":
            hole = np.tensordot(ooov[q, :, p, :], t2[r, :], axes=([0], [0]))
        else:
            hole = np.tensordot(ooov[q, :, p, :], t2[:, r], axes=([0], [0]))
        if kind == "dropped_hole":
            return part
        if kind == "hole_sign":
            return part + hole
        return part - hole
    return x_term


@pytest.mark.parametrize("kind", ["dropped_hole", "hole_sign", "transposed_t2", "hole_index"])
def test_planted_contraction_mistakes_break_the_pin(monkeypatch, kind):
    x = make_inputs(3, 4, 10, 1)
    ref = spinorb_t_energy(*x.arrays())
    monkeypatch.setattr(cs, "x_term", _mutant_x(kind))
    bad = cs.t_energy(*x.arrays())
    assert _rel(bad, ref) > 1e-6


def test_planted_singles_and_weight_mistakes_break_the_pin(monkeypatch):
    x = make_inputs(3, 4, 10, 1)
    ref = spinorb_t_energy(*x.arrays())
    orig_v = cs.v_tensor

    def v_no_singles(i, j, k, w, t1, ovov, *rest):
        return w.copy()
    monkeypatch.setattr(cs, "v_tensor", v_no_singles)
    assert _rel(cs.t_energy(*x.arrays()), ref) > 1e-6
    monkeypatch.setattr(cs, "v_tensor", orig_v)

    orig_table = cs.triple_table
    monkeypatch.setattr(cs, "triple_table", lambda n: [(i, j, k, 6) for (i, j, k, m) in orig_table(n)])
    assert _rel(cs.t_energy(*x.arrays()), ref) > 1e-6
    monkeypatch.setattr(cs, "triple_table", orig_table)

    def z_wrong(i, j, k, v, eps_o, eps_v):  # coefficients of the garbled printed form
        num = (4.0 * np.einsum("cab->abc", v) + np.einsum("bca->abc", v)
               - 2.0 * (np.einsum("cba->abc", v) + np.einsum("acb->abc", v) + np.einsum("bac->abc", v)))
        d = eps_o[i] + eps_o[j] + eps_o[k] - eps_v[:, None, None] - eps_v[None, :, None] - eps_v[None, None, :]
        return num / d
    monkeypatch.setattr(cs, "z_tensor", z_wrong)
    assert _rel(cs.t_energy(*x.arrays()), ref) > 1e-6


def test_fsum_total_matches_pairwise_total():
    x = make_inputs(6, 30, 120, 0)
    e, terms = t_energy(*x.arrays(), return_triples=True)
    assert len(terms) == 6 * 7 * 8 // 6 - 6
    assert _rel(e, float(np.sum(terms))) < 1e-14
    assert math.isfinite(e)
