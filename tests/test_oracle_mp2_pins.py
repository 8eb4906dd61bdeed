"""Pins of the MP2 oracle against facts other than itself: the spin-orbital
textbook definition (tiny systems), the sign (each occupied pair's energy is
<= 0 because 2x^2 + 2y^2 - 2xy >= 0 and D < 0), exact power-of-two
homogeneity (E(2B) = 16 E(B)), vanishing cases, and planted mistakes."""
import numpy as np
import pytest

import oracle.mp2 as om
from synth import draw_factors


def _factors(o, v, naux, seed):
    b, eps_o, eps_v, _ = draw_factors(o, v, naux, seed)
    return eps_o, eps_v, np.ascontiguousarray(b[:, :o, o:])


TINY = [(1, 2, 4, 0), (2, 3, 6, 1), (3, 4, 8, 2), (3, 5, 10, 3), (4, 4, 12, 4), (2, 6, 9, 5)]


@pytest.mark.parametrize("o,v,naux,seed", TINY)
def test_mp2_equals_spin_orbital(o, v, naux, seed):
    eo, ev, b = _factors(o, v, naux, seed)
    e = om.mp2_energy(eo, ev, b)
    es = om.spinorb_mp2_energy(eo, ev, b)
    assert abs(e - es) <= 1e-12 * abs(es)


def test_pair_energies_are_negative_and_vanish_without_integrals():
    eo, ev, b = _factors(5, 9, 20, 7)
    assert all(e < 0.0 for _, e in om.pair_energies(eo, ev, b))
    assert om.mp2_energy(eo, ev, np.zeros_like(b)) == 0.0


def test_homogeneity_power_of_two_bit_exact():
    eo, ev, b = _factors(4, 7, 15, 8)
    assert om.mp2_energy(eo, ev, 2.0 * b) == 16.0 * om.mp2_energy(eo, ev, b)


@pytest.mark.parametrize("kind", ["no_exchange", "exchange_not_transposed", "factor_one", "no_pair_weight"])
def test_planted_mistakes_break_the_pin(monkeypatch, kind):
    eo, ev, b = _factors(3, 5, 10, 3)
    ref = om.spinorb_mp2_energy(eo, ev, b)

    def bad(eps_o, eps_v, b_ov):
        g = om._ovov(b_ov)
        out = []
        n = b_ov.shape[1]
        for i in range(n):
            for j in range(i, n):
                k = g[i, :, j, :]
                d = eps_o[i] + eps_o[j] - eps_v[:, None] - eps_v[None, :]
                x = k if kind == "exchange_not_transposed" else k.T
                c = 1.0 if kind == "factor_one" else 2.0
                num = c * k * k if kind == "no_exchange" else k * (c * k - x)
                e = float(np.sum(num / d))
                out.append(((i, j), e if (i == j or kind == "no_pair_weight") else 2.0 * e))
        return out
    monkeypatch.setattr(om, "pair_energies", bad)
    assert abs(om.mp2_energy(eo, ev, b) - ref) > 1e-6 * abs(ref)
