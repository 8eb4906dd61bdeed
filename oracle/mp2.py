"""Closed-shell MP2 correlation energy with density-fitted integrals, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (paper section on MP2, Eq. 1, with the density-fitted
integrals of section 2.2):

    (ia|jb) = sum_Q B^Q_ia B^Q_jb
    E_MP2   = sum_{i,j occupied} sum_{a,b virtual}
              (ia|jb) [2 (ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b)

The sum runs over all ordered (i, j, a, b); ``pair_energies`` returns the
contribution of each unordered occupied pair i <= j (weight 2 for i < j, by
the symmetry (ia|jb) = (jb|ia)), and the total is their exactly rounded sum.
``spinorb_mp2_energy`` is the textbook spin-orbital definition
E = 1/4 sum_{IJAB} |<IJ||AB>|^2 / D_IJ^AB (Szabo & Ostlund, ch. 6), written
with full rank-4 tensors for tiny systems; it pins the closed-shell form.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["pair_energies", "mp2_energy", "spinorb_mp2_energy"]


def _ovov(b_ov):
    """(ia|jb)[i][a][j][b] from b_ov[Q][i][a]."""
    naux, nocc, nvir = b_ov.shape
    m = b_ov.reshape(naux, nocc * nvir)
    return (m.T @ m).reshape(nocc, nvir, nocc, nvir)


def pair_energies(eps_o, eps_v, b_ov):
    """Energy of each occupied pair i <= j (list of ((i, j), e_ij))."""
    g = _ovov(b_ov)
    nocc = b_ov.shape[1]
    out = []
    for i in range(nocc):
        for j in range(i, nocc):
            k = g[i, :, j, :]                       # (ia|jb) as [a][b]
            d = eps_o[i] + eps_o[j] - eps_v[:, None] - eps_v[None, :]
            e = float(np.sum(k * (2.0 * k - k.T) / d))  # k.T[a][b] = (ib|ja)
            out.append(((i, j), e if i == j else 2.0 * e))
    return out


def mp2_energy(eps_o, eps_v, b_ov):
    """E_MP2, the exactly rounded sum of the pair energies."""
    return math.fsum(e for _, e in pair_energies(eps_o, eps_v, b_ov))


def spinorb_mp2_energy(eps_o, eps_v, b_ov):
    """1/4 sum |<IJ||AB>|^2 / (f_I + f_J - f_A - f_B) over spin orbitals."""
    g = _ovov(b_ov)  # (ia|jb)
    nocc, nvir = g.shape[0], g.shape[1]
    o_sp, v_sp = np.repeat(np.arange(nocc), 2), np.repeat(np.arange(nvir), 2)
    o_s, v_s = np.tile([0, 1], nocc), np.tile([0, 1], nvir)
    same = (o_s[:, None] == v_s[None, :]).astype(np.float64)  # [I, A]
    # <IJ|AB> = (IA|JB) d(s_I,s_A) d(s_J,s_B)
    gs = g[np.ix_(o_sp, v_sp, o_sp, v_sp)] * same[:, :, None, None] * same[None, None, :, :]
    ijab = gs.transpose(0, 2, 1, 3)                      # [I, J, A, B] = <IJ|AB>
    anti = ijab - ijab.transpose(0, 1, 3, 2)             # <IJ||AB>
    fo, fv = eps_o[o_sp], eps_v[v_sp]
    d = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
    return float(np.sum(anti * anti / d) / 4.0)
