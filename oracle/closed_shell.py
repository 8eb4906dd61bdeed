"""Closed-shell (T) energy, plain FP64 loop over unique occupied triples.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed (paper section 2.4.2, Eqs. 2-7; the closed-shell (T)
correction of Raghavachari et al. 1989 for a canonical RHF reference):

For an occupied triple (i, j, k) and virtuals (a, b, c) define, for any
ordered occupied triple (p, q, r) and virtuals (x, y, z),

    X_pqr(x, y, z) = sum_d (px|yd) t_{rq}^{zd} - sum_l (px|ql) t_{lr}^{yz}

and sum it over the six simultaneous permutations of the pairs
(i,a), (j,b), (k,c)  (the operator P of Eq. 2):

    W_abc = X_ijk(a,b,c) + X_ikj(a,c,b) + X_jik(b,a,c)
          + X_jki(b,c,a) + X_kij(c,a,b) + X_kji(c,b,a).

The singles ("disconnected") term of Eqs. 6-7 enters through

    V_abc = W_abc + t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb),

the energy denominator of Eq. 3 is D_abc = e_i + e_j + e_k - e_a - e_b - e_c,
and with

    Z_abc = [4 V_abc + V_bca + V_cab - 2 V_acb - 2 V_bac - 2 V_cba] / D_abc

(V_bca is V evaluated at virtual positions (b, c, a) for the same i, j, k)
each unique triple i <= j <= k contributes

    e_ijk = (m / 3) * sum_abc W_abc Z_abc,

m = 6 if i < j < k, m = 3 if exactly two indices coincide; triples with
i = j = k contribute exactly zero and are skipped.  E_T = sum of e_ijk.

Readings of the paper's equations (they are garbled in the text):
 1. The hole term of Eq. 2 is  -sum_l (ia|jl) t_{lk}^{bc}  (a sum over l
    with a minus sign), not "+ (ia|jl) t_kl^bc" inside the sum over d.
 2. The numerator of Eq. 3 is the operator 4 + (two cyclic permutations)
    - 2 (three transpositions) applied to V (not to w); its coefficients
    sum to zero, as they must for E_T = 0 when nocc = 1.
 3. The "alpha" of Eq. 3 that removes double counting is, for this loop
    over occupied triples, the weight m / 3.
 4. "P = sum over all permutations of abc" is the sum over the six
    simultaneous permutations of the index pairs.
 5. The Fock term x_k F_ck of Eqs. 5 and 7 vanishes for a canonical HF
    reference (f_ov = 0).  For a reference with diagonal occupied and
    virtual Fock blocks (orbital energies e) but f_ov != 0 it enters, like
    the singles term, through V:
        V_abc += f_ia t_jk^bc + f_jb t_ik^ac + f_kc t_ij^ab
    (fock_ov[i][a] = f_ia; optional argument, None = canonical).
 6. The singles term y_k t_k^c of Eqs. 6-7 is folded into V above: because
    the operator in Z is symmetric under the sum over abc, the two routes
    give the same energy.
The spin-orbital brute force in ``spin_orbital`` pins all of these.

Integral layouts: ovvv[i][a][b][c] = (ia|bc), ooov[j][l][i][a] = (jl|ia)
(so (ia|jl) = ooov[j][l][i][a]), ovov[i][a][j][b] = (ia|jb),
t2[i][j][a][b] = t_ij^ab, t1[i][a] = t_i^a.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["triple_table", "x_term", "w_tensor", "v_tensor", "z_tensor",
           "triple_energy", "t_energy"]


def triple_table(nocc: int):
    """Unique occupied triples i <= j <= k without i = j = k, with weight m.

    Ordered lexicographically by (i, j, k).
    """
    out = []
    for i in range(nocc):
        for j in range(i, nocc):
            for k in range(j, nocc):
                if i == j == k:
                    continue
                m = 6 if (i < j < k) else 3
                out.append((i, j, k, m))
    return out


def x_term(p, q, r, t2, ovvv, ooov):
    """X_pqr(x,y,z) = sum_d (px|yd) t_rq^zd - sum_l (px|ql) t_lr^yz  (Eq. 2)."""
    nvir = t2.shape[2]
    # particle part: (px|yd) over rows (x,y) times t_rq^{zd} over columns z
    part = (ovvv[p].reshape(nvir * nvir, nvir) @ t2[r, q].T).reshape(nvir, nvir, nvir)
    # hole part: (px|ql) = ooov[q][l][p][x]; t_lr^yz = t2[l][r][y][z]
    hole = np.tensordot(ooov[q, :, p, :], t2[:, r], axes=([0], [0]))
    return part - hole


def w_tensor(i, j, k, t2, ovvv, ooov):
    """W_abc for one occupied triple: the six-fold pair permutation of X."""
    w = x_term(i, j, k, t2, ovvv, ooov)
    w = w + np.einsum("acb->abc", x_term(i, k, j, t2, ovvv, ooov))
    w = w + np.einsum("bac->abc", x_term(j, i, k, t2, ovvv, ooov))
    w = w + np.einsum("bca->abc", x_term(j, k, i, t2, ovvv, ooov))
    w = w + np.einsum("cab->abc", x_term(k, i, j, t2, ovvv, ooov))
    w = w + np.einsum("cba->abc", x_term(k, j, i, t2, ovvv, ooov))
    return w


def v_tensor(i, j, k, w, t1, ovov, t2=None, fock_ov=None):
    """V_abc = W_abc + t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb)
             [+ f_ia t_jk^bc + f_jb t_ik^ac + f_kc t_ij^ab  if fock_ov is given]."""
    v = w.copy()
    v += t1[i][:, None, None] * ovov[j, :, k, :][None, :, :]
    v += t1[j][None, :, None] * ovov[i, :, k, :][:, None, :]
    v += t1[k][None, None, :] * ovov[i, :, j, :][:, :, None]
    if fock_ov is not None:
        v += fock_ov[i][:, None, None] * t2[j, k][None, :, :]
        v += fock_ov[j][None, :, None] * t2[i, k][:, None, :]
        v += fock_ov[k][None, None, :] * t2[i, j][:, :, None]
    return v


def z_tensor(i, j, k, v, eps_o, eps_v):
    """Z_abc = [4V_abc + V_bca + V_cab - 2V_acb - 2V_bac - 2V_cba] / D_abc."""
    num = (4.0 * v
           + np.einsum("bca->abc", v)
           + np.einsum("cab->abc", v)
           - 2.0 * np.einsum("acb->abc", v)
           - 2.0 * np.einsum("bac->abc", v)
           - 2.0 * np.einsum("cba->abc", v))
    d = (eps_o[i] + eps_o[j] + eps_o[k]
         - eps_v[:, None, None] - eps_v[None, :, None] - eps_v[None, None, :])
    return num / d


def triple_energy(i, j, k, m, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, fock_ov=None):
    """e_ijk = (m/3) sum_abc W_abc Z_abc for one unique triple."""
    w = w_tensor(i, j, k, t2, ovvv, ooov)
    v = v_tensor(i, j, k, w, t1, ovov, t2, fock_ov)
    z = z_tensor(i, j, k, v, eps_o, eps_v)
    return (m / 3.0) * float(np.sum(w * z))


def t_energy(eps_o, eps_v, t1, t2, ovvv, ooov, ovov, return_triples=False, fock_ov=None):
    """E_T, summed over unique triples with math.fsum (exactly rounded)."""
    nocc = t1.shape[0]
    terms = []
    for (i, j, k, m) in triple_table(nocc):
        terms.append(triple_energy(i, j, k, m, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, fock_ov))
    e = math.fsum(terms)
    if return_triples:
        return e, terms
    return e
