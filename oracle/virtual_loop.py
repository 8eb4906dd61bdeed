"""Closed-shell (T) energy, plain FP64 loop over unique virtual triples.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper organises its (T) iteration (section 2.4.2, Eqs. 2-4 and 6-7)
around the virtual triples (a, b, c): for each one it forms tensors over the
three occupied indices and accumulates the energy.  The quantity is the E_T
of ``closed_shell`` (the same sum over all i, j, k, a, b, c); only the order
of the sums is different, so the two oracles pin each other.

For fixed virtuals (a, b, c) and any ordered virtual triple (p, q, r) define
over the occupied indices (x, y, z)

    X^{pqr}(x, y, z) = sum_d (xp|qd) t_{zy}^{rd} - sum_l (xp|yl) t_{lz}^{qr}

(Eq. 2 with the virtual indices held fixed) and sum the six simultaneous
permutations of the pairs (i,a), (j,b), (k,c):

    W^{ijk} = X^{abc}(i,j,k) + X^{acb}(i,k,j) + X^{bac}(j,i,k)
            + X^{bca}(j,k,i) + X^{cab}(k,i,j) + X^{cba}(k,j,i).

The singles term (Eqs. 6-7) and the optional f_ov term enter V as in the
occupied loop,

    V^{ijk} = W^{ijk} + t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb)
              [+ f_ia t_jk^bc + f_jb t_ik^ac + f_kc t_ij^ab],

D^{ijk} = e_i + e_j + e_k - e_a - e_b - e_c (Eq. 3), and because every term
is unchanged when the pairs are permuted together (V^{ijk}_{bca} =
V^{kij}_{abc}), the numerator operator of Eq. 3 acts on the occupied
positions:

    Z^{ijk} = [4 V^{ijk} + V^{jki} + V^{kij} - 2 V^{ikj} - 2 V^{jik} - 2 V^{kji}] / D^{ijk}.

Each unique virtual triple a <= b <= c contributes

    e_abc = (m / 3) * sum_{ijk} W^{ijk} Z^{ijk},

m = 6 if a < b < c and 3 if exactly two coincide (the double-counting
factor of Eq. 3 for this loop); a = b = c contributes exactly zero (W and V
are then symmetric in i, j, k and the operator's coefficients sum to zero)
and is skipped.  E_T = sum of e_abc.

Layouts as in ``closed_shell``: ovvv[i][a][b][c] = (ia|bc), ooov[j][l][i][a]
= (jl|ia), ovov[i][a][j][b] = (ia|jb), t2[i][j][a][b], t1[i][a],
fock_ov[i][a].
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["virtual_triple_table", "x_term_fixed_virtuals", "w_occ_tensor", "v_occ_tensor",
           "z_occ_tensor", "virtual_triple_energy", "t_energy_virtual_loop"]


def virtual_triple_table(nvir: int):
    """Unique virtual triples a <= b <= c without a = b = c, with weight m,
    in lexicographic order of (a, b, c)."""
    out = []
    for a in range(nvir):
        for b in range(a, nvir):
            for c in range(b, nvir):
                if a == b == c:
                    continue
                out.append((a, b, c, 6 if (a < b < c) else 3))
    return out


def x_term_fixed_virtuals(p, q, r, t2, ovvv, ooov):
    """X^{pqr}(x,y,z) = sum_d (xp|qd) t_zy^rd - sum_l (xp|yl) t_lz^qr, an
    array over the occupied indices [x][y][z]."""
    # particle part: rows x: (xp|qd) = ovvv[x][p][q][d]; t_zy^{rd} = t2[z][y][r][d]
    part = np.tensordot(ovvv[:, p, q, :], t2[:, :, r, :], axes=([1], [2]))  # [x][z][y]
    part = part.transpose(0, 2, 1)
    # hole part: (xp|yl) = ooov[y][l][x][p]; t_lz^{qr} = t2[l][z][q][r]
    hole = np.tensordot(ooov[:, :, :, p], t2[:, :, q, r], axes=([1], [0]))  # [y][x][z]
    hole = hole.transpose(1, 0, 2)
    return part - hole


def w_occ_tensor(a, b, c, t2, ovvv, ooov):
    """W^{ijk} for one virtual triple: the six-fold pair permutation of X."""
    x = lambda p, q, r: x_term_fixed_virtuals(p, q, r, t2, ovvv, ooov)
    w = x(a, b, c).copy()                           # X^{abc}(i,j,k)
    w += x(a, c, b).transpose(0, 2, 1)              # X^{acb}(i,k,j)
    w += x(b, a, c).transpose(1, 0, 2)              # X^{bac}(j,i,k)
    w += np.einsum("jki->ijk", x(b, c, a))          # X^{bca}(j,k,i)
    w += np.einsum("kij->ijk", x(c, a, b))          # X^{cab}(k,i,j)
    w += np.einsum("kji->ijk", x(c, b, a))          # X^{cba}(k,j,i)
    return w


def v_occ_tensor(a, b, c, w, t1, ovov, t2=None, fock_ov=None):
    """V^{ijk} = W^{ijk} + t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb) [+ f_ov terms]."""
    v = w.copy()
    v += t1[:, a][:, None, None] * ovov[:, b, :, c][None, :, :]
    v += t1[:, b][None, :, None] * ovov[:, a, :, c][:, None, :]
    v += t1[:, c][None, None, :] * ovov[:, a, :, b][:, :, None]
    if fock_ov is not None:
        v += fock_ov[:, a][:, None, None] * t2[:, :, b, c][None, :, :]
        v += fock_ov[:, b][None, :, None] * t2[:, :, a, c][:, None, :]
        v += fock_ov[:, c][None, None, :] * t2[:, :, a, b][:, :, None]
    return v


def z_occ_tensor(a, b, c, v, eps_o, eps_v):
    """Z^{ijk} = [4V^{ijk} + V^{jki} + V^{kij} - 2V^{ikj} - 2V^{jik} - 2V^{kji}] / D^{ijk}."""
    num = (4.0 * v
           + np.einsum("jki->ijk", v)
           + np.einsum("kij->ijk", v)
           - 2.0 * np.einsum("ikj->ijk", v)
           - 2.0 * np.einsum("jik->ijk", v)
           - 2.0 * np.einsum("kji->ijk", v))
    d = (eps_o[:, None, None] + eps_o[None, :, None] + eps_o[None, None, :]
         - eps_v[a] - eps_v[b] - eps_v[c])
    return num / d


def virtual_triple_energy(a, b, c, m, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, fock_ov=None):
    """e_abc = (m/3) sum_ijk W^{ijk} Z^{ijk} for one unique virtual triple."""
    w = w_occ_tensor(a, b, c, t2, ovvv, ooov)
    v = v_occ_tensor(a, b, c, w, t1, ovov, t2, fock_ov)
    z = z_occ_tensor(a, b, c, v, eps_o, eps_v)
    return (m / 3.0) * float(np.sum(w * z))


def t_energy_virtual_loop(eps_o, eps_v, t1, t2, ovvv, ooov, ovov, return_triples=False, fock_ov=None):
    """E_T as the exactly rounded sum (math.fsum) of e_abc over unique virtual triples."""
    nvir = t1.shape[1]
    terms = [virtual_triple_energy(a, b, c, m, eps_o, eps_v, t1, t2, ovvv, ooov, ovov, fock_ov)
             for (a, b, c, m) in virtual_triple_table(nvir)]
    e = math.fsum(terms)
    if return_triples:
        return e, terms
    return e
