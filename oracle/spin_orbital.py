"""Brute-force spin-orbital (T) energy for tiny systems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the textbook definition of the (T) correction (Raghavachari,
Trucks, Pople & Head-Gordon 1989; written in spin orbitals as in Crawford &
Schaefer, Rev. Comp. Chem. 14, 2000), evaluated with full rank-6 tensors.
It shares nothing with the closed-shell loop except the inputs, and it is
what pins that loop (signs, coefficients, weights and which integral goes
where).

Spin orbitals P = (p, s), s in {alpha, beta}; index 2p + s.
  <pq||rs> = <pq|rs> - <pq|sr>,   <pq|rs> = (pr|qs) d(s_p,s_r) d(s_q,s_s)
  t_I^A     = t_i^a d(s_I, s_A)
  t_IJ^AB   = t_ij^ab d(s_I,s_A) d(s_J,s_B) - t_ij^ba d(s_I,s_B) d(s_J,s_A)
  D_IJK^ABC = f_I + f_J + f_K - f_A - f_B - f_C
  D t(c)    = P(I/JK) P(A/BC) [ sum_E t_JK^AE <EI||BC> - sum_M t_IM^BC <MA||JK> ]
  D t(d)    = P(I/JK) P(A/BC) [ t_I^A <JK||BC> + f_IA t_JK^BC ]
              (f_IA = f_ia d(s_I,s_A): the occupied-virtual Fock block of a
              non-canonical reference with diagonal oo and vv blocks; zero,
              and the term absent, for canonical HF)
  P(I/JK) f(IJK) = f(IJK) - f(JIK) - f(KJI)
  E_T       = (1/36) sum t(c) D (t(c) + t(d))

The spatial integrals come from the same arrays the closed-shell path
takes: (eb|ic) = ovvv[i][c][e][b], (mj|ak) = ooov[m][j][k][a],
(jb|kc) = ovov[j][b][k][c].  Size: (2o)^3 (2v)^3 doubles, so keep
o <= 4 and v <= 6.
"""
from __future__ import annotations

import numpy as np

__all__ = ["spinorb_t_energy"]


def _spin_delta(n):
    """s[P] = spin of spin orbital P = 2p + s."""
    return np.tile(np.array([0, 1]), n)


def _spatial(n):
    return np.repeat(np.arange(n), 2)


def _p_occ(t):
    """P(I/JK) on the first three axes: f(IJK) - f(JIK) - f(KJI)."""
    return (t - np.einsum("JIKabc->IJKabc", t) - np.einsum("KJIabc->IJKabc", t))


def _p_vir(t):
    """P(A/BC) on the last three axes."""
    return (t - np.einsum("ijkBAC->ijkABC", t) - np.einsum("ijkCBA->ijkABC", t))


def spinorb_t_energy(eps_o, eps_v, t1, t2, ovvv, ooov, ovov, fock_ov=None):
    """E_T from the spin-orbital definition (tiny systems only); fock_ov[i][a]
    = f_ia adds the f_ov t2 part of the disconnected triples."""
    nocc, nvir = t1.shape
    so, sv = 2 * nocc, 2 * nvir
    if so * sv > 8 * 12 + 1e-9 and (so ** 3) * (sv ** 3) > 3.0e6:
        raise ValueError("spin-orbital brute force is for tiny systems only")
    o_sp, v_sp = _spatial(nocc), _spatial(nvir)
    o_s, v_s = _spin_delta(nocc), _spin_delta(nvir)

    def d(a, b):
        return (a[:, None] == b[None, :]).astype(np.float64)

    # amplitudes
    t1s = t1[o_sp][:, v_sp] * d(o_s, v_s)
    t2sp = t2[np.ix_(o_sp, o_sp, v_sp, v_sp)]
    t2sp_swap = t2[np.ix_(o_sp, o_sp, v_sp, v_sp)].transpose(0, 1, 3, 2)  # t_ij^ba at (I,J,A,B)
    same_ia = d(o_s, v_s)  # [I, A]
    t2s = (t2sp * same_ia[:, None, :, None] * same_ia[None, :, None, :]
           - t2sp_swap * same_ia[:, None, None, :] * same_ia[None, :, :, None])

    # <EI||BC> = (EB|IC) d(E,B) d(I,C) - (EC|IB) d(E,C) d(I,B);  (eb|ic) = ovvv[i][c][e][b]
    eb_ic = ovvv.transpose(2, 3, 0, 1)  # [e][b][i][c] = ovvv[i][c][e][b]
    g1 = eb_ic[np.ix_(v_sp, v_sp, o_sp, v_sp)]
    g1 = g1 * d(v_s, v_s)[:, :, None, None] * d(o_s, v_s)[None, None, :, :]   # (E,B),(I,C)
    g1 = g1.transpose(0, 2, 1, 3)  # -> [E, I, B, C]
    g_vovv = g1 - g1.transpose(0, 1, 3, 2)

    # <MA||JK> = (MJ|AK) d(M,J) d(A,K) - (MK|AJ) d(M,K) d(A,J); (mj|ak) = ooov[m][j][k][a]
    mj_ka = ooov[np.ix_(o_sp, o_sp, o_sp, v_sp)]  # [M, J, K, A]
    g2 = mj_ka * d(o_s, o_s)[:, :, None, None] * d(o_s, v_s)[None, None, :, :]  # (M,J),(K,A)
    g2 = g2.transpose(0, 3, 1, 2)  # -> [M, A, J, K]
    g_ovoo = g2 - g2.transpose(0, 1, 3, 2)

    # <JK||BC> = (JB|KC) d(J,B) d(K,C) - (JC|KB) d(J,C) d(K,B)
    jb_kc = ovov[np.ix_(o_sp, v_sp, o_sp, v_sp)]  # [J, B, K, C]
    g3 = jb_kc * d(o_s, v_s)[:, :, None, None] * d(o_s, v_s)[None, None, :, :]
    g3 = g3.transpose(0, 2, 1, 3)  # -> [J, K, B, C]
    g_oovv = g3 - g3.transpose(0, 1, 3, 2)

    fo = eps_o[o_sp]
    fv = eps_v[v_sp]
    dnm = (fo[:, None, None, None, None, None] + fo[None, :, None, None, None, None]
           + fo[None, None, :, None, None, None] - fv[None, None, None, :, None, None]
           - fv[None, None, None, None, :, None] - fv[None, None, None, None, None, :])

    conn = (np.einsum("JKAE,EIBC->IJKABC", t2s, g_vovv)
            - np.einsum("IMBC,MAJK->IJKABC", t2s, g_ovoo))
    tc = _p_vir(_p_occ(conn)) / dnm
    disc = np.einsum("IA,JKBC->IJKABC", t1s, g_oovv)
    if fock_ov is not None:
        fs = fock_ov[o_sp][:, v_sp] * d(o_s, v_s)
        disc = disc + np.einsum("IA,JKBC->IJKABC", fs, t2s)
    td = _p_vir(_p_occ(disc)) / dnm
    return float(np.sum(tc * dnm * (tc + td)) / 36.0)
