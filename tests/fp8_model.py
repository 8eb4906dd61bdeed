"""CPU model of the FP8 contraction mode, for its parity gate.

Test infrastructure: a model of what the FP8 mode computes, written from the
format definitions, not from the library's code.  Each contraction factor is
quantised as the mode stores it:

  * per row and per block of 32 consecutive contraction elements, a shared
    power-of-two scale 2^e with e = ceil(log2(amax / 448)) (the smallest
    power of two that brings the block's largest magnitude to at most 448,
    the largest finite OCP FP8 e4m3 value; stored as an E8M0 byte e + 127,
    e clamped to [-127, 127], e = -127 for an all-zero block);
  * every element as the e4m3 value nearest to x 2^-e (ties to even):
    normal numbers (1 + m/8) 2^E with E in [-6, 8] and m in 0..7 (448 =
    1.75 * 2^8 at the top), subnormals m 2^-9, m in 0..7.

The products of e4m3 values and their sums are then taken exactly (FP64,
where the device accumulates in FP32, a relative difference of ~1e-7 that
is far below the quantisation error), and the energy is formed from the
quantised contractions exactly as the FP64 oracle forms it from exact ones
(singles term, denominator and sums in FP64 from the unquantised inputs).

The contraction index of each factor, along which the 32-blocks run:
  (Pu|yd) and t_Pq^ud along d;  -(Pu|ql) and t_lP^yu along l.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.closed_shell import triple_table, v_tensor, z_tensor

E4M3_MAX = 448.0
BLOCK = 32


def e4m3_round(y: np.ndarray) -> np.ndarray:
    """Nearest OCP e4m3 value of y (ties to even), |y| <= 448 assumed."""
    a = np.abs(y)
    out = np.zeros_like(a)
    sub = a < 2.0 ** -6
    out[sub] = np.round(a[sub] * 512.0) / 512.0  # subnormal step 2^-9 (0 .. 8 steps)
    nrm = ~sub & (a > 0)
    _, ex = np.frexp(a[nrm])                      # a = f 2^ex, f in [0.5, 1): exponent E = ex - 1
    step = np.ldexp(1.0, ex - 4)                  # 3 mantissa bits: 2^(E - 3)
    q = np.round(a[nrm] / step) * step
    out[nrm] = np.minimum(q, E4M3_MAX)
    return np.copysign(out, y)


def block_exponents(amax: np.ndarray) -> np.ndarray:
    """e = ceil(log2(amax / 448)), clamped to [-127, 127]; -127 for amax = 0."""
    e = np.full(amax.shape, -127.0)
    nz = amax > 0
    m, ex = np.frexp(amax[nz] / E4M3_MAX)
    e[nz] = np.where(m == 0.5, ex - 1, ex)
    return np.clip(e, -127, 127)


def quantise_last_axis(x: np.ndarray) -> np.ndarray:
    """FP8 value of every element of x, blocks of 32 along the last axis."""
    k = x.shape[-1]
    kp = -(-k // BLOCK) * BLOCK
    xp = np.zeros(x.shape[:-1] + (kp,))
    xp[..., :k] = x
    blocks = xp.reshape(x.shape[:-1] + (kp // BLOCK, BLOCK))
    e = block_exponents(np.max(np.abs(blocks), axis=-1))[..., None]
    q = e4m3_round(np.ldexp(blocks, -e.astype(np.int64))) * np.exp2(e)
    return q.reshape(xp.shape)[..., :k]


def quantised_factors(t2, ovvv, ooov):
    """The four factors as the FP8 mode holds them (FP64 arrays of e4m3 values
    times their block scales):
      qo[P][u][y][d]  = (Pu|yd)             blocks along d
      qt[P][q][u][d]  = t_Pq^ud             blocks along d
      qh[q][P][u][l]  = (Pu|ql) = ooov[q][l][P][u]     blocks along l
      ql[R][y][w][l]  = t_lR^yw = t2[l][R][y][w]       blocks along l"""
    qo = quantise_last_axis(ovvv)
    qt = quantise_last_axis(t2)
    qh = quantise_last_axis(np.ascontiguousarray(np.transpose(ooov, (0, 2, 3, 1))))
    ql = quantise_last_axis(np.ascontiguousarray(np.transpose(t2, (1, 2, 3, 0))))
    return qo, qt, qh, ql


def x_term_q(p, q, r, qo, qt, qh, ql):
    """X_pqr(x,y,z) = sum_d (px|yd) t_rq^zd - sum_l (px|ql) t_lr^yz from the
    quantised factors."""
    nvir = qo.shape[1]
    part = (qo[p].reshape(nvir * nvir, nvir) @ qt[r, q].T).reshape(nvir, nvir, nvir)
    hole = np.einsum("xl,yzl->xyz", qh[q, p], ql[r])
    return part - hole


def w_tensor_q(i, j, k, qf):
    w = x_term_q(i, j, k, *qf)
    w = w + np.einsum("acb->abc", x_term_q(i, k, j, *qf))
    w = w + np.einsum("bac->abc", x_term_q(j, i, k, *qf))
    w = w + np.einsum("bca->abc", x_term_q(j, k, i, *qf))
    w = w + np.einsum("cab->abc", x_term_q(k, i, j, *qf))
    w = w + np.einsum("cba->abc", x_term_q(k, j, i, *qf))
    return w


def t_energy_fp8(eps_o, eps_v, t1, t2, ovvv, ooov, ovov, return_triples=False):
    """E_T with FP8-quantised contraction factors (model of the FP8 mode)."""
    qf = quantised_factors(t2, ovvv, ooov)
    terms = []
    for (i, j, k, m) in triple_table(t1.shape[0]):
        w = w_tensor_q(i, j, k, qf)
        v = v_tensor(i, j, k, w, t1, ovov)
        z = z_tensor(i, j, k, v, eps_o, eps_v)
        terms.append((m / 3.0) * float(np.sum(w * z)))
    e = math.fsum(terms)
    return (e, terms) if return_triples else e
