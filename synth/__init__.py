"""Seeded synthetic inputs for the closed-shell (T) energy.

This module is shared by the oracle, the tests and the benchmark. It draws
random density-fitting factors and orbital energies and forms from them the
inputs the (T) step consumes: MO integrals in chemists' notation, MP1 doubles
amplitudes and random singles. It contains none of the (T) arithmetic itself.

Workload recipe (the paper benchmarks water clusters in cc-pVXZ bases, whose
geometries and converged amplitudes are not available here; these seeded
inputs of the same shape stand in for them):

* B[Q,p,q] = (X + X^T)/2 with X[Q,p,q] ~ N(0, 0.05^2), n = nocc + nvir
  orbitals (occupied first), Q over naux fitting functions;
* eps_o ~ U[-2, -0.3] sorted ascending, eps_v ~ U[0.1, 3] sorted ascending;
* t1 ~ N(0, 0.01^2);
* (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s]  (density-fitted integrals, the
  paper's section on mean-field methods factorises the ERIs this way);
* t2[i,j,a,b] = (ia|jb) / (eps_i + eps_j - eps_a - eps_b)  (MP1 amplitudes).

Draw order per seed (fixed; changing it changes every stored value):
X, eps_o, eps_v, t1, all from numpy.random.default_rng(seed).

Array layouts (row-major, last index fastest) are those of the C ABI:
  eps_o[nocc], eps_v[nvir], t1[nocc][nvir], t2[nocc][nocc][nvir][nvir],
  ovvv[i][a][b][c] = (ia|bc), ooov[j][l][i][a] = (jl|ia),
  ovov[i][a][j][b] = (ia|jb).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "TInputs",
    "draw_factors",
    "direct_sum_inputs",
    "make_inputs",
    "serving_stream",
    "CONFIGS",
]

# Workloads: (nocc, nvir, naux, seed).  "small" finishes in the oracle in
# well under a second; the others are the single-GPU measurement shapes.
CONFIGS = {
    "small": (6, 30, 120, 0),
    "large_fragment": (32, 300, 1000, 0),
    "precision_sweep": (24, 240, 800, 0),
    "largest_fragment": (48, 480, 1600, 0),
}


@dataclass
class TInputs:
    nocc: int
    nvir: int
    eps_o: np.ndarray
    eps_v: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    ovvv: np.ndarray
    ooov: np.ndarray
    ovov: np.ndarray

    def arrays(self):
        """The seven input arrays in ABI argument order."""
        return (self.eps_o, self.eps_v, self.t1, self.t2, self.ovvv, self.ooov, self.ovov)

    def nbytes(self) -> int:
        return sum(a.nbytes for a in self.arrays())


def draw_factors(nocc: int, nvir: int, naux: int, seed: int):
    """Draw (B, eps_o, eps_v, t1) in the fixed order."""
    if nocc < 1 or nvir < 1 or naux < 1:
        raise ValueError("nocc, nvir and naux must be positive")
    rng = np.random.default_rng(seed)
    n = nocc + nvir
    x = rng.normal(0.0, 0.05, (naux, n, n))
    b = 0.5 * (x + x.transpose(0, 2, 1))
    del x
    eps_o = np.sort(rng.uniform(-2.0, -0.3, nocc))
    eps_v = np.sort(rng.uniform(0.1, 3.0, nvir))
    t1 = rng.normal(0.0, 0.01, (nocc, nvir))
    return b, eps_o, eps_v, t1


def _integrals(b: np.ndarray, nocc: int):
    """ovvv, ooov, ovov from the factors B (FP64, BLAS products over Q)."""
    naux, n, _ = b.shape
    nvir = n - nocc
    b_oo = np.ascontiguousarray(b[:, :nocc, :nocc]).reshape(naux, nocc * nocc)
    b_ov = np.ascontiguousarray(b[:, :nocc, nocc:]).reshape(naux, nocc * nvir)
    b_vv = np.ascontiguousarray(b[:, nocc:, nocc:]).reshape(naux, nvir * nvir)
    ovvv = (b_ov.T @ b_vv).reshape(nocc, nvir, nvir, nvir)
    ooov = (b_oo.T @ b_ov).reshape(nocc, nocc, nocc, nvir)
    ovov = (b_ov.T @ b_ov).reshape(nocc, nvir, nocc, nvir)
    return ovvv, ooov, ovov


def make_inputs(nocc: int, nvir: int, naux: int, seed: int) -> TInputs:
    """Seeded FP64 inputs for one (T) solve (see the module docstring)."""
    b, eps_o, eps_v, t1 = draw_factors(nocc, nvir, naux, seed)
    ovvv, ooov, ovov = _integrals(b, nocc)
    del b
    denom = (eps_o[:, None, None, None] + eps_o[None, :, None, None]
             - eps_v[None, None, :, None] - eps_v[None, None, None, :])
    t2 = np.ascontiguousarray(ovov.transpose(0, 2, 1, 3)) / denom
    return TInputs(nocc, nvir, eps_o, eps_v, t1, t2,
                   np.ascontiguousarray(ovvv), np.ascontiguousarray(ooov),
                   np.ascontiguousarray(ovov))


def direct_sum_inputs(shapes):
    """Inputs of several non-interacting fragments as one system: each
    fragment (nocc, nvir, naux, seed) keeps the draw of make_inputs, its DF
    factors live on its own Q range and its own orbitals, and cross singles
    are zero.  Orbital order: the occupied orbitals of every fragment, then
    the virtuals of every fragment.  Returns the seven FP64 ABI arrays."""
    draws = [draw_factors(o, v, q, s) for (o, v, q, s) in shapes]
    no = sum(o for (o, _, _, _) in shapes)
    nv = sum(v for (_, v, _, _) in shapes)
    nq = sum(q for (_, _, q, _) in shapes)
    n = no + nv
    b = np.zeros((nq, n, n))
    t1 = np.zeros((no, nv))
    eps_o, eps_v = [], []
    q0, o0, v0 = 0, 0, 0
    for (o, v, q, _), (bf, eo, ev, t1f) in zip(shapes, draws):
        idx = list(range(o0, o0 + o)) + list(range(no + v0, no + v0 + v))
        b[np.ix_(range(q0, q0 + q), idx, idx)] = bf
        t1[o0:o0 + o, v0:v0 + v] = t1f
        eps_o.append(eo)
        eps_v.append(ev)
        q0, o0, v0 = q0 + q, o0 + o, v0 + v
    ovvv, ooov, ovov = _integrals(b, no)
    eps_o, eps_v = np.concatenate(eps_o), np.concatenate(eps_v)
    den = (eps_o[:, None, None, None] + eps_o[None, :, None, None]
           - eps_v[None, None, :, None] - eps_v[None, None, None, :])
    t2 = np.ascontiguousarray(ovov.transpose(0, 2, 1, 3)) / den
    return (eps_o, eps_v, t1, t2, np.ascontiguousarray(ovvv), np.ascontiguousarray(ooov),
            np.ascontiguousarray(ovov))


def make_df_inputs(nocc: int, nvir: int, naux: int, seed: int):
    """The inputs of make_inputs(nocc, nvir, naux, seed) with (ia|bc) replaced
    by its density-fitting factors: returns (eps_o, eps_v, t1, t2, b_ov, b_vv,
    ooov, ovov), b_ov[Q][i][a] = B[Q, i, nocc + a], b_vv[Q][b][c] = B[Q,
    nocc + b, nocc + c] of the same draw (so sum_Q b_ov b_vv is the ovvv of
    make_inputs up to the rounding of the product)."""
    b, eps_o, eps_v, t1 = draw_factors(nocc, nvir, naux, seed)
    x = make_inputs(nocc, nvir, naux, seed)
    b_ov = np.ascontiguousarray(b[:, :nocc, nocc:])
    b_vv = np.ascontiguousarray(b[:, nocc:, nocc:])
    return (x.eps_o, x.eps_v, x.t1, x.t2, b_ov, b_vv, x.ooov, x.ovov)


def make_mp2_inputs_device(nocc: int, nvir: int, naux: int, seed: int, device="cuda:0"):
    """Inputs of the density-fitted MP2 energy on a HIP device: (eps_o, eps_v,
    b_ov[naux][nocc][nvir]) with the distributions of make_inputs (orbital
    energies as there; b_ov = (X_ov + X_vo^T) / 2, X ~ N(0, 0.05^2), the
    occupied-virtual block of the symmetrised factor), drawn block-wise so
    that no (nocc + nvir)^2 factor is formed."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f64 = torch.float64
    x_ov = torch.randn((naux, nocc, nvir), generator=g, device=device, dtype=f64) * 0.05
    x_vo = torch.randn((naux, nvir, nocc), generator=g, device=device, dtype=f64) * 0.05
    b_ov = (0.5 * (x_ov + x_vo.transpose(1, 2))).contiguous()
    del x_ov, x_vo
    eps_o = torch.sort(torch.rand(nocc, generator=g, device=device, dtype=f64) * 1.7 - 2.0).values
    eps_v = torch.sort(torch.rand(nvir, generator=g, device=device, dtype=f64) * 2.9 + 0.1).values
    return eps_o.contiguous(), eps_v.contiguous(), b_ov


def serving_stream(n_requests: int = 256, seed: int = 4, rate: float | None = None):
    """Fragment shapes for the serving workload.

    nocc ~ U{8..40}, nvir = round(r * nocc) with r ~ U[6, 10],
    naux = round(3.3 * (nocc + nvir)); fragment f uses seed 10000 + f.
    Shapes come from default_rng(seed); arrival gaps come from a separate
    default_rng(seed + 1) stream as standard exponentials scaled by 1/rate,
    so the shapes do not depend on the rate.  Without a rate every request
    arrives at t = 0 (closed loop).  Returns a list of dicts with nocc, nvir,
    naux, seed, t_arrive.
    """
    rng = np.random.default_rng(seed)
    shapes = []
    for f in range(n_requests):
        nocc = int(rng.integers(8, 41))
        r = float(rng.uniform(6.0, 10.0))
        nvir = int(round(r * nocc))
        naux = int(round(3.3 * (nocc + nvir)))
        shapes.append(dict(nocc=nocc, nvir=nvir, naux=naux, seed=10000 + f))
    gaps = np.random.default_rng(seed + 1).standard_exponential(n_requests)
    t = 0.0
    for f, s in enumerate(shapes):
        if rate:
            t += float(gaps[f]) / rate
        s["t_arrive"] = t
    return shapes


def unique_triple_count(nocc: int) -> int:
    """Number of occupied triples i<=j<=k with not i=j=k (a counting fact)."""
    return nocc * (nocc + 1) * (nocc + 2) // 6 - nocc


def flops_alg(nocc: int, nvir: int) -> float:
    """Algorithmic flop count of one solve over unique triples.

    Six permuted contraction terms per triple, each 2 v^4 (particle) +
    2 o v^3 (hole) flops.
    """
    return 12.0 * unique_triple_count(nocc) * float(nvir) ** 3 * (nvir + nocc)


def _check() -> None:  # pragma: no cover - tiny self check
    x = make_inputs(2, 3, 4, 0)
    assert math.isfinite(float(x.t2.sum()))


def make_inputs_device(nocc: int, nvir: int, naux: int, seed: int, device="cuda:0", factors=False):
    """Same recipe as make_inputs, generated on a HIP device with torch.

    For the serving workload, whose 256 fragments hold ~1 TB of FP64 inputs in
    total: each fragment is generated on the GPU when it arrives.  The draws
    come from torch's device generator seeded with `seed`, so the values
    differ from make_inputs(…, seed) (a different random stream with the same
    distributions).  Returns the seven ABI arrays as contiguous FP64 tensors;
    with factors=True, (ia|bc) is not formed and the eight arrays of the
    density-fitting entry are returned instead: (eps_o, eps_v, t1, t2, b_ov,
    b_vv, ooov, ovov) with b_ov[Q][i][a], b_vv[Q][b][c].
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n = nocc + nvir
    f64 = torch.float64
    x = torch.randn((naux, n, n), generator=g, device=device, dtype=f64) * 0.05
    b = 0.5 * (x + x.transpose(1, 2))
    del x
    eps_o = torch.sort(torch.rand(nocc, generator=g, device=device, dtype=f64) * 1.7 - 2.0).values
    eps_v = torch.sort(torch.rand(nvir, generator=g, device=device, dtype=f64) * 2.9 + 0.1).values
    t1 = torch.randn((nocc, nvir), generator=g, device=device, dtype=f64) * 0.01
    b_oo = b[:, :nocc, :nocc].reshape(naux, nocc * nocc).t().contiguous()
    b_ov = b[:, :nocc, nocc:].reshape(naux, nocc * nvir)
    b_vv = b[:, nocc:, nocc:].reshape(naux, nvir * nvir).contiguous()
    b_ovt = b_ov.t().contiguous()
    ovvv = None if factors else (b_ovt @ b_vv).reshape(nocc, nvir, nvir, nvir)
    ooov = (b_oo @ b_ov.contiguous()).reshape(nocc, nocc, nocc, nvir)
    ovov = (b_ovt @ b_ov.contiguous()).reshape(nocc, nvir, nocc, nvir)
    f_ov = b_ov.reshape(naux, nocc, nvir).contiguous() if factors else None
    f_vv = b_vv.reshape(naux, nvir, nvir) if factors else None
    del b, b_oo, b_ov, b_vv, b_ovt
    denom = (eps_o[:, None, None, None] + eps_o[None, :, None, None]
             - eps_v[None, None, :, None] - eps_v[None, None, None, :])
    t2 = (ovov.permute(0, 2, 1, 3) / denom).contiguous()
    if factors:
        return tuple(a.contiguous() for a in (eps_o, eps_v, t1, t2, f_ov, f_vv, ooov, ovov))
    return tuple(a.contiguous() for a in (eps_o, eps_v, t1, t2, ovvv, ooov, ovov))


SUMMARY_ARRAYS = ("eps_o", "eps_v", "t1", "t2", "ovvv", "ooov", "ovov")


def input_summary(x) -> dict:
    """Identifies the inputs x a stored result was computed from: for each
    array, over a strided sample (every 4099th element), the sum, the sum of
    magnitudes and a sum weighted by (position mod 13) - 6 (which also sees
    a reordering).  The integrals are BLAS products over Q, whose rounding
    differs between machines in the last bits, so summaries are compared
    with summary_matches, not for equality."""
    out = {}
    for name in SUMMARY_ARRAYS:
        a = getattr(x, name).reshape(-1)[::4099]
        w = (np.arange(a.size) % 13) - 6.0
        out[name] = [float(a.sum()), float(np.abs(a).sum()), float(np.dot(w, a))]
    return out


def summary_matches(stored: dict, x, rel: float = 1e-12) -> bool:
    """True when the inputs x have the stored summary up to rounding: every
    sum within rel times six times the sample's sum of magnitudes (a
    different draw or layout changes them at order one)."""
    now = input_summary(x)
    for name in SUMMARY_ARRAYS:
        s0, m0, w0 = stored[name]
        s1, m1, w1 = now[name]
        tol = rel * 6.0 * max(m0, 1e-300)
        if abs(s0 - s1) > tol or abs(m0 - m1) > tol or abs(w0 - w1) > tol:
            return False
    return True
