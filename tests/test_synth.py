"""The seeded input generator: determinism and the symmetries its recipe
promises (the (T) tests and the benchmark rely on them)."""
import numpy as np

from synth import direct_sum_inputs, draw_factors, make_df_inputs, make_inputs, serving_stream


def test_same_seed_same_inputs_other_seed_other_inputs():
    a, b, c = make_inputs(4, 11, 30, 5), make_inputs(4, 11, 30, 5), make_inputs(4, 11, 30, 6)
    for x, y, z in zip(a.arrays(), b.arrays(), c.arrays()):
        assert np.array_equal(x, y)
    assert not np.array_equal(a.ovvv, c.ovvv)


def test_factor_and_integral_symmetries():
    o, v = 4, 9
    bq, eps_o, eps_v, t1 = draw_factors(o, v, 25, 2)
    assert np.array_equal(bq, bq.transpose(0, 2, 1))  # B[Q, p, q] = B[Q, q, p]
    x = make_inputs(o, v, 25, 2)
    # (ia|bc) = (ia|cb); (ia|jb) = (jb|ia); (jl|ia) = (lj|ia)
    assert np.allclose(x.ovvv, x.ovvv.transpose(0, 1, 3, 2), rtol=0, atol=1e-15)
    assert np.allclose(x.ovov, x.ovov.transpose(2, 3, 0, 1), rtol=0, atol=1e-15)
    assert np.allclose(x.ooov, x.ooov.transpose(1, 0, 2, 3), rtol=0, atol=1e-15)
    # t_ij^ab = t_ji^ba (MP1 amplitudes)
    assert np.allclose(x.t2, x.t2.transpose(1, 0, 3, 2), rtol=0, atol=1e-15)


def test_orbital_energies_sorted_with_a_gap():
    for seed in range(5):
        x = make_inputs(5, 20, 40, seed)
        assert np.all(np.diff(x.eps_o) >= 0) and np.all(np.diff(x.eps_v) >= 0)
        assert x.eps_o.max() < x.eps_v.min()


def test_df_inputs_reproduce_the_integrals():
    o, v, q, seed = 3, 7, 20, 4
    eps_o, eps_v, t1, t2, b_ov, b_vv, ooov, ovov = make_df_inputs(o, v, q, seed)
    x = make_inputs(o, v, q, seed)
    ovvv = np.einsum("Qia,Qbc->iabc", b_ov, b_vv)
    assert np.allclose(ovvv, x.ovvv, rtol=0, atol=1e-14)
    assert np.array_equal(t2, x.t2) and np.array_equal(ovov, x.ovov)


def test_direct_sum_keeps_each_fragment():
    shapes = [(2, 5, 9, 1), (3, 4, 8, 2)]
    eps_o, eps_v, t1, t2, ovvv, ooov, ovov = direct_sum_inputs(shapes)
    a, b = make_inputs(*shapes[0]), make_inputs(*shapes[1])
    assert np.array_equal(eps_o, np.concatenate([a.eps_o, b.eps_o]))
    assert np.allclose(ovvv[:2, :5, :5, :5], a.ovvv, rtol=0, atol=1e-15)
    assert np.allclose(ovvv[2:, 5:, 5:, 5:], b.ovvv, rtol=0, atol=1e-15)
    assert np.all(ovvv[:2, 5:, :, :] == 0) and np.all(t1[:2, 5:] == 0)


def test_serving_stream_shapes():
    s = serving_stream(256)
    assert len(s) == 256
    for r in s:
        assert 8 <= r["nocc"] <= 40
        assert 6 * r["nocc"] - 1 <= r["nvir"] <= 10 * r["nocc"] + 1
        assert r["naux"] == round(3.3 * (r["nocc"] + r["nvir"]))
    assert serving_stream(16) == serving_stream(256)[:16]


def test_input_summary_tolerates_rounding_only():
    """The stored-input summary matches the same draw with the integrals
    perturbed in the last bits (as another machine's BLAS rounds them), and
    rejects another seed, a transposed array and a one-element change."""
    import dataclasses

    import numpy as np

    from synth import input_summary, make_inputs, summary_matches
    x = make_inputs(6, 40, 100, 3)
    ref = input_summary(x)
    assert summary_matches(ref, x)
    ulp = dataclasses.replace(x, ovvv=x.ovvv * (1.0 + 2.0 ** -52 * np.sign(np.sin(np.arange(x.ovvv.size)))
                                                .reshape(x.ovvv.shape)))
    assert summary_matches(ref, ulp)
    assert not summary_matches(ref, make_inputs(6, 40, 100, 4))
    tr = dataclasses.replace(x, ovov=np.ascontiguousarray(x.ovov.transpose(0, 3, 2, 1)))
    assert not summary_matches(ref, tr)
    one = x.t2.copy()
    one.reshape(-1)[0] += 1e-6
    assert not summary_matches(ref, dataclasses.replace(x, t2=one))
