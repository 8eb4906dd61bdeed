"""Host-side checks of the C ABI (no GPU needed).

The library loads, exports every function include/bqc.h declares, and the
argument checks that precede any device work return the documented codes.
"""
import ctypes
import os

import numpy as np
import pytest

import paper_2502_17963_amd as bqc
from paper_2502_17963_amd import binding
from synth import make_inputs


def test_library_exports_every_declared_function():
    L = bqc.lib()
    names = bqc.header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/bqc.h but not exported"


def test_version_and_counts():
    L = bqc.lib()
    assert L.bqc_version() >= 100
    for o in range(0, 9):
        expect = max(o * (o + 1) * (o + 2) // 6 - o, 0)
        assert bqc.num_triples(o) == expect
    assert bqc.footprint(0, 10) == -1 and bqc.footprint(3, 0) == -1
    assert bqc.footprint(4, 20, "fp64") > 0


def test_footprint_grows_with_size_and_shrinks_with_precision():
    f64 = bqc.footprint(32, 300, "fp64")
    f32 = bqc.footprint(32, 300, "fp32")
    assert f64 > 8 * 32 * 300 ** 3  # holds at least the FP64 (ia|bc)
    assert bqc.footprint(32, 320, "fp64") > f64
    assert f32 > 0


def test_footprint_of_formulations():
    L = bqc.lib()
    o, v = 32, 300
    base = L.bqc_t_footprint(o, v, 2)
    assert L.bqc_t_footprint_ex(o, v, 2, 0, 0) == base
    vir = bqc.footprint(o, v, "bf16x3", formulation="virtual")
    # the virtual loop adds transposes of t1 and (ia|jb) (o^2 v^2 doubles)
    assert vir - base >= 8 * (o * v) ** 2
    fock = bqc.footprint(o, v, "bf16x3", formulation="virtual", fock=True)
    assert fock - vir >= 8 * (o * v) ** 2  # and of t2 with an f_ov block
    assert bqc.footprint(o, v, "bf16x3", fock=True) - base == 8 * o * v + 256
    for args in [(0, v, 2, 0, 0), (o, 0, 2, 0, 0), (o, v, 9, 0, 0), (o, v, 2, 2, 0), (o, v, 3, 1, 0)]:
        assert L.bqc_t_footprint_ex(*args) == -1, args


def _call(o, v, arrays, E=True, precision=0, triple_range=(0, 0), formulation=0):
    ptrs = [None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrays]
    e = ctypes.c_double(123.0)
    opts = binding.TOpts()
    opts.precision = precision
    opts.formulation = formulation
    opts.triple_begin, opts.triple_end = triple_range
    rc = bqc.lib().bqc_t_energy_ex(o, v, *ptrs, ctypes.byref(opts), ctypes.byref(e) if E else None, None)
    return rc, e.value


def test_invalid_sizes_and_pointers():
    x = make_inputs(3, 5, 10, 0)
    arr = list(x.arrays())
    assert _call(0, 5, arr)[0] == binding.EINVAL
    assert _call(3, 0, arr)[0] == binding.EINVAL
    for k in range(7):
        bad = list(arr)
        bad[k] = None
        rc, e = _call(3, 5, bad)
        assert rc == binding.EINVAL and e == 123.0  # output untouched on error
    assert _call(3, 5, arr, E=False)[0] == binding.EINVAL
    assert _call(3, 5, arr, precision=7)[0] == binding.EINVAL
    assert "precision" in bqc.last_error()


def test_triple_range_checks():
    # o = 4: 16 unique triples; a share is [begin, end) with 0 <= begin < end <= 16
    x = make_inputs(4, 6, 12, 0)
    arr = list(x.arrays())
    assert bqc.num_triples(4) == 16
    for rng in [(1, 0), (-1, 3), (3, 3), (5, 2), (0, 17), (16, 17)]:
        rc, e = _call(4, 6, arr, triple_range=rng)
        assert rc == binding.EINVAL and e == 123.0, rng
        assert "triple range" in bqc.last_error()


def test_formulation_checks():
    x = make_inputs(4, 6, 12, 0)
    arr = list(x.arrays())
    for f in (-1, 2, 7):
        rc, e = _call(4, 6, arr, formulation=f)
        assert rc == binding.EINVAL and e == 123.0 and "formulation" in bqc.last_error()
    # the virtual-triple loop has no FP8 contraction
    rc, e = _call(4, 6, arr, precision=3, formulation=1)
    assert rc == binding.EINVAL and e == 123.0
    # its shares count virtual triples: nvir = 6 has 50 of them, nocc = 4 only 16
    assert bqc.num_triples(6) == 50
    for rng in [(0, 51), (50, 51), (3, 3)]:
        rc, e = _call(4, 6, arr, triple_range=rng, formulation=1)
        assert rc == binding.EINVAL and e == 123.0 and "triple range" in bqc.last_error(), rng
    # a share valid only for the virtual count passes the argument checks
    # (it then fails for want of a device here, or runs on one)
    rc, _ = _call(4, 6, arr, triple_range=(16, 50), formulation=1)
    assert rc != binding.EINVAL


def test_too_many_triples_rejected():
    # nvir = 2344 has 2.149e9 unique virtual triples, beyond what one solve indexes;
    # the check precedes any read of the large arrays
    o, v = 1, 2344
    assert bqc.num_triples(v) > 2**31 - 1 and bqc.num_triples(2343) <= 2**31 - 1
    eps_o, eps_v = np.array([-1.0]), np.linspace(0.1, 3.0, v)
    tiny = np.zeros(4)
    arr = [eps_o, eps_v, tiny, tiny, tiny, tiny, tiny]
    rc, e = _call(o, v, arr, formulation=1)
    assert rc == binding.EINVAL and e == 123.0 and "unique triples" in bqc.last_error()


def test_density_fitting_argument_checks():
    from synth import make_df_inputs
    a = [np.ascontiguousarray(x) for x in make_df_inputs(3, 5, 10, 0)]
    L = bqc.lib()

    def call(naux, arrays):
        ptrs = [None if x is None else x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for x in arrays]
        e = ctypes.c_double(123.0)
        opts = binding.TOpts()
        rc = L.bqc_t_energy_df(3, 5, naux, *ptrs, ctypes.byref(opts), ctypes.byref(e), None)
        return rc, e.value

    assert call(0, a) == (binding.EINVAL, 123.0)
    assert "naux" in bqc.last_error()
    for k in range(8):
        bad = list(a)
        bad[k] = None
        assert call(10, bad) == (binding.EINVAL, 123.0), k


def test_non_finite_fock_rejected():
    x = make_inputs(3, 5, 10, 0)
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in x.arrays()]
    f = np.zeros((3, 5))
    f[1, 2] = np.inf
    opts = binding.TOpts()
    opts.fock_ov = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    e = ctypes.c_double(123.0)
    rc = bqc.lib().bqc_t_energy_ex(3, 5, *ptrs, ctypes.byref(opts), ctypes.byref(e), None)
    assert rc == binding.EINVAL and e.value == 123.0
    assert "fock" in bqc.last_error()


def test_mp2_argument_checks():
    from synth import draw_factors
    b, eo, ev, _ = draw_factors(3, 5, 10, 0)
    b_ov = np.ascontiguousarray(b[:, :3, 3:])
    L = bqc.lib()
    P = ctypes.POINTER(ctypes.c_double)

    def call(o, v, naux, arrays, precision=0):
        ptrs = [None if a is None else a.ctypes.data_as(P) for a in arrays]
        opts = binding.TOpts()
        opts.precision = precision
        e = ctypes.c_double(123.0)
        return L.bqc_mp2_energy_df(o, v, naux, *ptrs, ctypes.byref(opts), ctypes.byref(e), None), e.value

    good = [eo, ev, b_ov]
    for args in [(0, 5, 10), (3, 0, 10), (3, 5, 0)]:
        assert call(*args, good) == (binding.EINVAL, 123.0)
    for k in range(3):
        bad = list(good)
        bad[k] = None
        assert call(3, 5, 10, bad) == (binding.EINVAL, 123.0)
    assert call(3, 5, 10, good, precision=2) == (binding.EINVAL, 123.0)
    assert "FP64" in bqc.last_error()


def test_gap_and_finiteness_checks():
    x = make_inputs(3, 5, 10, 0)
    eo = x.eps_o.copy()
    eo[-1] = x.eps_v[0]  # max occupied == min virtual: no gap
    rc, e = _call(3, 5, [eo, *x.arrays()[1:]])
    assert rc == binding.EINVAL and e == 123.0
    assert "gap" in bqc.last_error()
    ev = x.eps_v.copy()
    ev[2] = np.nan
    rc, _ = _call(3, 5, [x.eps_o, ev, *x.arrays()[2:]])
    assert rc == binding.EINVAL and "finite" in bqc.last_error()


def test_server_argument_checks():
    L = bqc.lib()
    out = ctypes.c_void_p()
    assert L.bqc_server_create(None, ctypes.byref(out)) == binding.EINVAL
    cfg = binding.ServerCfg()
    cfg.precision = 9
    assert L.bqc_server_create(ctypes.byref(cfg), ctypes.byref(out)) == binding.EINVAL
    assert L.bqc_server_destroy(None) == binding.EINVAL
    t = ctypes.c_uint64()
    assert L.bqc_t_poll(None, 1, None, None) == binding.EINVAL
    x = make_inputs(2, 3, 6, 0)
    ptrs = [a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in x.arrays()]
    assert L.bqc_t_submit(None, 2, 3, *ptrs, ctypes.byref(t)) == binding.EINVAL


# Offsets of the boundary's base fields (the first four options and the
# first six statistics), in the order and C layout the boundary fixes; the
# extension fields follow them.
_BASE_OPTS = [("precision", 0), ("device", 4), ("inputs_on_device", 8), ("stream", 16)]
_BASE_STATS = [("queue_s", 0), ("upload_s", 8), ("gpu_s", 16), ("total_s", 24), ("flops", 32),
               ("footprint_bytes", 40)]


def _c_layout(tmp_path):
    """offsetof / sizeof of every field of bqc_t_opts and bqc_t_stats, from a
    C program compiled against include/bqc.h."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    fields = {"bqc_t_opts": [f for f, _ in binding.TOpts._fields_],
              "bqc_t_stats": [f for f, _ in binding.TStats._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "bqc.h"', "int main(void) {"]
    for st, names in fields.items():
        lines.append(f'printf("{st} sizeof %zu\\n", sizeof({st}));')
        for n in names:
            lines.append(f'printf("{st} {n} %zu\\n", offsetof({st}, {n}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-I" + inc, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    lay = {}
    for line in out.splitlines():
        st, name, val = line.split()
        lay[(st, name)] = int(val)
    return lay


def test_struct_base_fields_lead_in_boundary_order(tmp_path):
    lay = _c_layout(tmp_path)
    for name, off in _BASE_OPTS:
        assert lay[("bqc_t_opts", name)] == off, name
    for name, off in _BASE_STATS:
        assert lay[("bqc_t_stats", name)] == off, name


def test_ctypes_structs_match_the_header(tmp_path):
    lay = _c_layout(tmp_path)
    for cls, st in ((binding.TOpts, "bqc_t_opts"), (binding.TStats, "bqc_t_stats")):
        assert ctypes.sizeof(cls) == lay[(st, "sizeof")]
        for name, _ in cls._fields_:
            assert getattr(cls, name).offset == lay[(st, name)], (st, name)


def test_noalloc_batch_query():
    """bqc_t_noalloc_batch: small shapes fit the 64 MiB array with the
    library's own batch size or a smaller one, large ones do not fit, and
    invalid arguments give -1."""
    import paper_2502_17963_amd as bqc
    bqc.lib()
    assert bqc.noalloc_batch(6, 30, "fp64") == 50       # every triple in one launch
    assert 1 <= bqc.noalloc_batch(10, 80, "bf16x3") < 210
    assert bqc.noalloc_batch(32, 300, "bf16x3") == 0     # (ia|bc) alone exceeds the array
    assert bqc.noalloc_batch(6, 30, "fp8", "virtual") == -1
    assert bqc.noalloc_batch(0, 30, "fp64") == -1


def test_batch_argument_checks():
    """bqc_t_energy_batch rejects bad arguments before any device work."""
    import ctypes

    import numpy as np

    import paper_2502_17963_amd as bqc
    from paper_2502_17963_amd.binding import Fragment, TOpts, TStats
    from synth import make_inputs
    L = bqc.lib()
    x = make_inputs(3, 5, 10, 0)
    arrs = [np.ascontiguousarray(a) for a in x.arrays()]
    dp = ctypes.POINTER(ctypes.c_double)

    def frag(o, v, a):
        f = Fragment()
        f.nocc, f.nvir = o, v
        for name, arr in zip(("eps_o", "eps_v", "t1", "t2", "ovvv", "ooov", "ovov"), a):
            setattr(f, name, arr.ctypes.data_as(dp))
        return f

    e = (ctypes.c_double * 4)()
    good = (Fragment * 2)(frag(3, 5, arrs), frag(3, 5, arrs))
    assert L.bqc_t_energy_batch(0, None, None, None, None) == 0
    assert L.bqc_t_energy_batch(-1, good, None, e, None) == -1
    assert L.bqc_t_energy_batch(2, None, None, e, None) == -1
    assert L.bqc_t_energy_batch(2, good, None, None, None) == -1
    bad = (Fragment * 2)(frag(3, 5, arrs), frag(0, 5, arrs))
    assert L.bqc_t_energy_batch(2, bad, None, e, None) == -1
    assert "fragment 1" in bqc.last_error()
    eo_bad = arrs[0].copy()
    eo_bad[0] = 5.0  # above every virtual energy: no gap
    gap = (Fragment * 2)(frag(3, 5, arrs), frag(3, 5, [eo_bad] + arrs[1:]))
    assert L.bqc_t_energy_batch(2, gap, None, e, None) == -1
    for field, val in [("formulation", 1), ("triple_end", 3), ("precision", 7)]:
        o = TOpts()
        setattr(o, field, val)
        assert L.bqc_t_energy_batch(2, good, ctypes.byref(o), e, ctypes.byref(TStats())) == -1, field
    assert bqc.batch_footprint([(6, 30), (4, 20)], "bf16x3") > bqc.batch_footprint([(6, 30)], "bf16x3") > 0
    assert bqc.batch_footprint([(0, 30)]) == -1
