"""CPU-only checks of the HIP library's host side: it loads and exports every
symbol include/omc.h declares, it validates arguments before touching a device,
and its own closed-form table builder (independent of the oracle's) agrees with
the oracle's tables. No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def omc():
    from paper_1503_01722_amd import omc
    omc.lib()
    return omc


def header_functions():
    names = set()
    for h in ("omc.h", "omc_dn.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(omc_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol(omc):
    names = header_functions()
    assert len(names) >= 28
    L = omc.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(omc.EXPORTS)


def test_default_params(omc):
    p = omc.default_params()
    assert (p.Eabs_e, p.Eabs_g, p.Wcc, p.kc, p.dmax_s, p.f_E) == (0.2, 0.05, 0.05, 0.2, 0.5, 0.25)
    assert p.n_batches == 10 and p.parity_fp64 == 0 and p.block_size == 256
    # the fields after the launch shape (a layout mismatch would show here)
    assert (p.graph_depth, p.beamlet_group, p.sparse_threshold) == (0, 0, 0.0)
    assert p.straggler_lanes == 16 and p.electron_mode == 0 and p.table_mode == 0
    assert p.photon_mode == 0
    assert p.tally_copies == 1 and p.source_order == 0 and p.event_lanes == 12
    assert (p.queue_factor, p.timing, p.chunk_histories) == (6, 0, 0)


def _create(omc, dens, mat, mats, dims=(4, 4, 4), h=(0.5, 0.5, 0.5)):
    holders = [omc._MaterialHolder(m) for m in mats]
    arr = (omc.Material * max(1, len(holders)))(*[x.struct for x in holders])
    ctx = C.c_void_p()
    rc = omc.lib().omc_create(C.byref(ctx), *dims, *h,
                              np.ascontiguousarray(dens, np.float32).ctypes.data_as(
                                  C.POINTER(C.c_float)),
                              np.ascontiguousarray(mat, np.uint8).ctypes.data_as(
                                  C.POINTER(C.c_uint8)), arr, len(holders))
    return rc, ctx


def gpu_present():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_argument_validation(omc, W):
    good_d = np.ones(64, np.float32)
    good_m = np.zeros(64, np.uint8)
    mats = [W.WATER]
    cases = [
        (good_d, good_m, mats, (0, 4, 4), (0.5, 0.5, 0.5)),          # empty dimension
        (good_d, good_m, mats, (4, 4, 2000), (0.5, 0.5, 0.5)),       # too large
        (good_d, good_m, mats, (4, 4, 4), (0.5, -1.0, 0.5)),         # negative voxel
        (np.where(np.arange(64) == 5, np.nan, 1).astype(np.float32), good_m, mats, (4, 4, 4),
         (0.5, 0.5, 0.5)),                                           # NaN density
        (np.where(np.arange(64) == 5, 0, 1).astype(np.float32), good_m, mats, (4, 4, 4),
         (0.5, 0.5, 0.5)),                                           # zero density
        (good_d, np.full(64, 3, np.uint8), mats, (4, 4, 4), (0.5, 0.5, 0.5)),  # bad material id
        (good_d, good_m, [], (4, 4, 4), (0.5, 0.5, 0.5)),            # no materials
    ]
    for d, m, ms, dims, h in cases:
        rc, ctx = _create(omc, d, m, ms, dims, h)
        assert rc == omc.OMC_EINVAL and not ctx.value
        assert omc.lib().omc_last_error(None)
    bad_mat = dict(W.WATER, I_eV=-1.0)
    rc, _ = _create(omc, good_d, good_m, [bad_mat])
    assert rc == omc.OMC_EINVAL
    # NULL context everywhere
    L = omc.lib()
    assert L.omc_set_source(None, None) == omc.OMC_EINVAL
    assert L.omc_set_params(None, None) == omc.OMC_EINVAL
    assert L.omc_run(None, 10, 1, 0, None, None) == omc.OMC_EINVAL
    assert L.omc_get_counters(None, None) == omc.OMC_EINVAL
    assert L.omc_set_phantom_ct(None, None, 0, None) == omc.OMC_EINVAL
    assert L.omc_get_phantom(None, None, None) == omc.OMC_EINVAL
    # a library of more than OMC_MAX_MATERIALS (32) compositions
    rc, _ = _create(omc, good_d, good_m, [W.WATER] * 33)
    assert rc == omc.OMC_EINVAL
    assert L.omc_autotune(None, 1000, 1, None) == omc.OMC_EINVAL
    out = omc.SparseOut()
    out.nnz = 7  # zeroed by the call before it checks anything else
    assert L.omc_run_beamlets(None, None, 1, 1, 0, None, C.byref(out)) == omc.OMC_EINVAL
    assert out.nnz == 0 and not out.row_ptr
    L.omc_free_sparse(None)
    L.omc_free_sparse(C.byref(out))
    L.omc_destroy(None)
    # denoiser: invalid volume sides are rejected before any device call
    h = C.c_void_p()
    for dims in ((12, 16, 16), (16, 16, 4), (1024, 16, 16)):
        assert L.omc_dn_create(C.byref(h), *dims, 0) == omc.OMC_EINVAL and not h.value
    assert L.omc_dn_num_params(None, None) == omc.OMC_EINVAL
    assert L.omc_dn_forward(None, None, None, None, 1.0, None, None) == omc.OMC_EINVAL
    assert L.omc_dn_debug_layer(5, 8, 8, 8, 16, 0, 16, *([None] * 8)) == omc.OMC_EINVAL
    assert L.omc_dn_last_error(None)
    L.omc_dn_destroy(None)
    if not gpu_present():
        rc, ctx = _create(omc, good_d, good_m, mats)
        assert rc == omc.OMC_EDEVICE and not ctx.value
        out = np.zeros(4, np.uint32)
        assert L.omc_debug_philox(1, 0, 0, 0, 1, out.ctypes.data_as(
            C.POINTER(C.c_uint32))) == omc.OMC_EDEVICE


@pytest.mark.parametrize("name", ["WATER", "LUNG", "BONE"])
def test_host_tables_match_oracle(omc, orc, W, name):
    """Two independent implementations of the closed forms agree to 1e-12."""
    spec = getattr(W, name)
    for Wcc, kc in ((0.05, 0.2), (0.2, 0.05)):
        a = omc.host_tables(spec, Wcc, kc)
        b = orc.mat_tables(spec, Wcc, kc)
        for k in omc.TABLE_ROWS:
            np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=0, err_msg=k)


def test_host_ms_table_matches_oracle(omc, orc):
    a, b = omc.host_ms_table(), orc.ms_table()
    # m1(A) = 1 - 1/(3A) + ... loses log10(A) digits to cancellation where A is
    # large (x near 8, A near 1000), so two bisections stop up to ~1e-10 apart there
    np.testing.assert_allclose(a[:480], b[:480], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=0)


def test_host_tables_spot_values(omc, W):
    t = omc.host_tables(W.WATER)
    E = np.exp2(np.log2(0.01) + np.arange(512) * np.log2(2000.0) / 511)
    i = int(np.argmin(abs(E - 1.0)))
    assert t["muC"][i] == pytest.approx(0.0707 * (1 + 0.0), rel=0.02)
    assert np.all(np.diff(t["R"]) > 0) and t["R"][0] == 0.0
    assert np.all(t["sigHat"] == np.maximum.accumulate(t["sigM"] + t["sigB"]))


def test_struct_layouts_match_header(omc, tmp_path):
    """Every ctypes mirror of an include/omc.h struct has the header's size and
    field offsets (compiled and measured with the host C compiler)."""
    pairs = {"omc_material": omc.Material, "omc_source": omc.Source, "omc_params": omc.Params,
             "omc_counters": omc.Counters, "omc_timing": omc.Timing, "omc_beamlet": omc.Beamlet,
             "omc_sparse_out": omc.SparseOut}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "omc.h"', "int main(void){"]
    for cname, py in pairs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, py in pairs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])


def test_builtin_library_arguments(omc):
    """mats == NULL selects the built-in water/lung/bone library: n_mats must be
    0 or 3 (checked before any device call), and the material-count error names
    the real limit."""
    L = omc.lib()
    d = np.ones(64, np.float32)
    m = np.full(64, 2, np.uint8)
    ctx = C.c_void_p()
    args = (C.byref(ctx), 4, 4, 4, 0.5, 0.5, 0.5, d.ctypes.data_as(C.POINTER(C.c_float)),
            m.ctypes.data_as(C.POINTER(C.c_uint8)), None)
    assert L.omc_create(*args, 5) == omc.OMC_EINVAL and not ctx.value
    assert b"built-in" in L.omc_last_error(None)
    m3 = np.full(64, 3, np.uint8)  # id 3 is outside the built-in library
    assert L.omc_create(C.byref(ctx), 4, 4, 4, 0.5, 0.5, 0.5,
                        d.ctypes.data_as(C.POINTER(C.c_float)),
                        m3.ctypes.data_as(C.POINTER(C.c_uint8)), None, 0) == omc.OMC_EINVAL
    from paper_1503_01722_amd import workloads as W
    rc, _ = _create(omc, d, np.zeros(64, np.uint8), [W.WATER] * 33)
    assert rc == omc.OMC_EINVAL and b"1..32" in L.omc_last_error(None)
