"""GPU tests of the material library (Sec. 2.1: 16 materials built from their
compositions) through the C ABI against the FP64 CPU oracle.

* The device holds the tables of the materials present in the phantom only;
  a phantom that uses a few ids of a larger library (not contiguous) gives
  the oracle's counters exactly.
* All 16 materials present: the per-material tables are read from global
  memory (they no longer fit the LDS at the requested occupancy) and the FP64
  build reproduces the oracle's counters exactly.
* Where the tables live (LDS or global memory) does not change a result: the
  same build gives identical counters in both modes.
"""
import numpy as np
import pytest

from parity import INT_COUNTERS, dose_parity, ledger_residual, sparse_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def omc():
    from paper_1503_01722_amd import omc
    omc.lib()
    return omc


def report(tag, **kv):
    print(tag, " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def ints(c):
    return {k: c[k] for k in INT_COUNTERS}


def gpu_run(omc, ph, src, n, seed=1, h0=0, **params):
    eng = omc.Engine(ph)
    eng.set_source(src)
    if params:
        eng.set_params(**params)
    d, d2 = eng.run(n, seed=seed, h0=h0)
    c = eng.counters()
    eng.close()
    return d, d2, c


def _sparse_library_phantom(W):
    """Three ids (2, 9, 15) of the 16-material library in slabs along z."""
    ph = W.layered_phantom((36, 16, 16), 0.5, [(0.0, 6.0, 15, 1.0), (6.0, 12.0, 2, 1.85),
                                               (12.0, 19.0, 9, 1.09)])
    ph["materials"] = W.MATERIALS_16
    return ph


def _cases(W):
    ph16 = W.sixteen_material_phantom()
    sp = _sparse_library_phantom(W)
    return {
        "sixteen_photons": (ph16, W.photon_beam((4.0, 4.0), (4.0, 4.0),
                                                spectrum=W.spectrum_6mv()), 3000, {}),
        "sixteen_electrons": (ph16, W.electron_beam(15.0, (2.0, 2.0), (4.0, 4.0)), 1500, {}),
        "sixteen_fixed_steps": (ph16, W.electron_beam(15.0, (2.0, 2.0), (4.0, 4.0)), 1500,
                                {"electron_mode": 1}),
        "sparse_library_lds": (sp, W.photon_beam((4.0, 4.0), (4.0, 4.0), mono_E=8.0), 3000,
                               {"table_mode": 1}),
        "sparse_library_global": (sp, W.electron_beam(12.0, (2.0, 2.0), (4.0, 4.0)), 1500,
                                  {"table_mode": 2}),
    }


@pytest.mark.parametrize("name", ["sixteen_photons", "sixteen_electrons", "sixteen_fixed_steps",
                                  "sparse_library_lds", "sparse_library_global"])
def test_fp64_library_parity(omc, orc, W, name):
    ph, src, n, params = _cases(W)[name]
    print(f"[fp64 materials] {name} n={n} materials={len(ph['materials'])}", flush=True)
    d, d2, c = gpu_run(omc, ph, src, n, seed=3, h0=1, parity_fp64=1, **params)
    od, od2, oc = orc.run(ph, src, n, seed=3, h0=1, params=params)
    report(name, **{k: c[k] for k in ("el_steps", "ph_flights", "push_el")})
    mism = {k: (c[k], oc[k]) for k in INT_COUNTERS if c[k] != oc[k]}
    assert not mism, mism
    assert ledger_residual(c) < 1e-9
    dose_parity(d, d2, od, od2, ph["density"], tag=name)


@pytest.mark.parametrize("fp64,phantom", [(0, "eight"), (0, "sixteen"), (1, "eight")])
def test_table_modes_identical(omc, W, fp64, phantom):
    """Tables staged in LDS (table_mode 1) and read from global memory
    (table_mode 2): the same counters, the dose to summation order."""
    ph = W.eight_material_phantom() if phantom == "eight" else W.sixteen_material_phantom()
    src = W.photon_beam((4.0, 4.0), (4.0, 4.0), spectrum=W.spectrum_6mv())
    n = 200_000 if not fp64 else 20_000
    print(f"[table modes] {phantom} fp64={fp64} n={n}", flush=True)
    out = []
    for mode in (1, 2):
        eng = omc.Engine(ph)
        eng.set_source(src)
        eng.set_params(parity_fp64=fp64, table_mode=mode)
        d, _ = eng.run(n, seed=5)
        out.append((d, eng.counters(), eng.timing()["tables_global"]))
        eng.close()
    (a, ca, ga), (b, cb, gb) = out
    assert (ga, gb) == (0, 1)
    assert ints(ca) == ints(cb)
    np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * b.max())


def test_lds_tables_too_large_refused(omc, W):
    """Sixteen materials in FP64 do not fit a work-group's LDS: table_mode 1
    is refused, table_mode 0 reads them from global memory."""
    ph = W.sixteen_material_phantom()
    eng = omc.Engine(ph)
    eng.set_source(W.photon_beam((4.0, 4.0), (4.0, 4.0), mono_E=2.0))
    eng.set_params(parity_fp64=1, table_mode=1)
    with pytest.raises(omc.OmcError) as e:
        eng.run(100)
    assert e.value.code == omc.OMC_EUNSUP
    eng.set_params(parity_fp64=1, table_mode=0)
    d, _ = eng.run(100)
    eng.close()
    assert d.sum() > 0
    other = omc.Engine(ph)
    with pytest.raises(omc.OmcError):
        other.set_params(table_mode=3)
    other.close()


# ------------------------------------------------------- CT to phantom (Sec. 2.1)
def _ct_case(W):
    """A synthetic CT volume with every int16 value of the CT range (and the
    calibration's nodes and bin bounds) written into its first rows."""
    hu = W.ct_volume((24, 40, 48), 0.5, seed=2)
    ramp = np.arange(-1024, 3072, dtype=np.int16)
    flat = hu.reshape(-1)
    flat[: ramp.size] = ramp
    return hu


@pytest.mark.parametrize("on_device", [0, 1])
def test_ct_mapping_bit_exact(omc, W, on_device):
    """Densities (FP32 bits) and material ids of the device mapping equal the
    oracle's, for host and device HU input."""
    import torch
    from oracle import ct
    hu = _ct_case(W)
    m = W.ct_calibration()
    ref = ct.phantom(hu, (0.5, 0.5, 0.5), W.MATERIALS_16, m)
    src = torch.from_numpy(hu).cuda() if on_device else hu
    eng = omc.Engine({"shape": hu.shape, "voxel": (0.5, 0.5, 0.5), "materials": W.MATERIALS_16,
                      "hu": src, "ct_map": m})
    d, mat = eng.get_phantom()
    eng.close()
    assert np.array_equal(d.view(np.uint32), ref["density"].view(np.uint32))
    assert np.array_equal(mat, ref["material"])


def test_fp64_parity_on_a_ct_phantom(omc, orc, W):
    """Transport on the device-mapped CT phantom gives the oracle's counters on
    the oracle-mapped phantom."""
    from oracle import ct
    hu = W.ct_volume((24, 40, 48), 0.5, seed=5)
    m = W.ct_calibration()
    ref = ct.phantom(hu, (0.5, 0.5, 0.5), W.MATERIALS_16, m)
    src = W.photon_beam((4.0, 4.0), (12.0, 10.0), spectrum=W.spectrum_6mv())
    eng = omc.Engine({"shape": hu.shape, "voxel": (0.5, 0.5, 0.5), "materials": W.MATERIALS_16,
                      "hu": hu, "ct_map": m})
    eng.set_source(src)
    eng.set_params(parity_fp64=1)
    d, d2 = eng.run(3000, seed=6)
    c = eng.counters()
    eng.close()
    od, _, oc = orc.run(ref, src, 3000, seed=6)
    report("ct", n_mats=len(np.unique(ref["material"])),
           **{k: c[k] for k in ("el_steps", "ph_flights")})
    assert ints(c) == ints(oc)
    dose_parity(d, None, od, None, ref["density"], tag="ct")


def _hip_runtime():
    """The HIP runtime already loaded in this process (torch's), by its path."""
    import ctypes as C
    import torch  # noqa: F401  (loads the runtime)
    torch.zeros(1, device="cuda")
    for ln in open("/proc/self/maps"):
        if "libamdhip64" in ln:
            return C.CDLL(ln.split()[-1])
    raise RuntimeError("no HIP runtime loaded")


def test_ct_mapping_errors_leave_the_phantom(omc, W):
    import ctypes as C
    hu = _ct_case(W)
    m = W.ct_calibration()
    eng = omc.Engine({"shape": hu.shape, "voxel": (0.5, 0.5, 0.5), "materials": W.MATERIALS_16,
                      "hu": hu, "ct_map": m})
    before = eng.get_phantom()
    bad_maps = [dict(m, hu=m["hu"][::-1]),                      # nodes not increasing
                dict(m, rho=[0.0] + m["rho"][1:]),               # density 0
                dict(m, material=[16] + m["material"][1:]),      # id beyond the library
                dict(m, upper=[0.0] + m["upper"][1:]),           # bounds not increasing
                dict(m, hu=[0.0], rho=[1.0])]                    # one node
    for bad in bad_maps:
        with pytest.raises(omc.OmcError) as e:
            eng.set_phantom_ct(hu, bad)
        assert e.value.code == omc.OMC_EINVAL
    L = omc.lib()
    nodes = np.asarray(m["hu"], np.float64)
    rho = np.asarray(m["rho"], np.float64)
    up = np.asarray(m["upper"], np.float64)
    mats = np.asarray(m["material"], np.int32)
    cm = omc.CtMap(len(nodes), nodes.ctypes.data_as(C.POINTER(C.c_double)),
                   rho.ctypes.data_as(C.POINTER(C.c_double)), len(mats),
                   up.ctypes.data_as(C.POINTER(C.c_double)),
                   mats.ctypes.data_as(C.POINTER(C.c_int)))
    # a 1 KB device allocation of its own (torch's allocator would hand out a
    # slice of a larger segment): far too small for the volume, refused by the
    # range check before any kernel reads it
    hip = _hip_runtime()
    p = C.c_void_p()
    assert hip.hipMalloc(C.byref(p), C.c_size_t(1024)) == 0
    try:
        assert L.omc_set_phantom_ct(eng._h, p, 1, C.byref(cm)) == omc.OMC_EINVAL
    finally:
        hip.hipFree(p)
    # host memory flagged as device memory
    assert L.omc_set_phantom_ct(eng._h, hu.ctypes.data_as(C.c_void_p), 1, C.byref(cm)) == \
        omc.OMC_EINVAL
    after = eng.get_phantom()
    eng.close()
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])


def test_fp64_library_graph_beamlets_and_phantom_swap(omc, orc, W):
    """One context on the 16-material library: graph mode with tables in global
    memory, beamlets, then a new phantom with another set of materials (new
    slots, new tables, a new capture) - each against the oracle."""
    ph16 = W.sixteen_material_phantom()
    src = W.photon_beam((4.0, 4.0), (4.0, 4.0), spectrum=W.spectrum_6mv())
    eng = omc.Engine(ph16)
    eng.set_source(src)
    eng.set_params(parity_fp64=1, graph_depth=2, chunk_histories=1000)
    eng.run(2500, seed=8)
    c = eng.counters()
    _, _, oc = orc.run(ph16, src, 2500, seed=8)
    assert ints(c) == ints(oc)
    allb = [(src, 700, 0), (W.photon_beam((2.0, 2.0), (3.0, 5.0), mono_E=3.0), 400, 700)]
    sp = eng.run_beamlets(allb, seed=9)
    cb = eng.counters()
    od, ocb = orc.run_beamlets(ph16, allb, seed=9)
    assert ints(cb) == ints(ocb)
    nvox = int(np.prod(ph16["shape"]))
    for b, ref in enumerate(od):
        g = sp.row(b, nvox).reshape(ph16["shape"])
        sparse_parity(g, ref, tag=f"library beamlet {b}")
    # the same dimensions, three other library materials
    sp_ph = W.layered_phantom(ph16["shape"], 0.5, [(0.0, 8.0, 9, 1.09), (8.0, 14.0, 14, 1.03),
                                                   (14.0, 25.0, 2, 1.85)])
    sp_ph["materials"] = W.MATERIALS_16
    eng.set_phantom(sp_ph)
    d, _ = eng.run(2500, seed=10)
    c2 = eng.counters()
    eng.close()
    od2, _, oc2 = orc.run(sp_ph, src, 2500, seed=10)
    assert ints(c2) == ints(oc2)
    dose_parity(d, None, od2, None, sp_ph["density"], tag="phantom swap")


def test_builtin_library_equals_explicit(omc, orc, W):
    """A context created with mats == NULL holds the built-in water, lung and
    bone: the FP64 build gives the same event counters as a context given those
    compositions explicitly, and as the oracle."""
    ph = W.slab_phantom(32, 1.0)
    src = W.photon_beam((10.0, 10.0), (16.0, 16.0), spectrum=W.spectrum_6mv())
    n = 20_000
    builtin = dict(ph, materials=None)
    cs = []
    for p in (builtin, ph):
        eng = omc.Engine(p)
        eng.set_source(src)
        eng.set_params(parity_fp64=1)
        eng.run(n, seed=6)
        cs.append(ints(eng.counters()))
        eng.close()
    _, _, oc = orc.run(ph, src, n, seed=6)
    assert cs[0] == cs[1] == ints(oc)
