"""GPU tests of the phase-space source (geometry 2: history h starts from record
h mod n of a list of particles on a plane, Sec. 2.3's alternative to the
analytic beam), through the C ABI against the FP64 CPU oracle.

* The FP64 parity build reproduces the oracle's integer counters exactly with
  photon and electron record lists (records cycled, some pointing away from
  the phantom), under a gantry rotation, with fixed electron steps, and in
  batched beamlets that mix phase-space and analytic sources.
* The FP32 build agrees with the FP64 build statistically on the full-size
  record list, and a record list drawn from the analytic point-source beam
  gives that beam's dose.
"""
import numpy as np
import pytest

from parity import INT_COUNTERS, dose_agreement, dose_parity, ledger_residual, sparse_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def omc():
    from paper_1503_01722_amd import omc
    omc.lib()
    return omc


def gpu_run(omc, ph, src, n, seed=1, h0=0, **params):
    eng = omc.Engine(ph)
    eng.set_source(src)
    if params:
        eng.set_params(**params)
    d, d2 = eng.run(n, seed=seed, h0=h0)
    c = eng.counters()
    eng.close()
    return d, d2, c


def report(tag, **kv):
    print(tag, " ".join(f"{k}={v}" for k, v in kv.items()), flush=True)


def ints(c):
    return {k: c[k] for k in INT_COUNTERS}


def _cases(W):
    out = {}
    ph = W.slab_phantom(64, 0.5)
    out["photons_slab"] = (ph, W.psf_source(W.phase_space(3000, seed=11, stray=0.05)), 7000, {})
    ph = W.water_phantom((32, 32, 32), 0.5)
    rec = W.phase_space(1000, particle=1, field=(2.0, 2.0), centre=(8.0, 8.0), seed=12,
                        stray=0.05)
    out["electrons_water"] = (ph, W.psf_source(rec, particle=1), 2500, {})
    out["electrons_fixed"] = (ph, W.psf_source(rec, particle=1), 2500, {"electron_mode": 1})
    ph = W.ellipsoid_phantom((40, 48, 48), 0.5, n_ell=6, seed=3)
    src = W.psf_source(W.phase_space(2000, field=(4.0, 4.0), centre=(12.0, 12.0), seed=13))
    src.update(gantry_deg=30.0, iso_x=12.0, iso_z=10.0)
    out["photons_gantry"] = (ph, src, 6000, {})
    out["one_record"] = (W.water_phantom((20, 20, 20), 0.5),
                         W.psf_source(np.array([[6.0, 5.0, 5.0, -0.5, 0.0, 0.0, 1.0, 0.0]],
                                               np.float32)), 2000, {})
    return out


CASES = ["photons_slab", "electrons_water", "electrons_fixed", "photons_gantry", "one_record"]


@pytest.mark.parametrize("name", CASES)
def test_fp64_phase_space_counters_identical(omc, orc, W, name):
    ph, src, n, params = _cases(W)[name]
    print(f"[fp64 phase space] {name} n={n} records={len(src['psf'])}", flush=True)
    d, d2, c = gpu_run(omc, ph, src, n, seed=2, h0=5, parity_fp64=1, **params)
    od, od2, oc = orc.run(ph, src, n, seed=2, h0=5, params=params)
    report(name, **{k: c[k] for k in ("el_steps", "ph_flights", "push_el", "push_ph")})
    mism = {k: (c[k], oc[k]) for k in INT_COUNTERS if c[k] != oc[k]}
    assert not mism, mism
    assert ledger_residual(c) < 1e-9
    for k in ("E_incident", "E_deposited", "E_escaped"):
        assert c[k] == pytest.approx(oc[k], rel=1e-9, abs=1e-9), k
    dose_parity(d, d2, od, od2, ph["density"], tag=name)


def test_fp64_phase_space_graph_mode(omc, orc, W):
    """Graph mode with chunks carried between generations reads the resident
    records the same way."""
    ph, src, n, _ = _cases(W)["photons_slab"]
    eng = omc.Engine(ph)
    eng.set_source(src)
    eng.set_params(parity_fp64=1, graph_depth=2, chunk_histories=1500)
    eng.run(n, seed=2, h0=5)
    c = eng.counters()
    # a second source on the same context replaces the resident records
    src2 = W.psf_source(W.phase_space(500, seed=21))
    eng.set_source(src2)
    eng.run(3000, seed=3)
    c2 = eng.counters()
    eng.close()
    _, _, oc = orc.run(ph, src, n, seed=2, h0=5)
    _, _, oc2 = orc.run(ph, src2, 3000, seed=3)
    assert ints(c) == ints(oc)
    assert ints(c2) == ints(oc2)


@pytest.mark.parametrize("depth", [0, 2])
def test_fp64_beamlets_with_phase_spaces(omc, orc, W, depth):
    """Batched beamlets mixing analytic sources and two record lists (one
    shared by two beamlets): every beamlet equals the oracle's run of it alone."""
    ph = W.ellipsoid_phantom((40, 48, 48), 0.5, n_ell=6, seed=3)
    ra = W.psf_source(W.phase_space(700, field=(2.0, 2.0), centre=(12.0, 12.0), seed=31))
    rb = W.psf_source(W.phase_space(300, particle=1, field=(1.0, 1.0), centre=(10.0, 14.0),
                                    seed=32), particle=1)
    rg = dict(ra, gantry_deg=90.0, iso_x=12.0, iso_z=10.0)
    an = W.photon_beam((1.0, 1.0), (12.0, 12.0), spectrum=W.spectrum_6mv())
    photons = [(ra, 900), (an, 400), (rg, 1200)]
    h, beams = 0, []
    for s, n in photons:
        beams.append((s, n, h))
        h += n
    print(f"[fp64 beamlets, phase space] depth={depth}", flush=True)
    eng = omc.Engine(ph)
    eng.set_params(parity_fp64=1, graph_depth=depth, chunk_histories=1000 if depth else 0,
                   queue_factor=8)
    sp = eng.run_beamlets(beams, seed=6)
    c = eng.counters()
    # electrons from a record list in a job of their own
    spe = eng.run_beamlets([(rb, 600, 0), (rb, 400, 600)], seed=6)
    ce = eng.counters()
    eng.close()
    od, oc = orc.run_beamlets(ph, beams, seed=6)
    ode, oce = orc.run_beamlets(ph, [(rb, 600, 0), (rb, 400, 600)], seed=6)
    assert ints(c) == ints(oc)
    assert ints(ce) == ints(oce)
    nvox = int(np.prod(ph["shape"]))
    for s, refs in ((sp, od), (spe, ode)):
        for b, ref in enumerate(refs):
            g = s.row(b, nvox).reshape(ph["shape"])
            sparse_parity(g, ref, tag=f"phase-space beamlet {b}")


def test_fp32_vs_fp64_phase_space(omc, W):
    """The bench's phase-space workload (2^20 records of 6 MV on the 128^3
    slab): the FP32 build against the FP64 build."""
    ph, src, _ = W.config("slab_6mv_psf")
    n = 4_000_000
    print(f"[fp32 vs fp64, phase space] n={n}", flush=True)
    a, a2, ca = gpu_run(omc, ph, src, n, seed=51)
    b, b2, cb = gpu_run(omc, ph, src, n, seed=52, parity_fp64=1)
    ref, _, _ = gpu_run(omc, ph, src, n, seed=53, parity_fp64=1)
    agr = dose_agreement(a, a2, b, b2, ref)
    report("slab_6mv_psf", **agr)
    assert agr["within2s"] > 0.90 and abs(agr["bias"]) < 0.003
    assert ledger_residual(ca) < 1e-9 and ca["watchdog"] == 0
    for k in ("ph_flights", "ph_compton", "el_moller", "push_el"):
        assert ca[k] / n == pytest.approx(cb[k] / n, rel=0.01), k


def test_phase_space_of_the_analytic_beam(omc, W):
    """Records drawn from the analytic 6 MV point-source beam (no angular
    spread, none pointing away) give the analytic beam's dose."""
    ph = W.slab_phantom(64, 0.5)
    field, centre = (6.0, 6.0), (16.0, 16.0)
    rec = W.phase_space(1 << 20, field=field, centre=centre, spread_deg=0.0, stray=0.0,
                        seed=61)
    an = W.photon_beam(field, centre, spectrum=W.spectrum_6mv())
    n = 1 << 20  # each record once: no latent variance from reused records
    print(f"[phase space vs analytic beam] n={n}", flush=True)
    a, a2, _ = gpu_run(omc, ph, W.psf_source(rec), n, seed=62)
    b, b2, _ = gpu_run(omc, ph, an, n, seed=63)
    ref, _, _ = gpu_run(omc, ph, an, n, seed=64)
    agr = dose_agreement(a, a2, b, b2, ref)
    report("psf_vs_analytic", **agr)
    assert agr["within2s"] > 0.90 and abs(agr["bias"]) < 0.003


# --------------------------------------------- records written by GPU code
def _device_records(n, seed):
    """A user source function on the GPU: particles drawn by torch kernels into
    a (n, 8) float32 device tensor (15 MeV-ish electrons and 6 MeV photons are
    not mixed: one particle type per source)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    r = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    r[:, 0] = 0.5 + 5.5 * torch.rand(n, generator=g, device="cuda")
    r[:, 1] = 14.0 + 4.0 * torch.rand(n, generator=g, device="cuda")
    r[:, 2] = 14.0 + 4.0 * torch.rand(n, generator=g, device="cuda")
    r[:, 3] = -0.5
    r[:, 4:6] = 0.05 * torch.randn((n, 2), generator=g, device="cuda")
    r[:, 6] = 1.0
    r[::41, 6] = -1.0  # some point away from the phantom
    torch.cuda.synchronize()
    return r


def test_fp64_device_records_parity(omc, orc, W):
    """Records a caller's GPU code wrote, read in place: counters equal the
    oracle's run of the same records copied to the host, and the dose equals
    the host-record path's."""
    ph = W.slab_phantom(64, 0.5)
    rec = _device_records(2500, seed=71)
    host = rec.cpu().numpy()
    n = 6000
    print(f"[fp64 device records] n={n} records={len(host)}", flush=True)
    d, d2, c = gpu_run(omc, ph, W.psf_source(rec), n, seed=7, h0=2, parity_fp64=1)
    hd, _, hc = gpu_run(omc, ph, W.psf_source(host), n, seed=7, h0=2, parity_fp64=1)
    od, _, oc = orc.run(ph, W.psf_source(host), n, seed=7, h0=2)
    report("device_records", **{k: c[k] for k in ("el_steps", "ph_flights", "push_el")})
    assert ints(c) == ints(oc) and ints(c) == ints(hc)
    dose_parity(d, None, od, None, ph["density"], tag="device records")
    scale = max(od.max(), 1e-300)
    np.testing.assert_allclose(d, hd, rtol=1e-12, atol=1e-15 * scale)


def test_device_records_graph_and_beamlets(omc, orc, W):
    """Device records in graph mode (FP32 against the host-record path, same
    counters) and in a beamlet job beside host records (FP64 against the
    oracle)."""
    ph = W.slab_phantom(64, 0.5)
    rec = _device_records(4000, seed=72)
    host = rec.cpu().numpy()
    runs = []
    for r in (rec, host):
        eng = omc.Engine(ph)
        eng.set_source(W.psf_source(r))
        eng.set_params(graph_depth=3, chunk_histories=20_000)
        d, _ = eng.run(100_000, seed=9)
        runs.append((d, ints(eng.counters())))
        eng.close()
    assert runs[0][1] == runs[1][1]
    np.testing.assert_allclose(runs[0][0], runs[1][0], rtol=1e-5, atol=1e-7 * runs[1][0].max())
    other = W.psf_source(W.phase_space(600, seed=73))
    beams = [(W.psf_source(rec), 700, 0), (other, 500, 700), (W.psf_source(rec), 300, 1200)]
    eng = omc.Engine(ph)
    eng.set_params(parity_fp64=1)
    sp = eng.run_beamlets(beams, seed=3)
    c = eng.counters()
    eng.close()
    hbeams = [(W.psf_source(host), 700, 0), (other, 500, 700), (W.psf_source(host), 300, 1200)]
    od, oc = orc.run_beamlets(ph, hbeams, seed=3)
    assert ints(c) == ints(oc)
    nvox = int(np.prod(ph["shape"]))
    for b, ref in enumerate(od):
        g = sp.row(b, nvox).reshape(ph["shape"])
        sparse_parity(g, ref, tag=f"device-record beamlet {b}")


def test_device_records_rejected(omc, W):
    """Bad device records and pointers are refused on the host or by the
    device check, before any transport kernel reads them; the context keeps
    its previous source."""
    import ctypes as C
    import torch
    ph = W.water_phantom((20, 20, 20), 0.5)
    eng = omc.Engine(ph)
    good = W.psf_source(W.phase_space(100, field=(4.0, 4.0), centre=(5.0, 5.0), seed=74))
    eng.set_source(good)
    bad = _device_records(1000, seed=75)
    bad[17, 0] = 0.0
    bad[903, 5] = float("nan")
    with pytest.raises(omc.OmcError) as e:
        eng.set_source(W.psf_source(bad))
    assert e.value.code == omc.OMC_EINVAL and "record 17:" in str(e.value)
    bad[17, 0] = 25.0
    with pytest.raises(omc.OmcError) as e:
        eng.set_source(W.psf_source(bad))
    assert "record 17:" in str(e.value)
    bad[17, 0] = 1.0
    with pytest.raises(omc.OmcError) as e:
        eng.set_source(W.psf_source(bad))
    assert "record 903:" in str(e.value)
    bad[903, 4:7] = 0.0
    with pytest.raises(omc.OmcError) as e:
        eng.set_source(W.psf_source(bad))
    assert "record 903:" in str(e.value)
    L = omc.lib()
    # more records than the allocation holds: refused by the range check
    t = _device_records(1000, seed=76)
    s, keep = omc._source_struct(W.psf_source(t))
    s.n_psf = 1 << 26
    assert L.omc_set_source(eng._h, C.byref(s)) == omc.OMC_EINVAL
    # host memory flagged as device memory: refused by the pointer check
    host = np.ascontiguousarray(t.cpu().numpy())
    s.n_psf = 1000
    s.psf = host.ctypes.data_as(C.POINTER(C.c_float))
    assert L.omc_set_source(eng._h, C.byref(s)) == omc.OMC_EINVAL
    s.psf_on_device = 2
    assert L.omc_set_source(eng._h, C.byref(s)) == omc.OMC_EINVAL
    # a beamlet with bad device records names the beamlet
    with pytest.raises(omc.OmcError) as e:
        eng.run_beamlets([(good, 10, 0), (W.psf_source(bad), 10, 10)])
    assert "beamlet 1" in str(e.value)
    # the previous source is still in place
    d, _ = eng.run(2000, seed=1)
    c = eng.counters()
    eng.close()
    assert d.sum() > 0 and c["E_incident"] > 0
    del keep
