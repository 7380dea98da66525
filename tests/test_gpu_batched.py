"""GPU tests of the batched path through the C ABI: the captured-graph
generation pipeline (with particles carried over between source chunks), the
batched-beamlet run with its compacted per-beamlet output, and the autotuner.

* The FP64 parity build reproduces the oracle's integer counters exactly in
  graph mode too, and a batched-beamlet run gives, beamlet by beamlet, the
  dose of the oracle's run of that beamlet alone (same seed and histories).
* Graph and host-driven generations transport the same particles: identical
  counters, dose equal up to FP64 summation order; a replayed graph picks up
  a new seed and history range.
* The full-size batched workload (512 beamlets on the 256 x 256 x 160 CT-like
  phantom) matches standalone runs of sampled beamlets.
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


def engine(omc, ph, src=None, **params):
    eng = omc.Engine(ph)
    if src is not None:
        eng.set_source(src)
    if params:
        eng.set_params(**params)
    return eng


def ints(c):
    return {k: c[k] for k in INT_COUNTERS}


# ------------------------------------------------------------ graph pipeline
@pytest.mark.parametrize("name,n,chunk,depth", [("water_e15", 3000, 700, 2),
                                                ("slab_small", 6000, 1500, 1),
                                                ("slab_small", 6000, 0, 12)])
def test_fp64_graph_parity_with_oracle(omc, orc, W, name, n, chunk, depth):
    """Graph mode with few generations per chunk (most particles carried into
    later chunks, the rest drained from the host): counters equal the
    oracle's."""
    if name == "water_e15":
        ph, src, _ = W.config("water_e15")
    else:
        ph = W.slab_phantom(32, 1.0)
        src = W.config("slab_6mv")[1]
    print(f"[fp64 graph] {name} n={n} chunk={chunk} depth={depth}", flush=True)
    eng = engine(omc, ph, src, parity_fp64=1, graph_depth=depth, chunk_histories=chunk,
                 queue_factor=8)
    d, _ = eng.run(n, seed=2, h0=5)
    c = eng.counters()
    eng.close()
    od, _, oc = orc.run(ph, src, n, seed=2, h0=5)
    report(name, iterations=c["iterations"], hwm_ph=c["queue_hwm_ph"], hwm_el=c["queue_hwm_el"])
    assert ints(c) == ints(oc)
    assert ledger_residual(c) < 1e-9
    dose_parity(d, None, od, None, ph["density"], tag=name)


def test_graph_and_host_driven_identical_fp32(omc, W):
    """FP32 production: graph replays with carry-over transport exactly the
    particles the host-driven loop does; a replay takes the new seed and h0."""
    ph = W.slab_phantom(64, 0.5)
    src = W.config("slab_6mv")[1]
    n = 400_000
    ref = engine(omc, ph, src)
    d0, _ = ref.run(n, seed=5, h0=100)
    c0 = ref.counters()
    d1, _ = ref.run(n, seed=6, h0=0)
    c1 = ref.counters()
    ref.close()
    eng = engine(omc, ph, src, graph_depth=2, chunk_histories=65_536)
    g0, _ = eng.run(n, seed=5, h0=100)   # captures
    cg0 = eng.counters()
    g1, _ = eng.run(n, seed=6, h0=0)     # replays with another seed and h0
    cg1 = eng.counters()
    g0b, _ = eng.run(n, seed=5, h0=100)  # and back
    cg0b = eng.counters()
    eng.close()
    report("graph", iterations=cg0["iterations"], host_iterations=c0["iterations"])
    assert ints(cg0) == ints(c0) and ints(cg0b) == ints(c0)
    assert ints(cg1) == ints(c1)
    assert ints(c0) != ints(c1)
    # every deposit (rounding residuals included) lands in the voxel and cell of
    # the particle that made it, so only the FP64 summation order differs
    for a, b in ((g0, d0), (g1, d1), (g0b, d0)):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * b.max())


def test_timed_fixed_depth_matches_graph(omc, W):
    """With timing on, the fixed-depth sequence runs eagerly with one HIP event
    pair per launch; it transports the same particles as the graph."""
    ph, src, _ = W.config("water_e15")
    eng = engine(omc, ph, src, graph_depth=4, chunk_histories=5000)
    eng.run(20_000, seed=1)
    c_graph = eng.counters()
    eng.set_params(timing=1)
    for _ in range(2):
        eng.run(20_000, seed=1)
        t = eng.timing()
        assert ints(eng.counters()) == ints(c_graph)
        assert t["launches"]["photon"] >= 16 and t["launches"]["electron"] >= 16
        assert t["launches"]["source"] == 4
        assert t["total_ms"]["electron"] > 0 and t["run_ms"] > 0
    eng.close()


# ------------------------------------------------------------------ beamlets
def _beam_set(W, ph, particle):
    nz, ny, nx = ph["shape"]
    hz, hy, hx = ph["voxel"]
    iso = (nx * hx / 2, ny * hy / 2, nz * hz / 2)
    spec = W.spectrum_6mv()
    out = []
    counts = [1, 7, 500, 1500, 2400, 1234]
    for k, (g, n) in enumerate(zip([0.0, 45.0, 90.0, 180.0, 270.0, 315.0], counts)):
        if particle == 0:
            src = (W.photon_beam((1.0, 1.0), (iso[0] + k - 2.5, iso[1]), spectrum=spec)
                   if k % 2 == 0 else
                   W.photon_beam((1.5, 0.5), (iso[0], iso[1] + 1.0), mono_E=2.0 + k))
        else:
            src = W.electron_beam(6.0 + 2 * k, (1.0, 1.0), (iso[0], iso[1]), parallel=False)
        src.update(z_field=iso[2], sx=iso[0], sy=iso[1], gantry_deg=g, iso_x=iso[0], iso_z=iso[2])
        out.append((src, n))
    h, beams = 0, []
    for src, n in out:
        beams.append((src, n, h))
        h += n
    return beams


@pytest.mark.parametrize("particle,group,depth", [(0, 0, 0), (0, 4, 2), (1, 0, 3), (1, 5, 0)])
def test_fp64_beamlets_match_oracle(omc, orc, W, particle, group, depth):
    """Every beamlet's dose equals the oracle's run of that beamlet alone, to
    FP32 output rounding; the run's counters equal the summed oracle counters."""
    ph = W.ellipsoid_phantom((40, 48, 48), 0.5, n_ell=6, seed=3)
    beams = _beam_set(W, ph, particle)
    print(f"[fp64 beamlets] particle={particle} group={group} depth={depth}", flush=True)
    eng = engine(omc, ph, parity_fp64=1, beamlet_group=group, graph_depth=depth,
                 chunk_histories=2000 if depth else 0, queue_factor=8)
    sp = eng.run_beamlets(beams, seed=4)
    c = eng.counters()
    eng.close()
    od, oc = orc.run_beamlets(ph, beams, seed=4)
    nvox = int(np.prod(ph["shape"]))
    assert ints(c) == ints(oc)
    assert ledger_residual(c) < 1e-9
    assert sp.row_ptr[0] == 0 and np.all(np.diff(sp.row_ptr.astype(np.int64)) >= 0)
    assert sp.nnz == int(sp.row_ptr[-1])
    for b, ref in enumerate(od):
        lo, hi = int(sp.row_ptr[b]), int(sp.row_ptr[b + 1])
        assert np.all(np.diff(sp.voxel[lo:hi].astype(np.int64)) > 0)
        g = sp.row(b, nvox).reshape(ph["shape"])
        sparse_parity(g, ref, tag=f"beamlet {b}")
        # every voxel with dose is present (threshold 0)
        assert np.array_equal(g > 0, ref.astype(np.float32) > 0)


def test_beamlets_threshold_and_device_output(omc, W):
    ph = W.ellipsoid_phantom((40, 48, 48), 0.5, n_ell=6, seed=3)
    beams = _beam_set(W, ph, 0)
    nvox = int(np.prod(ph["shape"]))
    eng = engine(omc, ph)
    full = eng.run_beamlets(beams, seed=4)
    c_full = eng.counters()
    eng.set_params(sparse_threshold=0.01)
    thr = eng.run_beamlets(beams, seed=4)
    c_thr = eng.counters()
    assert ints(c_thr) == ints(c_full)
    for b in range(len(beams)):
        dfull = full.row(b, nvox)
        dthr = thr.row(b, nvox)
        cut = 0.01 * dfull.max()
        keep = dfull > cut
        # same transport, so the same voxels pass (values differ by summation order)
        close = np.abs(dfull - cut) <= 1e-5 * cut
        assert np.array_equal((dthr > 0)[~close], keep[~close])
        np.testing.assert_allclose(dthr[keep & ~close], dfull[keep & ~close], rtol=1e-5)
    eng.set_params(sparse_threshold=0.0)
    dev = eng.run_beamlets(beams, seed=4, on_device=True)
    assert dev.on_device and dev.nnz == full.nnz
    assert np.array_equal(dev.row_ptr, full.row_ptr)
    dev.free()
    eng.close()


def test_beamlet_errors(omc, W):
    ph = W.water_phantom((8, 8, 8), 1.0)
    eng = engine(omc, ph)
    e = W.electron_beam(6.0, (1.0, 1.0), (4.0, 4.0))
    p = W.photon_beam((1.0, 1.0), (4.0, 4.0), mono_E=1.0)
    with pytest.raises(omc.OmcError) as ex:
        eng.run_beamlets([(e, 10, 0), (p, 10, 10)])
    assert ex.value.code == omc.OMC_EINVAL
    with pytest.raises(omc.OmcError) as ex:
        eng.run_beamlets([(e, 0, 0)])
    assert ex.value.code == omc.OMC_EINVAL
    with pytest.raises(omc.OmcError) as ex:
        eng.run_beamlets([(e, 10, 2**32 - 5)])
    assert ex.value.code == omc.OMC_EINVAL
    with pytest.raises(omc.OmcError) as ex:
        eng.run_beamlets([(dict(e, fx=-1.0), 10, 0)])
    assert ex.value.code == omc.OMC_EINVAL
    sp = eng.run_beamlets([(e, 10, 0)])
    assert sp.n_beamlets == 1 and sp.nnz > 0
    eng.close()


def test_autotune_keeps_physics(omc, W):
    """The tuned launch shape transports the same particles."""
    ph = W.slab_phantom(64, 0.5)
    src = W.config("slab_6mv")[1]
    eng = engine(omc, ph, src)
    eng.run(200_000, seed=3)
    c0 = eng.counters()
    best = eng.autotune(200_000, seed=9)
    report("autotune", **{k: best[k] for k in ("block_size", "blocks_per_cu", "chunk_histories",
                                               "graph_depth", "queue_factor")})
    assert best["block_size"] in (128, 256) and 1 <= best["blocks_per_cu"] <= 8
    assert 2 <= best["queue_factor"] <= 64
    eng.run(200_000, seed=3)
    assert ints(eng.counters()) == ints(c0)
    eng.close()


# ------------------------------------------------------- full-size workload
def test_full_size_beamlets_sampled(omc, W):
    """The batched workload at full size (512 beamlets, about 2.8e8 histories,
    256 x 256 x 160 phantom) in the launch shape the benchmark uses; three
    sampled beamlets equal standalone runs of the same histories (same
    particles, so equal to summation order and FP32 output rounding)."""
    ph = W.ellipsoid_phantom()
    beams = W.beamlet_job(ph)
    print(f"[full beamlets] {len(beams)} beamlets, {sum(n for _, n, _ in beams)} histories",
          flush=True)
    eng = engine(omc, ph, graph_depth=W.BEAMLET_GRAPH_DEPTH, chunk_histories=W.BEAMLET_CHUNK,
                 blocks_per_cu=W.BEAMLET_BLOCKS_PER_CU)
    sp = eng.run_beamlets(beams, seed=1)
    c = eng.counters()
    report("full", nnz=sp.nnz, iterations=c["iterations"], watchdog=c["watchdog"],
           hwm_ph=c["queue_hwm_ph"], hwm_el=c["queue_hwm_el"])
    assert ledger_residual(c) < 1e-9 and c["watchdog"] == 0
    nvox = int(np.prod(ph["shape"]))
    counts = np.array([n for _, n, _ in beams])
    for b in (int(np.argmin(counts)), len(beams) // 2, int(np.argmax(counts))):
        src, n, h0 = beams[b]
        one = engine(omc, ph, src, n_batches=1)
        d, _ = one.run(n, seed=1, h0=h0)
        one.close()
        g = sp.row(b, nvox)
        d = d.ravel()
        np.testing.assert_allclose(g, d.astype(np.float32), rtol=1e-5, atol=1e-7 * d.max())
    eng.close()


# ------------------------------------------------------ stragglers set aside
def test_fp64_set_aside_parity_with_oracle(omc, orc, W):
    """A generation large enough (several records per lane of a one-work-group-
    per-CU grid) moves its stragglers to the next generation with their exact
    stream position and step state: the counters still equal the oracle's,
    and equal a run that keeps them."""
    ph = W.slab_phantom(32, 1.0)
    src = W.config("slab_6mv")[1]
    n = 400_000
    print(f"[fp64 set-aside] slab 32^3 n={n}", flush=True)
    eng = engine(omc, ph, src, parity_fp64=1, blocks_per_cu=1, straggler_lanes=40)
    d, _ = eng.run(n, seed=8, h0=11)
    c = eng.counters()
    eng.set_params(straggler_lanes=0)
    d0, _ = eng.run(n, seed=8, h0=11)
    c0 = eng.counters()
    eng.close()
    report("set-aside", moved=c["set_aside"], iterations=c["iterations"],
           iterations_without=c0["iterations"])
    assert c["set_aside"] > 0 and c0["set_aside"] == 0
    assert ints(c) == ints(c0)
    od, _, oc = orc.run(ph, src, n, seed=8, h0=11)
    assert ints(c) == ints(oc)
    dose_parity(d, None, od, None, ph["density"], tag="set-aside")
    np.testing.assert_allclose(d, d0, rtol=1e-9, atol=1e-12 * d0.max())


def test_fp32_set_aside_electrons_and_graph(omc, W):
    """15 MeV electrons (long tracks, many deltas) in FP32, graph mode with
    carry-over, stragglers set aside or not: the same particles throughout."""
    ph, src, _ = W.config("water_e15")
    n = 300_000
    runs = []
    for lanes, depth in ((0, 0), (48, 0), (48, 3)):
        eng = engine(omc, ph, src, blocks_per_cu=1, straggler_lanes=lanes, graph_depth=depth)
        d, _ = eng.run(n, seed=3)
        runs.append((d, eng.counters()))
        eng.close()
    report("electrons", moved=[r[1]["set_aside"] for r in runs])
    assert runs[1][1]["set_aside"] > 0
    for d, c in runs[1:]:
        assert ints(c) == ints(runs[0][1])
        np.testing.assert_allclose(d, runs[0][0], rtol=1e-9, atol=1e-12 * d.max())
