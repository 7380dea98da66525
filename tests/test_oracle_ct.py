"""Pins of the oracle's CT-to-phantom mapping (Sec. 2.1, after Schneider et al.
2000) against facts that do not come from the oracle itself: exact node values,
a calibration whose arithmetic is exact, numpy's own linear interpolation, the
clamping and bin rules checked by a plain loop, and the shape of the library."""
import numpy as np
import pytest

from oracle import ct


def _map(W):
    return W.ct_calibration()


def test_density_at_nodes_is_the_node_density(W):
    m = _map(W)
    for h, r in zip(m["hu"], m["rho"]):
        assert ct.density(np.array([h]), m["hu"], m["rho"])[0] == np.float32(r)


def test_exact_calibration_line():
    """Nodes (-1024, 1) and (1024, 3): the slope 2^-10 is exact, so every density
    is 1 + (h + 1024) / 1024 exactly (before the one rounding to FP32)."""
    h = np.arange(-1024, 1025, dtype=np.int16)
    got = ct.density(h, [-1024.0, 1024.0], [1.0, 3.0])
    want = (1.0 + (h.astype(np.float64) + 1024.0) / 1024.0).astype(np.float32)
    assert np.array_equal(got, want)


def test_agrees_with_numpy_interp(W):
    """numpy's np.interp (its own implementation) within one FP32 ulp on every
    HU value of the int16 CT range."""
    m = _map(W)
    h = np.arange(-1024, 3072, dtype=np.int16)
    got = ct.density(h, m["hu"], m["rho"])
    ref = np.interp(h.astype(np.float64), m["hu"], m["rho"]).astype(np.float32)
    ulp = np.spacing(np.maximum(np.abs(ref), np.float32(1e-30)))
    assert np.all(np.abs(got - ref) <= ulp)
    # monotone where the calibration is
    assert np.all(np.diff(got) >= 0)


def test_clamped_outside_the_nodes():
    H, P = [-500.0, 0.0, 500.0], [0.5, 1.0, 1.5]
    h = np.array([-32768, -1000, -501, -500, 500, 501, 3000, 32767], dtype=np.int16)
    got = ct.density(h, H, P)
    assert list(got[:4]) == [np.float32(0.5)] * 4
    assert list(got[4:]) == [np.float32(1.5)] * 4


def test_material_bins_by_a_plain_loop(W):
    m = _map(W)
    rng = np.random.default_rng(3)
    h = rng.integers(-1024, 3072, 4000).astype(np.int16)
    # every bin bound and its neighbours
    bounds = [u for u in m["upper"] if np.isfinite(u)]
    h = np.concatenate([h, np.array([b + d for b in bounds for d in (-1, 0, 1)], np.int16)])
    got = ct.material(h, m["upper"], m["material"])
    for v, g in zip(h, got):
        b = 0
        while b < len(m["material"]) - 1 and not (float(v) < m["upper"][b]):
            b += 1
        assert g == m["material"][b], int(v)
    # h exactly on a bound belongs to the next bin
    assert ct.material(np.array([-120], np.int16), m["upper"], m["material"])[0] == 3


def test_calibration_covers_the_library(W):
    m = _map(W)
    assert sorted(m["material"]) == list(range(len(W.MATERIALS_16)))
    assert np.all(np.diff(m["hu"]) > 0) and np.all(np.diff(m["rho"]) > 0)
    assert np.all(np.diff(m["upper"]) > 0)


def test_phantom_of_a_ct_volume(W):
    hu = W.ct_volume((20, 24, 24), 0.5, seed=4)
    ph = ct.phantom(hu, (0.5, 0.5, 0.5), W.MATERIALS_16, _map(W))
    assert ph["density"].shape == hu.shape and ph["density"].dtype == np.float32
    assert ph["material"].dtype == np.uint8 and ph["material"].max() < 16
    assert np.all(ph["density"] > 0)
    # air outside the body, lung inside: both present
    assert {7, 1} <= set(np.unique(ph["material"]).tolist())


@pytest.mark.parametrize("h", [-1000, -120, 0, 100, 1600])
def test_transport_phantom_from_ct_runs_in_the_oracle(orc, W, h):
    """A uniform CT volume maps to a uniform phantom the oracle transports with
    a closed energy ledger."""
    hu = np.full((10, 8, 8), h, np.int16)
    ph = ct.phantom(hu, (0.5, 0.5, 0.5), W.MATERIALS_16, _map(W))
    src = W.photon_beam((1.0, 1.0), (2.0, 2.0), mono_E=2.0, parallel=True)
    _, _, c = orc.run(ph, src, 200, seed=1, threads=1)
    assert abs(c["E_incident"] - c["E_deposited"] - c["E_escaped"]) < 1e-9 * c["E_incident"]
