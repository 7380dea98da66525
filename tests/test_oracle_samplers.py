"""Pins for the oracle's samplers (CPU only): chi-square against analytic or
independently integrated distributions, and kinematic identities.

Samplers follow the paper's Sec. 2.1: Klein-Nishina for Compton, the energy
differential Moller and bremsstrahlung cross sections for hard events, and a
multiple-scattering angle for the random hinge.
"""
import numpy as np
import pytest
from scipy import integrate, stats

MC2 = 0.51099895
RE = 2.8179403262e-13


def chi2_pvalue(samples, edges, probs):
    counts, _ = np.histogram(samples, bins=edges)
    exp = probs / probs.sum() * len(samples)
    keep = exp > 5
    chi2 = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    return stats.chi2.sf(chi2, keep.sum() - 1)


def kn_dcs(E, c):
    k = E / MC2
    r = 1.0 / (1.0 + k * (1.0 - c))
    return 0.5 * RE**2 * r * r * (r + 1.0 / r - (1.0 - c * c))


def compton_pvalue(orc, E, n=200_000):
    """chi-square p-value of the oracle's Compton scattering angles against the
    Klein-Nishina cross section integrated by quadrature; 0 if a sample breaks
    the Compton kinematics or leaves [eps0, 1]."""
    eps, cost, words = orc.sample_compton(E, n, seed=11)
    k = E / MC2
    if not (np.allclose(eps, 1.0 / (1.0 + k * (1.0 - cost)), rtol=1e-12)
            and np.all(eps >= 1.0 / (1.0 + 2.0 * k) - 1e-15) and np.all(eps <= 1.0)):
        return 0.0
    edges = np.linspace(-1, 1, 41)
    probs = np.array([integrate.quad(lambda c: kn_dcs(E, c), a, b, epsabs=0, epsrel=1e-10)[0]
                      for a, b in zip(edges[:-1], edges[1:])])
    return chi2_pvalue(cost, edges, probs)


@pytest.mark.parametrize("E", [0.05, 0.5, 5.0])
def test_compton_angle_chi2(orc, E):
    n = 200_000
    eps, cost, words = orc.sample_compton(E, n, seed=11)
    assert compton_pvalue(orc, E, n) > 1e-4
    # three uniforms per rejection round
    assert np.all(words % 3 == 0) and words.min() == 3
    # Compton kinematics: E'/E = 1/(1 + k(1 - cos))
    k = E / MC2
    assert np.allclose(eps, 1.0 / (1.0 + k * (1.0 - cost)), rtol=1e-12)
    assert np.all(eps >= 1.0 / (1.0 + 2.0 * k) - 1e-15) and np.all(eps <= 1.0)
    # three uniforms per rejection round
    assert np.all(words % 3 == 0) and words.min() == 3


def moller_pvalue(orc, T, n=200_000):
    """chi-square p-value of the oracle's Moller eps = W/T samples against the
    Moller cross section differential in eps, integrated by quadrature; 0 if a
    sample leaves [Wcc/T, 1/2]."""
    Wcc = 0.05
    e0 = Wcc / T
    tau = T / MC2
    g = tau + 1
    a2 = (tau / g) ** 2
    b = (2 * tau + 1) / g**2
    pdf = lambda e: 1 / e**2 + 1 / (1 - e) ** 2 + a2 - b / (e * (1 - e))
    s = orc.sample_moller(T, Wcc, n, seed=5)
    if s.min() < e0 or s.max() > 0.5:
        return 0.0
    edges = np.geomspace(e0, 0.5, 41)
    probs = np.array([integrate.quad(pdf, lo, hi, epsabs=0, epsrel=1e-10)[0]
                      for lo, hi in zip(edges[:-1], edges[1:])])
    return chi2_pvalue(s, edges, probs)


@pytest.mark.parametrize("T", [0.3, 2.0, 15.0])
def test_moller_chi2(orc, T):
    assert moller_pvalue(orc, T) > 1e-4


# Mistakes in the Moller sampler (a mixture of the 1/eps^2, 1/(1-eps)^2 and
# a^2 terms, kept with probability f/h) planted in a copy of the oracle: each
# must fail the chi-square pin at one of the energies above.
MOLLER_MUTATIONS = {
    "second_term_dropped": ("const double w2 = 2.0 - 1.0 / (1.0 - e0);", "const double w2 = 0.0;"),
    "interference_term_dropped": ("if (ua * h <= h - b / q) return eps;",
                                  "if (ua * h <= h) return eps;"),
    "third_weight_without_a2": ("const double w3 = a2 * (0.5 - e0);",
                                "const double w3 = (0.5 - e0);"),
    "second_inverse_unscaled": ("eps = 1.0 - 1.0 / (2.0 - ue * w2);",
                                "eps = 1.0 - 1.0 / (2.0 - ue);"),
}


@pytest.mark.parametrize("name", sorted(MOLLER_MUTATIONS))
def test_moller_planted_mistake_is_caught(orc, name, tmp_path):
    import os
    import shutil
    old, new = MOLLER_MUTATIONS[name]
    src = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    for f in os.listdir(src):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(src, f), tmp_path / f)
    path = tmp_path / "transport.c"
    text = path.read_text()
    assert text.count(old) == 1, name
    path.write_text(text.replace(old, new))
    lib = orc.build(src_dir=str(tmp_path), lib_path=str(tmp_path / "liboracle_planted.so"))
    with orc.library(lib):
        worst = min(moller_pvalue(orc, T) for T in (0.3, 2.0, 15.0))
    assert worst <= 1e-4, f"the Moller chi-square pin did not catch {name} (p = {worst})"


def brems_pvalue(orc, T, n=200_000):
    """chi-square p-value of the oracle's bremsstrahlung photon energies against
    the (1/k)(4/3 - 4/3 y + y^2) spectrum on [kc, T] (its closed-form CDF); 0 if
    a sample leaves [kc, T]."""
    kc = 0.2
    cdf = lambda k: 4 / 3 * np.log(k / kc) - 4 / 3 * (k - kc) / T + (k * k - kc * kc) / (2 * T * T)
    s = orc.sample_brems(T, kc, n, seed=9)
    if s.min() < kc or s.max() > T:
        return 0.0
    edges = np.geomspace(kc, T, 41)
    return chi2_pvalue(s, edges, np.diff(cdf(edges)))


@pytest.mark.parametrize("T", [0.5, 3.0, 15.0])
def test_brems_chi2(orc, T):
    assert brems_pvalue(orc, T) > 1e-4


# Mistakes in the Klein-Nishina (Butcher-Messel) and bremsstrahlung samplers
# planted in a copy of the oracle: each must fail its chi-square pin at one
# of the energies above.
SAMPLER_MUTATIONS = {
    "compton_branch_weights_swapped": (
        "compton", "if (ua * (a1 + a2) < a1) eps = exp(-a1 * ub);",
        "if (ua * (a1 + a2) < a2) eps = exp(-a1 * ub);"),
    "compton_rejection_without_eps": (
        "compton", "if (uc <= 1.0 - eps * sin2 / (1.0 + eps * eps)) {",
        "if (uc <= 1.0 - sin2 / (1.0 + eps * eps)) {"),
    "compton_second_branch_linear": (
        "compton", "else eps = sqrt(e0 * e0 + (1.0 - e0 * e0) * ub);",
        "else eps = e0 + (1.0 - e0) * ub;"),
    "brems_rejection_without_quadratic": (
        "brems", "if (ub <= 1.0 - y + 0.75 * y * y) return k;", "if (ub <= 1.0 - y) return k;"),
    "brems_envelope_linear": (
        "brems", "const double k = kc * exp(ua * lr);", "const double k = kc + ua * (T - kc);"),
}


@pytest.mark.parametrize("name", sorted(SAMPLER_MUTATIONS))
def test_sampler_planted_mistake_is_caught(orc, name, tmp_path):
    import os
    import shutil
    which, old, new = SAMPLER_MUTATIONS[name]
    src = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
    for f in os.listdir(src):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(src, f), tmp_path / f)
    path = tmp_path / "transport.c"
    text = path.read_text()
    assert text.count(old) == 1, name
    path.write_text(text.replace(old, new))
    lib = orc.build(src_dir=str(tmp_path), lib_path=str(tmp_path / "liboracle_planted.so"))
    with orc.library(lib):
        if which == "compton":
            worst = min(compton_pvalue(orc, E) for E in (0.05, 0.5, 5.0))
        else:
            worst = min(brems_pvalue(orc, T) for T in (0.5, 3.0, 15.0))
    assert worst <= 1e-4, f"the {which} chi-square pin did not catch {name} (p = {worst})"


@pytest.mark.parametrize("x", [1e-4, 0.05, 0.7, 4.0])
def test_multiple_scattering_moment_and_shape(orc, x):
    """The deflection has the exact first moment <1 - cos> = 1 - exp(-x) after a
    path of x transport mean free paths, and the screened-Rutherford shape."""
    n = 200_000
    s = orc.sample_ms(x, n, seed=3)
    assert s.min() >= 0 and s.max() <= 2
    m1 = -np.expm1(-x)
    # table interpolation error in log2 A is far below the statistical error
    assert abs(s.mean() - m1) < 5 * s.std() / np.sqrt(n) + 1e-6 * m1
    A = None
    tab = orc.ms_table()
    import ctypes as C
    A = orc.lib().orc_ms_screening(tab.ctypes.data_as(C.POINTER(C.c_double)), x)
    F = lambda c: (1 / (2 * A) - 1 / (c + 2 * A)) / (1 / (2 * A) - 1 / (2 + 2 * A))
    edges = np.concatenate([[0], np.geomspace(max(A * 1e-3, 1e-12), 2, 40)])
    assert chi2_pvalue(s, edges, np.diff(F(edges))) > 1e-4


def test_rotation_invariants(orc):
    rng = np.random.default_rng(4)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        th, ph = rng.uniform(0, np.pi), rng.uniform(0, 2 * np.pi)
        c, s = np.cos(th), np.sin(th)
        r1 = orc.rotate(d, c, s, np.cos(ph), np.sin(ph))
        r2 = orc.rotate(d, c, s, -np.cos(ph), -np.sin(ph))  # azimuth + pi
        assert np.linalg.norm(r1) == pytest.approx(1.0, abs=1e-12)
        assert r1 @ d == pytest.approx(c, abs=1e-12)
        # opposite azimuths are mirror images about d
        assert np.allclose(r1 + r2, 2 * c * d, atol=1e-12)
        # quarter-turn azimuths are orthogonal in the plane perpendicular to d
        r3 = orc.rotate(d, c, s, np.cos(ph + np.pi / 2), np.sin(ph + np.pi / 2))
        assert (r1 - c * d) @ (r3 - c * d) == pytest.approx(0.0, abs=1e-12)
    # the polar-axis branch
    r = orc.rotate([0, 0, 1.0], 0.6, 0.8, 1.0, 0.0)
    assert np.allclose(r, [0.8, 0.0, 0.6])
    r = orc.rotate([0, 0, -1.0], 0.6, 0.8, 0.0, 1.0)
    assert np.allclose(r, [0.0, 0.8, -0.6])


def test_source_spectrum_and_field(orc, W):
    ph = W.slab_phantom(32, 1.0)
    spec = W.spectrum_6mv()
    src = W.photon_beam((10.0, 10.0), (16.0, 16.0), spectrum=spec)
    n = 100_000
    E, x, d = orc.sample_source(ph, src, n, seed=2)
    edges, w = spec
    assert chi2_pvalue(E, edges, w) > 1e-4
    # uniform inside each bin: fractional positions uniform
    b = np.searchsorted(edges, E) - 1
    frac = (E - edges[b]) / (edges[b + 1] - edges[b])
    assert stats.kstest(frac, "uniform").pvalue > 1e-4
    # field at the surface, uniform in the 10x10 square
    assert np.all(x[:, 2] == 0.0)
    assert np.all(np.abs(x[:, 0] - 16) <= 5) and np.all(np.abs(x[:, 1] - 16) <= 5)
    assert stats.kstest((x[:, 0] - 11) / 10, "uniform").pvalue > 1e-4
    # directions point away from the focal spot at SSD 100
    S = np.array([16.0, 16.0, -100.0])
    v = (x - S) / np.linalg.norm(x - S, axis=1)[:, None]
    assert np.allclose(v, d, atol=1e-12)
    # mean energy of the synthetic 6 MV spectrum
    assert 1.2 < E.mean() < 1.8


def test_source_gantry_and_miss(orc, W):
    ph = W.water_phantom((20, 20, 20), 1.0)
    src = W.photon_beam((2.0, 2.0), (10.0, 10.0), mono_E=1.0, parallel=True)
    src.update(gantry_deg=90.0, iso_x=10.0, iso_z=10.0, z_field=10.0)
    E, x, d = orc.sample_source(ph, src, 1000, seed=1)
    # gantry 90: the beam travels along +x and enters through the x = 0 face
    assert np.allclose(d, [1.0, 0.0, 0.0], atol=1e-12)
    assert np.allclose(x[:, 0], 0.0, atol=1e-12)
    assert np.all(np.abs(x[:, 2] - 10.0) <= 1.0 + 1e-12)
    # a field entirely beside the phantom misses
    src2 = W.photon_beam((2.0, 2.0), (40.0, 10.0), mono_E=1.0, parallel=True)
    E2, x2, _ = orc.sample_source(ph, src2, 100, seed=1)
    assert np.all(E2 == 0.0) and np.all(np.isnan(x2))
