"""Pins of the oracle's electron physics at transport level (CPU only).

Each check compares the oracle's transport code with a consequence of the
mathematics it implements, computed here independently (closed-form cross
sections and stopping powers, integrated with scipy), so that a plausible
mistake in the transport fails it:

* Hard events (Sec. 2.1: a Woodcock scheme over the continuous energy loss of a
  step). The first real hard event of an electron is a thinned Poisson process
  in mass path tau with rate sigma_hard(T(tau)), T(tau) from the CSDA relation
  dT/dtau = -S_r(T): its survival is exp(-integral of sigma_hard), and the
  event is Moller with probability sigma_M / sigma_hard at that energy.
* Multiple scattering (Sec. 2.1: random hinge with an angular deflection per
  step). With hard events off the steps of a track are deterministic; the mean
  cosines of independent deflections multiply (Goudsmit-Saunderson), so the
  mean direction cosine after k steps is the product of exp(-x_i),
  x_i = s_i rho / lambda_1(T_mid,i); the hinge at a uniform fraction of the
  step gives the first step a lateral second moment of s^2 <sin^2> / 3.
* Secondary kinematics (Sec. 2.1): momentum and energy balance of Compton
  scattering and of Moller scattering, the bremsstrahlung photon at the angle
  mc^2 / (T + mc^2), isotropic back-to-back annihilation photons and pair
  particles along the photon.

The planted-mistake tests build copies of the oracle with one mistake each
(sigma taken at the step's start, no new mean free path after a candidate,
lambda_1 at the start energy, the hinge at the middle of the step, and four
kinematic slips) and show that the corresponding check fails on each.
"""
import ctypes as C
import os
import shutil

import numpy as np
import pytest
from scipy import integrate, optimize, stats

MC2 = 0.51099895
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ------------------------------------------------------------------ helpers
def _closed(orc, W, name, mat, *a):
    f = orc.fn(name)
    return f(C.byref(mat.struct), *a)


def centre_source(W, E, direction=(0.0, 0.0, 1.0), L=40.0):
    """A one-record phase space at the centre of an L cm cube of water."""
    rec = np.array([[E, L / 2, L / 2, L / 2, *direction, 0.0]], np.float32)
    src = {"particle": 1, "geometry": 2, "psf": rec, "n_bins": 0, "mono_E": 0.0,
           "fx": 1.0, "fy": 1.0, "cx": 0.0, "cy": 0.0}
    return W.water_phantom((1, 1, 1), L), src


def csda_path(orc, W, T0, Tend, Wcc, kc):
    """Mass path tau(T) and the hard-event integrals along a CSDA track in
    water from closed forms: dT/dtau = -S_r(T), dLambda/dtau = sigma_hard(T),
    dLambda_M/dtau = sigma_M(T). Integrated in T (dtau = dT / S_r)."""
    mat = orc.material(W.WATER)

    def S(T):
        return (_closed(orc, W, "orc_scol_restricted", mat, T, Wcc)
                + _closed(orc, W, "orc_srad_restricted", mat, T, kc))

    def sig(T):
        return (_closed(orc, W, "orc_sigma_moller", mat, T, Wcc),
                _closed(orc, W, "orc_sigma_brems", mat, T, kc))

    def rhs(T, y):
        s = S(T)
        sm, sb = sig(T)
        return [-1.0 / s, -(sm + sb) / s, -sm / s]

    sol = integrate.solve_ivp(rhs, (T0, Tend), [0.0, 0.0, 0.0], rtol=1e-9, atol=1e-12,
                              dense_output=True, method="DOP853")
    return sol, S, sig


# ------------------------------------------------------------- hard events
# The method's thresholds (Moller 50 keV), where sigma_hard hardly changes
# along a track, and a Moller threshold of 250 keV, where sigma_M climbs from
# zero at 0.5 MeV to its plateau within the track, so that the majorant and
# the acceptance at the step's end matter and a mistake in them shows
HARD = {"method": dict(T0=3.0, Wcc=0.05, kc=0.2), "steep": dict(T0=3.0, Wcc=0.25, kc=0.2)}


def check_hard_events(orc, W, case="steep", n=200_000):
    """First real hard event of 3 MeV electrons in water: survival in mass path,
    Moller fraction and energy at the event. Returns (ok, detail)."""
    T0, Wcc, kc = HARD[case]["T0"], HARD[case]["Wcc"], HARD[case]["kc"]
    ph, src = centre_source(W, T0)
    params = {"Wcc": Wcc, "kc": kc}
    tau, Tev, kind = orc.first_hard(ph, src, n, seed=11, params=params)
    Eabs = 0.2
    sol, S, sig = csda_path(orc, W, T0, Eabs, Wcc, kc)
    # tau(T) is increasing as T falls: invert on a fine grid
    Tg = np.linspace(T0, Eabs, 4001)
    yg = sol.sol(Tg)
    tau_g, lam_g, lamM_g = yg[0], yg[1], yg[2]
    tau_tot = tau_g[-1]
    detail = {}
    ok = True
    ev = kind > 0
    # survival at fractions of the whole mass path
    for frac in (0.05, 0.15, 0.3, 0.5, 0.7, 0.9, 0.99):
        tq = frac * tau_tot
        lam = np.interp(tq, tau_g, lam_g)
        k = int(np.sum(~ev | (tau > tq)))
        pv = stats.binomtest(k, n, np.exp(-lam)).pvalue
        detail[f"S({frac})"] = (k / n, float(np.exp(-lam)), pv)
        ok &= pv > 1e-4
    # no event at all before absorption
    k0 = int(np.sum(~ev))
    p0 = float(np.exp(-lam_g[-1]))
    pv0 = stats.binomtest(k0, n, p0).pvalue
    detail["none"] = (k0 / n, p0, pv0)
    ok &= pv0 > 1e-4
    # kind of the first event: P(Moller) = int sigma_M e^-Lambda / int sigma e^-Lambda
    dens = np.exp(-lam_g)
    num = np.trapezoid(np.gradient(lamM_g, tau_g) * dens, tau_g)
    den = np.trapezoid(np.gradient(lam_g, tau_g) * dens, tau_g)
    pm = num / den
    km = int(np.sum(kind == 1))
    pvm = stats.binomtest(km, int(ev.sum()), pm).pvalue
    detail["moller_frac"] = (km / max(ev.sum(), 1), pm, pvm)
    ok &= pvm > 1e-4
    # the energy at the event is the CSDA energy after that mass path
    Tq = np.interp(tau[ev], tau_g, Tg)
    rel = float(np.max(np.abs(Tev[ev] - Tq) / Tq))
    detail["T_rel_err"] = rel
    ok &= rel < 2e-3
    return bool(ok), detail


@pytest.mark.parametrize("case", sorted(HARD))
def test_hard_event_law(orc, W, case):
    ok, detail = check_hard_events(orc, W, case)
    print(detail)
    assert ok, detail


# ------------------------------------------------------ multiple scattering
def screening_A(x):
    """Screening A with mean 1 - cos = 1 - exp(-x) for the screened-Rutherford
    form 1 - cos = 2 A u / (1 + A - u), u uniform (its mean is
    2A((1 + A) ln((1 + A)/A) - 1))."""
    target = -np.expm1(-x)

    def m1(A):
        return 2 * A * ((1 + A) * np.log1p(1 / A) - 1)

    return optimize.brentq(lambda la: m1(np.exp(la)) - target, -60, 12, xtol=1e-14)


def sin2_mean(x):
    A = np.exp(screening_A(x))
    m1 = integrate.quad(lambda u: 2 * A * u / (1 + A - u), 0, 1, limit=200)[0]
    m2 = integrate.quad(lambda u: (2 * A * u / (1 + A - u)) ** 2, 0, 1, limit=200)[0]
    return 2 * m1 - m2


def ms_steps(orc, W, T0, rho=1.0, dmax=0.5, fE=0.25, Eabs=0.2):
    """Deterministic step lengths, energies and x_i = s rho K1(T_mid) of a
    track with hard events off, from closed forms (no hinge truncation in a
    large voxel)."""
    mat = orc.material(W.WATER)
    Wcc, kc = 10.0, 20.0  # no hard Moller or bremsstrahlung below 20 MeV

    def S(T):
        return (_closed(orc, W, "orc_scol_restricted", mat, T, Wcc)
                + _closed(orc, W, "orc_srad_restricted", mat, T, kc))

    def Rm(T):  # mass range measured from Eabs
        return integrate.quad(lambda e: 1.0 / S(e), Eabs, T, limit=200, epsabs=1e-13)[0]

    def Tinv(r):
        return optimize.brentq(lambda T: Rm(T) - r, Eabs, T0 + 1e-9, xtol=1e-14)

    steps, T = [], T0
    while T > Eabs * (1 + 1e-9):
        RT = Rm(T)
        d_maxe = (RT - Rm((1 - fE) * T)) / rho if (1 - fE) * T > Eabs else np.inf
        d_abs = RT / rho
        d = min(dmax, d_maxe, d_abs)
        Tn = Eabs if d == d_abs else Tinv(RT - rho * d)
        Tmid = 0.5 * (T + Tn)
        x = d * rho * orc.fn("orc_K1")(C.byref(mat.struct), Tmid)
        steps.append((d, T, Tn, x))
        T = Tn
    return steps


def check_ms(orc, W, T0=2.0, n=40_000):
    """Mean direction cosine after each step against the product of exp(-x_i),
    the energies of the deterministic steps, and the first step's lateral and
    longitudinal moments against the random hinge."""
    ph, src = centre_source(W, T0)
    params = {"Wcc": 10.0, "kc": 20.0}
    tr = orc.trace_range(ph, src, n, seed=5, params=params, cap=64)
    steps = ms_steps(orc, W, T0)
    k_max = min(len(steps), min(len(t) for t in tr) - 1)
    detail = {"steps": len(steps)}
    ok = True
    # energies after each step (deterministic), from every history
    E = np.array([[t[k, 10] for k in range(k_max)] for t in tr])
    Ex = np.array([s[2] for s in steps[:k_max]])
    rel = float(np.max(np.abs(E - Ex) / Ex))
    detail["E_rel_err"] = rel
    ok &= rel < 2e-4
    # <w_k> = prod exp(-x_i)
    wk = np.array([[t[k, 9] for k in range(k_max)] for t in tr])
    pred = np.exp(-np.cumsum([s[3] for s in steps[:k_max]]))
    mean = wk.mean(axis=0)
    se = wk.std(axis=0, ddof=1) / np.sqrt(n)
    z = (mean - pred) / se
    detail["w_mean"] = np.round(mean, 4).tolist()
    detail["w_pred"] = np.round(pred, 4).tolist()
    detail["w_z"] = np.round(z, 2).tolist()
    ok &= bool(np.all(np.abs(z) < 5))
    # first step: displacement s (xi + (1 - xi) cos) along z and (1 - xi) s sin
    # across: means s (1 + <cos>)/2 and s^2 <sin^2>/3 for xi uniform
    d0, _, _, x0 = steps[0]
    p1 = np.array([t[0, 4:7] for t in tr]) - np.asarray(src["psf"][0, 1:4], np.float64)
    lat2 = p1[:, 0] ** 2 + p1[:, 1] ** 2
    pl = d0 ** 2 * sin2_mean(x0) / 3
    zl = (lat2.mean() - pl) / (lat2.std(ddof=1) / np.sqrt(n))
    pz = d0 * (1 + np.exp(-x0)) / 2
    zz = (p1[:, 2].mean() - pz) / (p1[:, 2].std(ddof=1) / np.sqrt(n))
    detail["lat2"] = (float(lat2.mean()), pl, float(zl))
    detail["z1"] = (float(p1[:, 2].mean()), pz, float(zz))
    ok &= abs(zl) < 5 and abs(zz) < 5
    return bool(ok), detail


@pytest.mark.parametrize("T0", [2.0, 0.8])
def test_multiple_scattering_along_the_track(orc, W, T0):
    ok, detail = check_ms(orc, W, T0)
    print(detail)
    assert ok, detail


def test_hinge_truncation_lands_on_faces(orc, W):
    """A step whose second hinge segment is cut at a voxel face ends exactly on
    that face (snapped), in every history of a fine grid."""
    ph = W.water_phantom((40, 40, 40), 0.05)
    src = W.electron_beam(1.0, (0.2, 0.2), (1.0, 1.0), parallel=True)
    tr = orc.trace_range(ph, src, 1000, seed=3, cap=4096)
    n_cut = 0
    for t in tr:
        code = t[:, 0].astype(int)
        cut = (code >= 25) & (code <= 28)  # 16 + limiter (maxs..event) + 8: crossed by the hinge
        n_cut += int(cut.sum())
        for r in t[cut]:
            pos = r[4:7] / 0.05
            assert np.min(np.abs(pos - np.round(pos))) < 1e-9, r
    assert n_cut > 100


# ------------------------------------------------------ secondary kinematics
def _sample(orc, W, which, args, n, seed=3, **params):
    ph = W.water_phantom((1, 1, 1), 1.0)
    src = W.photon_beam((1.0, 1.0), (0.5, 0.5), mono_E=1.0)
    p = {"Eabs_e": 0.0, "Eabs_g": 0.0}
    p.update(params)
    return orc.sample_event(which, args, n, ph, src, seed=seed, params=p)


def pmom(T):
    return np.sqrt(T * (T + 2 * MC2))


DIR0 = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])


def check_compton(orc, W, E=2.0, n=20_000):
    r, _ = _sample(orc, W, "compton", [E, *DIR0], n)
    Ep, d, Te, de = r[:, 0], r[:, 1:4], r[:, 5], r[:, 6:9]
    ok = bool(np.all(r[:, 4] == 1) and np.all(r[:, 13] == 1))
    ok &= bool(np.allclose(Ep + Te, E, rtol=0, atol=1e-12 * E))
    # photon momentum E d0 = E' d + p_e de with |p_e| = sqrt(Te (Te + 2 mc^2)):
    # the Compton relation between E' and the scattering angle
    pe = E * DIR0 - Ep[:, None] * d
    err = np.abs(np.linalg.norm(pe, axis=1) - pmom(Te)) / E
    ok &= bool(np.max(err) < 1e-9)
    ok &= bool(np.max(np.abs(np.cross(pe, de))) < 1e-9 * E)
    return ok, {"max_momentum_err": float(np.max(err))}


def check_moller(orc, W, T=3.0, n=20_000):
    r, _ = _sample(orc, W, "moller", [T, *DIR0], n)
    Tp, d, Wd, dd = r[:, 0], r[:, 1:4], r[:, 5], r[:, 6:9]
    ok = bool(np.all(r[:, 4] == 1) and np.allclose(Tp + Wd, T, rtol=0, atol=1e-12 * T))
    bal = pmom(T) * DIR0 - pmom(Tp)[:, None] * d - pmom(Wd)[:, None] * dd
    err = float(np.max(np.linalg.norm(bal, axis=1)) / pmom(T))
    ok &= err < 1e-9
    return ok, {"max_momentum_err": err}


def check_brems(orc, W, T=5.0, n=20_000):
    r, _ = _sample(orc, W, "brems", [T, *DIR0], n)
    Tn, d, k, dg = r[:, 0], r[:, 1:4], r[:, 5], r[:, 6:9]
    ok = bool(np.all(r[:, 4] == 1) and np.all(r[:, 13] == 0))
    ok &= bool(np.allclose(Tn + k, T, rtol=0, atol=1e-12 * T))
    ok &= bool(np.allclose(d, DIR0, rtol=0, atol=1e-15))
    cos = dg @ DIR0
    err = float(np.max(np.abs(cos - np.cos(MC2 / (T + MC2)))))
    ok &= err < 1e-12
    # the azimuth of the photon about the electron is uniform
    ref = np.cross(DIR0, [1.0, 0.0, 0.0])
    ref /= np.linalg.norm(ref)
    perp = dg - cos[:, None] * DIR0
    phi = np.arctan2(perp @ np.cross(DIR0, ref), perp @ ref)
    ks = stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue
    ok &= ks > 1e-4
    return ok, {"max_angle_err": err, "azimuth_ks": ks}


def check_annihilation(orc, W, n=40_000):
    r, _ = _sample(orc, W, "annihilation", [0.0, *DIR0], n)
    ok = bool(np.all(r[:, 4] == 2) and np.all(r[:, 13] == 0) and np.all(r[:, 14] == 0))
    ok &= bool(np.all(r[:, 5] == MC2) and np.all(r[:, 9] == MC2))
    a, b = r[:, 6:9], r[:, 10:13]
    ok &= bool(np.allclose(a, -b, rtol=0, atol=1e-15))
    # isotropic: each direction cosine uniform on [-1, 1], mean direction zero
    ks = [stats.kstest((a[:, j] + 1) / 2, "uniform").pvalue for j in range(3)]
    ok &= min(ks) > 1e-4
    return ok, {"ks": ks}


def check_pair(orc, W, E=8.0, n=20_000):
    r, _ = _sample(orc, W, "pair", [E, *DIR0], n)
    ok = bool(np.all(r[:, 4] == 2) and np.all(r[:, 13] == 1) and np.all(r[:, 14] == 2))
    K = E - 2 * MC2
    ok &= bool(np.allclose(r[:, 5] + r[:, 9], K, rtol=0, atol=1e-12 * E))
    ok &= bool(np.allclose(r[:, 6:9], DIR0, atol=1e-15) and np.allclose(r[:, 10:13], DIR0,
                                                                       atol=1e-15))
    ks = stats.kstest(r[:, 5] / K, "uniform").pvalue
    ok &= ks > 1e-4
    return ok, {"ks": ks}


KINEMATICS = {"compton": check_compton, "moller": check_moller, "brems": check_brems,
              "annihilation": check_annihilation, "pair": check_pair}


@pytest.mark.parametrize("name", sorted(KINEMATICS))
def test_secondary_kinematics(orc, W, name):
    ok, detail = KINEMATICS[name](orc, W)
    print(name, detail)
    assert ok, detail


def test_ms_deflection_sampler_event(orc, W):
    """The hinge deflection as the transport applies it: the new direction
    makes exactly the sampled angle with the old one, with a uniform azimuth,
    and the sampled 1 - cos has mean 1 - exp(-x)."""
    x = 0.3
    r, _ = _sample(orc, W, "ms", [0.0, *DIR0, x], 40_000)
    omc, d = r[:, 15], r[:, 1:4]
    assert np.allclose(d @ DIR0, 1 - omc, rtol=0, atol=1e-12)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    se = omc.std(ddof=1) / np.sqrt(len(omc))
    assert abs(omc.mean() - (1 - np.exp(-x))) < 5 * se + 2e-4


# ------------------------------------------------------- planted mistakes
# Each entry: the check it must fail and the textual edits of transport.c.
MUTATIONS = {
    "sigma_at_step_start": ("hard", [
        ("/* Test hook (orc_first_hard)", "static double g_T0;\n/* Test hook (orc_first_hard)"),
        ("    orc__grid_pos(p->E, &i, &f);\n    const double sM = lerp(T->sigM, i, f);",
         "    orc__grid_pos(g_T0, &i, &f);\n    const double sM = lerp(T->sigM, i, f);"),
        ("        const double T0 = p->E;\n        int i;\n        double f;\n"
         "        orc__grid_pos(T0, &i, &f);\n        const double RT = lerp(T->R, i, f);\n"
         "        const double shm = lerp(T->sigHat, i, f);\n        const double sig_hat",
         "        const double T0 = p->E;\n        g_T0 = T0;\n        int i;\n        double f;\n"
         "        orc__grid_pos(T0, &i, &f);\n        const double RT = lerp(T->R, i, f);\n"
         "        const double shm = lerp(T->sigHat, i, f);\n        const double sig_hat")]),
    "no_new_mean_free_path": ("hard", [
        ("        t->c.el_hard_fict++;\n    }\n    p->nmfp = -log(rng_u(&p->rng));",
         "        t->c.el_hard_fict++;\n    }\n    (void)0;")]),
    "lambda1_at_step_start": ("ms", [
        ("const double xs = d * rho * orc_table_lookup(T->K1, Tmid);",
         "const double xs = d * rho * orc_table_lookup(T->K1, T0);")]),
    "hinge_at_step_middle": ("ms", [
        ("                const double xi = rng_u(&p->rng);\n                const double s1 = xi * d;",
         "                const double xi = 0.5 + 0.0 * rng_u(&p->rng);\n"
         "                const double s1 = xi * d;")]),
    "moller_delta_same_azimuth": ("moller", [
        ("orc_rotate(dd, cd, sd, -cf, -sf);", "orc_rotate(dd, cd, sd, cf, sf);")]),
    "brems_angle_without_rest_mass": ("brems", [
        ("const double th = MC2 / (T + MC2);", "const double th = MC2 / T;")]),
    "compton_recoil_sign": ("compton", [
        ("pe[a] = E * d0[a] - Ep * p->d[a];", "pe[a] = E * d0[a] + Ep * p->d[a];")]),
    "annihilation_forward_only": ("annihilation", [
        ("    const double c = 2.0 * rng_u(r) - 1.0;\n    const double phi = 2.0 * PI * rng_u(r);",
         "    const double c = rng_u(r);\n    const double phi = 2.0 * PI * rng_u(r);")]),
}

CHECKS = {"hard": lambda orc, W: check_hard_events(orc, W, "steep", n=100_000),
          "ms": lambda orc, W: check_ms(orc, W, 2.0, n=20_000),
          **KINEMATICS}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(orc, W, name, tmp_path):
    check, edits = MUTATIONS[name]
    src = os.path.join(ROOT, "oracle")
    for f in os.listdir(src):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(src, f), tmp_path / f)
    path = tmp_path / "transport.c"
    text = path.read_text()
    for old, new in edits:
        assert text.count(old) >= 1, (name, old)
        text = text.replace(old, new, 1)
    path.write_text(text)
    lib = orc.build(src_dir=str(tmp_path), lib_path=str(tmp_path / "liboracle_planted.so"))
    with orc.library(lib):
        ok, detail = CHECKS[check](orc, W)
    print(name, detail)
    assert not ok, f"the {check} check did not catch the planted mistake {name}"
