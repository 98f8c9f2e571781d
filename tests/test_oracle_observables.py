"""Pins for the oracle's lensing potential (Sec. 2.1), time-delay scale (Eq. time_delay) and
the flux and time-delay chi^2 terms (Sec. 3.2 Eq. chi2_flux / msrc, Sec. 3.3 Eq. chi2_td /
dt0 / td_approx)."""
import numpy as np
import pytest
from scipy import integrate

from paper_2609_08649_amd import workloads as W

POINT, SIS, SIE, PJE, NFW, ENFW, SHEAR, MPOLE3 = 0, 1, 2, 3, 4, 5, 6, 7


def row(t, x=0.0, y=0.0, b=1.0, q=1.0, pa=0.0, s=0.0, a=0.0):
    return np.array([[t, x, y, b, q, pa, s, a]], dtype=np.float64)


PROFILES = [
    ("point", row(POINT, 0.3, -0.2, b=1.3)),
    ("sis", row(SIS, -0.4, 0.1, b=2.0)),
    ("csie", row(SIE, 0.2, 0.5, b=3.0, s=0.4)),
    ("esie", row(SIE, 0.2, 0.5, b=3.0, q=0.65, pa=0.7, s=0.4)),
    ("esie_s0", row(SIE, 0.2, 0.5, b=3.0, q=0.65, pa=0.7, s=0.0)),
    ("cpje", row(PJE, -1.0, 0.4, b=2.5, s=0.3, a=6.0)),
    ("cpje_s0", row(PJE, -1.0, 0.4, b=2.5, s=0.0, a=6.0)),
    ("epje", row(PJE, -1.0, 0.4, b=2.5, q=0.7, pa=2.1, s=0.3, a=6.0)),
    ("nfw", row(NFW, 0.5, 0.5, b=0.25, s=9.0)),
    ("enfw", row(ENFW, 0.5, 0.5, b=0.25, q=0.7, pa=0.4, s=9.0)),
    ("shear", row(SHEAR, 0.5, -0.5, b=0.07, pa=0.9)),
    ("mpole3", row(MPOLE3, -0.5, 0.5, b=0.05, pa=2.0)),
]


@pytest.mark.parametrize("name,tab", PROFILES, ids=[p[0] for p in PROFILES])
def test_potential_gradient_is_deflection(orc, name, tab):
    """alpha = grad psi (Sec. 2.1): central differences of the potential against the
    deflection, at points inside and outside cores, scale radii and cut radii."""
    x, y = W.random_points(5, 40, 14.0)
    h = 1e-5
    px = lambda xx, yy: orc.potential(tab, xx, yy)[0]
    gx = (px(x + h, y) - px(x - h, y)) / (2 * h)
    gy = (px(x, y + h) - px(x, y - h)) / (2 * h)
    m = orc.maps(tab, x, y, 0.5)
    scale = 1 + np.hypot(m["ax"], m["ay"])
    assert np.max(np.abs(gx - m["ax"]) / scale) < 2e-7, name
    assert np.max(np.abs(gy - m["ay"]) / scale) < 2e-7, name


def test_potential_laplacian_is_twice_kappa(orc):
    """nabla^2 psi = 2 kappa (second differences of psi against the convergence)."""
    tab = np.concatenate([PROFILES[3][1], PROFILES[7][1], PROFILES[9][1]])
    x, y = W.random_points(6, 30, 10.0)
    h = 1e-3
    p = lambda xx, yy: orc.potential(tab, xx, yy)[0]
    lap = (p(x + h, y) + p(x - h, y) + p(x, y + h) + p(x, y - h) - 4 * p(x, y)) / (h * h)
    k = orc.maps(tab, x, y, 0.5)["kappa"]
    assert np.allclose(lap, 2 * k, rtol=1e-4, atol=1e-5)


def test_elliptical_nfw_potential_tends_to_circular(orc):
    x, y = W.random_points(7, 20, 20.0)
    c = orc.potential(row(NFW, 0.5, 0.5, b=0.25, s=9.0), x, y)[0]
    e = orc.potential(row(ENFW, 0.5, 0.5, b=0.25, q=0.999999, pa=0.3, s=9.0), x, y)[0]
    assert np.allclose(e - e[0], c - c[0], rtol=1e-5, atol=1e-6)


def test_potential_rotation_covariance(orc):
    x, y = W.random_points(8, 20, 8.0)
    t = 0.9
    c, s = np.cos(t), np.sin(t)
    for tab in (PROFILES[4][1], PROFILES[7][1], PROFILES[9][1]):
        t0 = tab.copy(); t0[0, 1:3] = 0.0
        t1 = t0.copy(); t1[0, 5] += t
        p0 = orc.potential(t0, x, y)[0]
        p1 = orc.potential(t1, c * x - s * y, s * x + c * y)[0]
        assert np.allclose(p0, p1, rtol=1e-11, atol=1e-11)


def test_time_delay_scale(orc):
    """(1+z_d)/c D_d D_s/D_ds theta0^2 from distances integrated here with scipy; it scales as
    1/H0 (distances do)."""
    c_kms, mpc_m, day = 299792.458, 3.0856775814913673e22, 86400.0

    def DA(z1, z2, H0=70.0, Om=0.3):
        I = integrate.quad(lambda z: 1 / np.sqrt(Om * (1 + z) ** 3 + 1 - Om), z1, z2, epsabs=1e-14, epsrel=1e-13)[0]
        return c_kms / H0 * I / (1 + z2)
    zd, zs = 0.5, 2.0
    T = (1 + zd) / (c_kms * 1e3) * DA(0, zd) * DA(0, zs) / DA(zd, zs) * mpc_m * (np.pi / 648000) ** 2 / day
    assert abs(orc.tdscale(zd, zs) / T - 1) < 1e-10
    assert abs(orc.tdscale(zd, zs, H0=35.0) / orc.tdscale(zd, zs) - 2) < 1e-10


# ------------------------------------------------------------------ flux and time-delay chi^2
def _exact_system(orc, seed=11):
    """A tiny lens, one source with >= 3 well-magnified oracle images (0.5 < |mu| < 50; the
    demagnified central image of a cored lens is dropped), exact magnitudes and delays."""
    model, _ = W.tiny_model(seed, n_main=2, n_mem=8, types=[2, 3])
    tab = orc.expand(model)
    rng = np.random.default_rng(seed)
    grid = {"x0": -30.0, "y0": -30.0, "h": 0.06, "nx": 1000, "ny": 1000}
    a = 0.62
    c0 = tab[:2, 1:3].mean(0)
    for b in c0 + rng.uniform(-2.0, 2.0, (80, 2)):
        fi = orc.find_images(tab, grid, b[None], np.array([a]))
        n = fi["count"][0]
        mu = fi["mu"][0, :n]
        keep = (np.abs(mu) > 0.5) & (np.abs(mu) < 50)
        if keep.sum() >= 3 and not fi["flags"][0]:
            return tab, b, a, fi["theta"][0, :n][keep].copy(), mu[keep].copy()
    raise AssertionError("no multiply imaged source")


def _cons(theta, a, extra):
    n = theta.shape[0]
    c = {"theta": theta, "family": np.zeros(n, np.int32), "sig1": np.full(n, 0.05), "sig2": np.full(n, 0.05),
         "phi": np.zeros(n), "a_fam": np.array([a])}
    c.update(extra)
    return c


def _observed(orc, tab, b, a, theta, mu, m0=24.0, t0=5.0):
    """Exact magnitudes m_i = m0 - 2.5 log10|mu_i| and delays T (|theta - beta|^2/2 - a psi) + t0."""
    T = orc.tdscale(0.5, 2.0)
    psi = orc.potential(tab, theta[:, 0], theta[:, 1])[0]
    d = theta - b
    n = theta.shape[0]
    return {"mag": m0 - 2.5 * np.log10(np.abs(mu)), "sig_mag": np.full(n, 0.1),
            "dt": T * (0.5 * np.sum(d * d, 1) - a * psi) + t0, "sig_dt": np.full(n, 0.5),
            "tscale": np.array([T])}


@pytest.mark.parametrize("img_mode", [False, True])
def test_exact_images_give_zero_flux_and_delay_chi2(orc, img_mode):
    tab, b, a, theta, mu = _exact_system(orc)
    c = _cons(theta, a, _observed(orc, tab, b, a, theta, mu))
    r = orc.chi2_obs(tab[None], c, img_mode=img_mode)
    assert r["flux"][0] < 1e-14
    assert r["td"][0] < 1e-10
    assert r["pos"][0] < 1e-10


def test_fermat_stationary_at_images(orc):
    """grad_theta of the arrival time T (|theta - beta|^2 / 2 - a psi) vanishes at an image."""
    tab, b, a, theta, mu = _exact_system(orc)
    h = 1e-5
    f = lambda x, y: 0.5 * ((x - b[0]) ** 2 + (y - b[1]) ** 2) - a * orc.potential(tab, x, y)[0]
    gx = (f(theta[:, 0] + h, theta[:, 1]) - f(theta[:, 0] - h, theta[:, 1])) / (2 * h)
    gy = (f(theta[:, 0], theta[:, 1] + h) - f(theta[:, 0], theta[:, 1] - h)) / (2 * h)
    assert np.max(np.abs(gx)) < 1e-7 and np.max(np.abs(gy)) < 1e-7


def test_nuisance_offsets_are_absorbed(orc):
    """A common offset of a family's magnitudes (m_src, Eq. msrc) or delays (dt_0, Eq. dt0)
    leaves the terms unchanged; a single offset image does not."""
    tab, b, a, theta, mu = _exact_system(orc)
    rng = np.random.default_rng(3)
    th = theta + rng.normal(0, 0.01, theta.shape)
    o = _observed(orc, tab, b, a, theta, mu)
    base = orc.chi2_obs(tab[None], _cons(th, a, o))
    o2 = dict(o, mag=o["mag"] + 0.7, dt=o["dt"] - 40.0)
    shifted = orc.chi2_obs(tab[None], _cons(th, a, o2))
    assert np.isclose(base["flux"][0], shifted["flux"][0], rtol=1e-9, atol=1e-12)
    assert np.isclose(base["td"][0], shifted["td"][0], rtol=1e-9, atol=1e-12)
    o3 = dict(o, mag=o["mag"] + np.r_[0.5, np.zeros(len(o["mag"]) - 1)])
    assert orc.chi2_obs(tab[None], _cons(th, a, o3))["flux"][0] > base["flux"][0] + 1.0


def test_linear_expansions_converge_to_image_plane(orc):
    """The source-plane flux and delay predictions (linear in beta_model - beta_obs) approach
    the image-plane ones quadratically as the astrometric noise shrinks."""
    tab, b, a, theta, mu = _exact_system(orc)
    o = _observed(orc, tab, b, a, theta, mu)
    o["sig_mag"] = np.full(len(mu), 1e-3)
    o["sig_dt"] = np.full(len(mu), 1e-3)
    rng = np.random.default_rng(4)
    noise = rng.normal(0, 1, theta.shape)
    diffs = []
    for eps in (1e-3, 1e-4):
        c = _cons(theta + eps * noise, a, o)
        s = orc.chi2_obs(tab[None], c, img_mode=False)
        i = orc.chi2_obs(tab[None], c, img_mode=True)
        diffs.append((abs(np.sqrt(s["flux"][0]) - np.sqrt(i["flux"][0])),
                      abs(np.sqrt(s["td"][0]) - np.sqrt(i["td"][0]))))
    # residuals are O(eps); their source- vs image-plane difference is O(eps^2)
    for k in range(2):
        assert diffs[1][k] < diffs[0][k] / 30 or diffs[1][k] < 1e-9


def test_terms_need_errors(orc):
    """Images without a positive error do not enter a term; no measurements give zero."""
    tab, b, a, theta, mu = _exact_system(orc)
    o = _observed(orc, tab, b, a, theta, mu)
    c = _cons(theta + 0.01, a, dict(o, sig_mag=np.zeros(len(mu)), sig_dt=-np.ones(len(mu))))
    r = orc.chi2_obs(tab[None], c)
    assert r["flux"][0] == 0.0 and r["td"][0] == 0.0
    r0 = orc.chi2_obs(tab[None], _cons(theta + 0.01, a, {}))
    assert r0["flux"][0] == 0.0 and r0["td"][0] == 0.0
    pos = orc.chi2_batch(tab[None], _cons(theta + 0.01, a, {}))["chi2_src"][0]
    assert np.isclose(r0["pos"][0], pos, rtol=1e-14)
