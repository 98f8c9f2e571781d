"""GPU parity of lf_chi2_terms (flux and time-delay chi^2, Sec. 3.2 and 3.3) against the FP64
oracle, on seeded constraints whose magnitudes and delays the oracle derives from the true
images (plus noise).

Tolerances.  FP64: each term to 1e-9 relative, widened by 1e-15 mu_max^2 for images near a
critical curve (the position weights grow as mu^2, so rounding of det A is amplified), and by
1e-15 mu_max^3 for the flux term (its expansion carries mu^2 grad det A).  MIXED: the terms are FP64 sums evaluated at
beta_model - beta_obs of the mixed source-plane fit, so they inherit its error, at most
3e-5" (|d alpha| <= 1e-5" enters beta_obs and, through the weighted mean, beta_model): it
moves each delay by T |beta_obs - theta| |d beta| and each model magnitude by 2.5/ln10 |mu|
|A^-T grad det A| |d beta|.  With these errors e_i, the chi^2 moves by at most
2 sqrt(chi^2 sum (e_i / sigma_i)^2) + sum (e_i / sigma_i)^2 (subtracting the weighted-mean
zero point is a projection and only shrinks the error vector), the bound used below, plus
1e-3 relative as for the position term."""
import numpy as np
import pytest

from paper_2609_08649_amd import workloads as W
from tests import lensdata
from tests.lensdata import mu_max, stable_image_plane
from tests.test_gpu_chi2 import _jitter

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available()
    from paper_2609_08649_amd import lensfield
    return lensfield


@pytest.fixture(scope="module")
def ctx(lf):
    c = lf.Context(0)
    yield c
    c.close()


def _gpu(ctx, lf, model, params, cons, mode, prec):
    import torch
    m = ctx.upload_model(model)
    c = ctx.upload_constraints(cons)
    pp = torch.as_tensor(params, device="cuda")
    chi, fl, terms, _ = ctx.chi2_terms(m, pp, params.shape[0], c, mode, prec)
    torch.cuda.synchronize()
    out = chi.cpu().numpy(), fl.cpu().numpy(), terms.cpu().numpy()
    c.release()
    m.release()
    return out


def _mixed_bound(orc, tabs, cons, chi_t, chi_f, dbeta=3e-5):
    """First-order bound on the change of chi^2_dt and chi^2_f from an error dbeta in
    beta_model - beta_obs (module docstring), per sample.  The sensitivities come from the
    oracle's fields at theta_obs: d t_i / d beta = T (beta_obs - theta) and d m_i / d beta =
    2.5 / ln 10 mu A^-T grad(det A), grad(det A) from the third derivatives."""
    a = cons["a_fam"][cons["family"]]
    T = cons["tscale"][cons["family"]] if "tscale" in cons else np.zeros_like(a)
    sdt = cons.get("sig_dt", np.zeros_like(a))
    smag = cons.get("sig_mag", np.zeros_like(a))
    et, ef = np.zeros(len(tabs)), np.zeros(len(tabs))
    for s, t in enumerate(tabs):
        m = orc.maps(t, cons["theta"][:, 0], cons["theta"][:, 1], 1.0)
        r = np.hypot(a * m["ax"], a * m["ay"])
        ht = sdt > 0
        et[s] = np.sum((T[ht] * r[ht] * dbeta / sdt[ht]) ** 2)
        A11, A12, A22 = 1 - a * m["p11"], -a * m["p12"], 1 - a * m["p22"]
        det = A11 * A22 - A12 ** 2
        gx = -a * (m["p111"] * A22 + A11 * m["p122"] - 2 * A12 * m["p112"])
        gy = -a * (m["p112"] * A22 + A11 * m["p222"] - 2 * A12 * m["p122"])
        vx, vy = (A22 * gx - A12 * gy) / det, (-A12 * gx + A11 * gy) / det
        sens = 2.5 / np.log(10) * np.abs(1 / det) * np.hypot(vx, vy) * dbeta
        hf = smag > 0
        ef[s] = np.sum((sens[hf] / smag[hf]) ** 2)
    return 2 * np.sqrt(chi_t * et) + et, 2 * np.sqrt(chi_f * ef) + ef


def _check(g_terms, o, prec, mu, bt=None, bf=None):
    for k, name in enumerate(("pos", "flux", "td")):
        ref, got = o[name], g_terms[:, k]
        if prec == "fp64":
            w = 1e-9 + 1e-15 * mu ** (3 if name == "flux" else 2)
            tol = w * np.abs(ref) + w
        elif name == "pos":
            tol = 1e-3 * np.abs(ref) + 1e-3
        else:
            tol = 1e-3 * np.abs(ref) + 1e-3 + (bt if name == "td" else bf)
        bad = np.abs(got - ref) > tol
        assert not bad.any(), (name, np.max(np.abs(got - ref) / (tol)), np.nonzero(bad)[0][:5])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("seed", [41, 42])
def test_observables_small_models(ctx, lf, orc, prec, seed):
    model, truth, cons = lensdata.small_observables(seed)
    params = _jitter(truth, 37, seed)
    P = lf.LF_PREC_FP64 if prec == "fp64" else lf.LF_PREC_MIXED
    tabs = orc.expand_batch(model, params)
    mu = mu_max(orc, tabs, cons)
    o = orc.chi2_obs(tabs, cons, img_mode=False)
    bt, bf = _mixed_bound(orc, tabs, cons, o["td"], o["flux"])
    chi, fl, terms = _gpu(ctx, lf, model, params, cons, 0, P)
    _check(terms, o, prec, mu, bt, bf)
    assert np.allclose(chi, terms.sum(1), rtol=1e-15, atol=0)
    assert o["flux"].min() > 0 and o["td"].min() > 0
    # image plane on the well-posed samples
    oi = orc.chi2_obs(tabs, cons, img_mode=True)
    st = stable_image_plane(orc, tabs, cons, orc.chi2_batch(tabs, cons, img_mode=True)["chi2_img"])
    assert st.sum() >= 10
    chi, fl, terms = _gpu(ctx, lf, model, params, cons, 1, P)
    sub = {k: v[st] for k, v in oi.items()}
    _check(terms[st], sub, prec, mu[st], bt[st], bf[st])
    assert np.array_equal(fl[st] & 12, oi["flags"][st] & 12)


def test_observables_cluster_full_size(ctx, lf, orc):
    """1024 samples x 150 images (magnitudes on ~5/6, delays on ~2/3 of them) x 302 halos,
    source plane, both precisions, every sample compared."""
    cfg = W.config2(n_samples=1024)
    cons = lensdata.cluster_observables()
    tabs = orc.expand_batch(cfg["model"], cfg["params"])
    o = orc.chi2_obs(tabs, cons, img_mode=False)
    mu = mu_max(orc, tabs, cons)
    bt, bf = _mixed_bound(orc, tabs, cons, o["td"], o["flux"])
    for prec, P in (("fp64", lf.LF_PREC_FP64), ("mixed", lf.LF_PREC_MIXED)):
        chi, fl, terms = _gpu(ctx, lf, cfg["model"], cfg["params"], cons, 0, P)
        _check(terms, o, prec, mu, bt, bf)


def test_observables_cluster_image_plane_subset(ctx, lf, orc):
    cfg = W.config2(n_samples=1024)
    cons = lensdata.cluster_observables()
    params = cfg["params"][:1] + 0.05 * (cfg["params"][:48] - cfg["params"][:1])
    tabs = orc.expand_batch(cfg["model"], params)
    mu = mu_max(orc, tabs, cons)
    oi = orc.chi2_obs(tabs, cons, img_mode=True)
    st = stable_image_plane(orc, tabs, cons, orc.chi2_batch(tabs, cons, img_mode=True)["chi2_img"])
    assert st.mean() >= 0.9
    bt, bf = _mixed_bound(orc, tabs, cons, oi["td"], oi["flux"])
    for prec, P in (("fp64", lf.LF_PREC_FP64), ("mixed", lf.LF_PREC_MIXED)):
        chi, fl, terms = _gpu(ctx, lf, cfg["model"], params, cons, 1, P)
        sub = {k: v[st] for k, v in oi.items()}
        _check(terms[st], sub, prec, mu[st], bt[st], bf[st])


def test_terms_without_data_equal_chi2_batch(ctx, lf):
    import torch
    model, truth, cons = lensdata.small_constraints(41)
    params = _jitter(truth, 9, 2)
    m = ctx.upload_model(model)
    c = ctx.upload_constraints(cons)
    pp = torch.as_tensor(params, device="cuda")
    for mode in (0, 1):
        a, fa, _ = ctx.chi2_batch(m, pp, 9, c, mode, lf.LF_PREC_MIXED)
        b, fb, t, _ = ctx.chi2_terms(m, pp, 9, c, mode, lf.LF_PREC_MIXED)
        assert torch.equal(a, b) and torch.equal(fa, fb)
        assert torch.equal(t[:, 0], a) and not t[:, 1:].any()
    c.release()
    m.release()


def test_only_delays_or_only_fluxes(ctx, lf, orc):
    """Either kind of data alone: the other term is zero in both implementations."""
    model, truth, cons = lensdata.small_observables(42)
    params = _jitter(truth, 8, 6)
    tabs = orc.expand_batch(model, params)
    mu = mu_max(orc, tabs, cons)
    for drop in (("mag", "sig_mag"), ("dt", "sig_dt", "tscale")):
        c2 = {k: v for k, v in cons.items() if k not in drop}
        o = orc.chi2_obs(tabs, c2)
        _, _, terms = _gpu(ctx, lf, model, params, c2, 0, lf.LF_PREC_FP64)
        _check(terms, o, "fp64", mu)
        assert not terms[:, 1 if drop[0] == "mag" else 2].any()


def test_observables_errors(ctx, lf):
    import torch
    model, truth, cons = lensdata.small_observables(41)
    n = cons["theta"].shape[0]
    for bad in (dict(cons, tscale=-cons["tscale"]), dict(cons, mag=np.full(n, np.nan)),
                dict(cons, sig_dt=np.full(n, np.inf))):
        with pytest.raises(lf.LfError) as e:
            ctx.upload_constraints(bad)
        assert e.value.status == lf.LF_E_INVALID_ARG
    c = ctx.upload_constraints(cons)
    with pytest.raises(lf.LfError) as e:                       # observables are attached once
        ctx.check(lf.lib().lf_constraints_observables(ctx.handle, c.handle, None, None, None, None, None))
    assert e.value.status == lf.LF_E_INVALID_ARG
    m = ctx.upload_model(model)
    pp = torch.as_tensor(_jitter(truth, 2, 1), device="cuda")
    with pytest.raises(lf.LfError) as e:                       # the batched graph has no such terms
        lf.Batch(ctx, [(m, c, pp, 2)])
    assert e.value.status == lf.LF_E_UNSUPPORTED
    m.release()
    c.release()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_observables_elliptical_nfw(ctx, lf, orc, prec):
    """Flux and delay terms of a lens with elliptical NFW halos and members: grad mu from their
    third derivatives, the potential from their quadrature; both chi^2 modes against the oracle."""
    import torch
    from tests.test_gpu_profiles_ext import enfw_model
    model = enfw_model(56)
    tab = orc.expand(model)
    rng = np.random.default_rng(56)
    cand = tab[0, 1:3] + rng.uniform(-3, 3, (400, 2))
    zs = rng.uniform(1.0, 6.0, 400)
    grid = {"x0": -30.0, "y0": -30.0, "h": 0.2, "nx": 300, "ny": 300}
    srcs = lensdata.select_sources(orc, tab, grid, cand, zs, model["z_d"], 4)
    cons = lensdata.constraints_from_sources(srcs, 10 ** 6, rng.normal(0, 0.03, (200, 2)), 0.3)
    cons = lensdata.observables(orc, tab, srcs, cons, model["z_d"], 57)
    assert cons["theta"].shape[0] >= 8
    tabs = tab[None]
    mu = mu_max(orc, tabs, cons)
    assert stable_image_plane(orc, tabs, cons, orc.chi2_batch(tabs, cons, img_mode=True)["chi2_img"])[0]
    m = ctx.upload_model(model)
    c = ctx.upload_constraints(cons)
    P = lf.LF_PREC_FP64 if prec == "fp64" else lf.LF_PREC_MIXED
    for mode in (0, 1):
        _, fl, terms, _ = ctx.chi2_terms(m, None, 1, c, mode, P)
        torch.cuda.synchronize()
        o = orc.chi2_obs(tabs, cons, img_mode=bool(mode))
        bt, bf = _mixed_bound(orc, tabs, cons, o["td"], o["flux"])
        _check(terms.cpu().numpy(), o, prec, mu, bt, bf)
        assert o["flux"][0] > 0 and o["td"][0] > 0
        assert np.array_equal(fl.cpu().numpy() & 12, o["flags"] & 12)
    c.release()
    m.release()
