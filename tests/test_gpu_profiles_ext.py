"""GPU parity of the external shear and m = 3 multipole components (the extra halo types of the
paper's Hera and SMACS models) against the oracle: maps with and without third derivatives,
chi^2 with delays (their potential) and the image finder, at the maps, chi^2 and finder bars."""
import numpy as np
import pytest

from paper_2609_08649_amd import workloads as W
from tests import lensdata
from tests.test_gpu_maps import BASE, D3, _run, check, ctx, lf  # noqa: F401  (fixtures)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_maps_hera_like(ctx, lf, orc, prec):
    """Two elliptical NFW halos + external shear + m = 3 multipole + 40 members."""
    model, _ = W.tiny_model(51, n_main=4, n_mem=40, types=[W.ENFW, W.ENFW, W.SHEAR, W.MPOLE3])
    x, y = W.random_points(51, 3001, 25.0)
    g = _run(ctx, lf, model, None, 1, (x, y), 0.6, prec)
    o = orc.maps(orc.expand(model), x, y, 0.6)
    check({k: v[0] for k, v in g.items()}, o, prec)
    assert np.array_equal(g["flags"][0] & 1, o["flags"] & 1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_third_derivatives_smacs_like(ctx, lf, orc, prec):
    """Cored SIE + shear + multipole + elliptical members: third derivatives and A3 fields."""
    model, _ = W.tiny_model(52, n_main=3, n_mem=25, types=[W.SIE, W.SHEAR, W.MPOLE3], elliptical_members=True)
    x, y = W.random_points(52, 1500, 20.0)
    g = _run(ctx, lf, model, None, 1, (x, y), 0.5, prec, outputs=BASE + D3)
    o = orc.maps(orc.expand(model), x, y, 0.5)
    check({k: v[0] for k, v in g.items()}, o, prec, d3=True)


def enfw_model(seed=54, n_mem=30, n_enfw=4):
    """Two elliptical NFW halos and a cored SIE, with dPIE members of which n_enfw are elliptical
    NFW members (kappa_s 0.05-0.2, r_s 3-8", q 0.6-0.9)."""
    model, _ = W.tiny_model(seed, n_main=3, n_mem=n_mem, types=[W.ENFW, W.ENFW, W.SIE])
    rng = np.random.default_rng(seed + 1000)
    mem = model["members"]
    lum = mem["lum"]
    typ = np.full(n_mem, W.PJE, np.int32)
    typ[:n_enfw] = W.ENFW
    enfw = typ == W.ENFW
    model["members"] = {
        "type": typ, "x": mem["x"], "y": mem["y"],
        "q": np.where(enfw, rng.uniform(0.6, 0.9, n_mem), 1.0), "pa": rng.uniform(0, np.pi, n_mem),
        "b0": np.where(enfw, rng.uniform(0.05, 0.2, n_mem), 0.8 * np.sqrt(lum)),
        "s0": np.where(enfw, rng.uniform(3.0, 8.0, n_mem), 0.05),
        "a0": np.where(enfw, 0.0, 8.0 * np.sqrt(lum)),
        "bmul": W.fixed(1.0), "smul": W.fixed(1.0), "amul": W.fixed(1.0)}
    return model


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_third_derivatives_elliptical_nfw(ctx, lf, orc, prec):
    """Third derivatives and A3 fields of elliptical NFW main halos and members (integrals L_n of
    kappa'' over the same quadrature as alpha and psi_ij) against the oracle's derivatives of its
    adaptive quadrature."""
    model = enfw_model()
    x, y = W.random_points(54, 2001, 20.0)
    g = _run(ctx, lf, model, None, 1, (x, y), 0.55, prec, outputs=BASE + D3)
    o = orc.maps(orc.expand(model), x, y, 0.55)
    assert np.max(np.abs(o["p111"])) > 1e-3
    check({k: v[0] for k, v in g.items()}, o, prec, d3=True, a=0.55)


def _system(orc, seed=53):
    model, _ = W.tiny_model(seed, n_main=3, n_mem=20, types=[W.SIE, W.SHEAR, W.MPOLE3])
    tab = orc.expand(model)
    rng = np.random.default_rng(seed)
    cand = tab[0, 1:3] + rng.uniform(-2, 2, (400, 2))      # around the cored SIE
    zs = rng.uniform(1.0, 6.0, 400)
    grid = {"x0": -30.0, "y0": -30.0, "h": 0.2, "nx": 300, "ny": 300}
    srcs = lensdata.select_sources(orc, tab, grid, cand, zs, model["z_d"], 4)
    cons = lensdata.constraints_from_sources(srcs, 10 ** 6, rng.normal(0, 0.03, (200, 2)), 0.3)
    return model, tab, srcs, lensdata.observables(orc, tab, srcs, cons, model["z_d"], seed + 1), grid


def test_chi2_with_delays(ctx, lf, orc):
    """Source-plane chi^2 with flux and delay terms (the potential of both new types)."""
    import torch
    model, tab, srcs, cons, _ = _system(orc)
    assert cons["theta"].shape[0] >= 8
    m = ctx.upload_model(model)
    c = ctx.upload_constraints(cons)
    chi, fl, terms, _ = ctx.chi2_terms(m, None, 1, c, 0, lf.LF_PREC_FP64)
    torch.cuda.synchronize()
    o = orc.chi2_obs(tab[None], cons)
    t = terms.cpu().numpy()[0]
    for k, name in enumerate(("pos", "flux", "td")):
        assert abs(t[k] - o[name][0]) <= 1e-9 * abs(o[name][0]) + 1e-9, name
    c.release()
    m.release()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_finder(ctx, lf, orc, prec):
    """Images of the system's sources: counts identical, positions to 1e-9" (FP64) / 1e-4"."""
    import torch
    model, tab, srcs, cons, grid = _system(orc)
    beta = np.array([s[0] for s in srcs])
    a = np.array([s[2] for s in srcs])
    ok = [lensdata.margin_ok(orc, tab, grid, b_, a_) for b_, a_ in zip(beta, a)]
    beta, a = beta[ok], a[ok]
    assert len(beta) >= 2
    o = orc.find_images(tab, grid, beta, a)
    m = ctx.upload_model(model)
    r = ctx.find_images(m, None, torch.as_tensor(beta, device="cuda"), torch.as_tensor(a, device="cuda"), grid, 16,
                        lf.LF_PREC_FP64 if prec == "fp64" else lf.LF_PREC_MIXED)
    torch.cuda.synchronize()
    cnt = r["count"].cpu().numpy()
    assert np.array_equal(cnt, o["count"])
    th = r["theta"].cpu().numpy()
    tol = 1e-9 if prec == "fp64" else 1e-4
    for s in range(len(beta)):
        n = cnt[s]
        for p in o["theta"][s, :n]:
            assert np.abs(th[s, :n] - p).max(1).min() < tol
    m.release()
