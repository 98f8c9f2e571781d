"""GPU parity of the contour-intersection finder (Sec. 2.3, lf_find_images_ms) against the
oracle's, and agreement of its polished images with the triangle-mapping finder.

FP64: counts identical, raw intersections to 1e-10" (the same arithmetic on vertex values
that agree to ~1e-15), polished images to 1e-9".  MIXED: vertex deflections within 1e-5",
so raw intersections within 1e-4" and counts identical for sources away from caustics."""
import numpy as np
import pytest

from paper_2609_08649_amd import workloads as W
from tests import lensdata

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


def _gpu_ms(ctx, lf, model, params, beta, a, grid, prec, polish):
    import torch
    m = ctx.upload_model(model)
    pp = torch.as_tensor(params[None], device="cuda") if params is not None and params.size else None
    r = ctx.find_images_ms(m, pp, torch.as_tensor(beta, device="cuda"), torch.as_tensor(a, device="cuda"), grid, 16,
                           prec, polish)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in r.items()}
    m.release()
    return out


def _same_images(g, o, tol, nsrc):
    assert np.array_equal(g["count"], o["count"]), (g["count"], o["count"])
    for s in range(nsrc):
        n = min(int(o["count"][s]), 16)
        if n:
            assert np.max(np.abs(g["theta"][s, :n] - o["theta"][s, :n])) < tol, s


def _sources(orc, tab, grid, seed, n=24, spread=2.5):
    rng = np.random.default_rng(seed)
    b = tab[0, 1:3] + rng.uniform(-spread, spread, (n, 2))
    a = rng.uniform(0.4, 0.9, n)
    keep = [lensdata.margin_ok(orc, tab, grid, bb, aa) for bb, aa in zip(b, a)]
    return b[keep], a[keep]


@pytest.mark.parametrize("seed", [4, 6])
def test_raw_and_polished_fp64(ctx, lf, orc, seed):
    model, truth = W.tiny_model(seed, n_main=2, n_mem=20, types=[2, 3], free_params=True)
    tab = orc.expand(model, truth)
    grid = {"x0": -25.0, "y0": -24.9, "h": 0.1, "nx": 500, "ny": 501}
    beta, a = _sources(orc, tab, grid, seed)
    assert len(beta) >= 10 and (orc.find_images(tab, grid, beta, a)["count"] > 1).sum() >= 10
    for polish, tol in ((False, 1e-10), (True, 1e-9)):
        o = orc.find_images_ms(tab, grid, beta, a, polish=polish)
        g = _gpu_ms(ctx, lf, model, truth, beta, a, grid, lf.LF_PREC_FP64, polish)
        _same_images(g, o, tol, len(beta))
        assert np.allclose(g["mu"], o["mu"], rtol=1e-8, atol=1e-10)


def test_polished_equals_triangle_mapping(ctx, lf, orc):
    import torch
    model, truth = W.tiny_model(8, n_main=2, n_mem=20, types=[2, 3], free_params=True)
    tab = orc.expand(model, truth)
    grid = {"x0": -25.0, "y0": -25.0, "h": 0.1, "nx": 500, "ny": 500}
    beta, a = _sources(orc, tab, grid, 8)
    g = _gpu_ms(ctx, lf, model, truth, beta, a, grid, lf.LF_PREC_FP64, True)
    m = ctx.upload_model(model)
    t = ctx.find_images(m, torch.as_tensor(truth[None], device="cuda"), torch.as_tensor(beta, device="cuda"),
                        torch.as_tensor(a, device="cuda"), grid, 16, lf.LF_PREC_FP64)
    torch.cuda.synchronize()
    m.release()
    tc, tt = t["count"].cpu().numpy(), t["theta"].cpu().numpy()
    assert np.array_equal(g["count"], tc)
    for s in range(len(beta)):
        for p in tt[s, :tc[s]]:
            assert np.abs(g["theta"][s, :tc[s]] - p).max(1).min() < 1e-9


def test_mixed(ctx, lf, orc):
    model, truth = W.tiny_model(6, n_main=2, n_mem=20, types=[2, 3], free_params=True)
    tab = orc.expand(model, truth)
    grid = {"x0": -25.0, "y0": -25.0, "h": 0.1, "nx": 500, "ny": 500}
    beta, a = _sources(orc, tab, grid, 9)
    o = orc.find_images_ms(tab, grid, beta, a)
    g = _gpu_ms(ctx, lf, model, truth, beta, a, grid, lf.LF_PREC_MIXED, False)
    _same_images(g, o, 1e-4, len(beta))


def test_cluster_2048_windows(ctx, lf, orc):
    """The 60 cluster sources on the 2048^2 grid (polished): the same images as the triangle
    finder; raw intersections on the whole grid equal the oracle's, in the same order."""
    import torch
    cfg = W.config2(n_samples=1)
    model, truth = cfg["model"], cfg["truth"]
    beta, _, a = lensdata.cluster_sources()
    grid = {"x0": -100.0, "y0": -100.0, "h": 200.0 / 2048, "nx": 2048, "ny": 2048}
    pol = _gpu_ms(ctx, lf, model, truth, beta, a, grid, lf.LF_PREC_FP64, True)
    m = ctx.upload_model(model)
    t = ctx.find_images(m, torch.as_tensor(truth[None], device="cuda"), torch.as_tensor(beta, device="cuda"),
                        torch.as_tensor(a, device="cuda"), grid, 16, lf.LF_PREC_FP64)
    torch.cuda.synchronize()
    m.release()
    tc, tt = t["count"].cpu().numpy(), t["theta"].cpu().numpy()
    match = 0
    for s in range(len(beta)):
        if pol["count"][s] == tc[s] and all(np.abs(pol["theta"][s, :tc[s]] - p).max(1).min() < 1e-9
                                            for p in tt[s, :tc[s]]):
            match += 1
    assert match >= len(beta) - 2, match          # sources next to caustics may differ
    # raw intersections on the whole grid against the oracle's (about 5 s of oracle time)
    raw = _gpu_ms(ctx, lf, model, truth, beta, a, grid, lf.LF_PREC_FP64, False)
    o = orc.find_images_ms(orc.expand(model, truth), grid, beta, a)
    assert np.array_equal(raw["count"], o["count"]), np.nonzero(raw["count"] != o["count"])
    assert o["count"].sum() >= 200
    for s in range(len(beta)):
        n = o["count"][s]
        assert np.max(np.abs(raw["theta"][s, :n] - o["theta"][s, :n]), initial=0) < 1e-10, s
