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
    finder; raw intersections inside three 192^2 windows equal the oracle's on the windows."""
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
    raw = _gpu_ms(ctx, lf, model, truth, beta, a, grid, lf.LF_PREC_FP64, False)
    tab = orc.expand(model, truth)
    h = grid["h"]
    for s in (0, 1, 2):
        p0 = raw["theta"][s, 0]
        i0 = int((p0[0] - grid["x0"]) / h) - 96
        j0 = int((p0[1] - grid["y0"]) / h) - 96
        win = {"x0": grid["x0"] + i0 * h, "y0": grid["y0"] + j0 * h, "h": h, "nx": 192, "ny": 192}
        o = orc.find_images_ms(tab, win, beta[s:s + 1], a[s:s + 1])
        lo_x, lo_y = win["x0"] + 0.5 * h, win["y0"] + 0.5 * h
        hi_x, hi_y = lo_x + 191 * h, lo_y + 191 * h
        inside = [q for q in raw["theta"][s, :raw["count"][s]] if lo_x < q[0] < hi_x and lo_y < q[1] < hi_y]
        assert o["count"][0] == len(inside) and len(inside) >= 1
        for q in inside:
            assert np.abs(o["theta"][0, :o["count"][0]] - q).max(1).min() < 1e-10
