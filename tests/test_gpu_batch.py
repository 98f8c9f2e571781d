"""Uneven batched chi^2 (persistent launch in a hipGraph, autotuned tiles): every item's
result is bit-identical to lf_chi2_batch on that item alone (both GPU), graph replays track
new parameter contents, and two items are compared with the oracle at the chi^2 tolerances."""
import os

import numpy as np
import pytest

from paper_2609_08649_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available()
    from paper_2609_08649_amd import lensfield
    return lensfield


@pytest.fixture(scope="module")
def ctx(lf, tmp_path_factory):
    os.environ["LF_AUTOTUNE_CACHE"] = str(tmp_path_factory.mktemp("tune") / "autotune.txt")
    c = lf.Context(0)
    yield c
    c.close()


def _cons(m, adis):
    a = np.array([adis(m["model"]["z_d"], z) for z in m["z_fam"]])
    n = m["n_img"]
    return {"theta": m["theta"], "family": m["family"], "sig1": np.full(n, 0.5), "sig2": np.full(n, 0.5),
            "phi": np.zeros(n), "a_fam": a}


@pytest.fixture(scope="module")
def cfg3(ctx, lf):
    import torch
    cfg = W.config3(walkers_per_model=96)
    items = []
    for m in cfg["models"]:
        mod = ctx.upload_model(m["model"])
        cons = ctx.upload_constraints(_cons(m, ctx.adis))
        p = torch.as_tensor(m["params"], device="cuda")
        items.append((mod, cons, p, p.shape[0]))
    return cfg, items


@pytest.mark.parametrize("mode,prec", [(0, "mixed"), (0, "fp64"), (1, "mixed")])
def test_batch_bit_identical_to_single_items(ctx, lf, cfg3, mode, prec):
    import torch
    cfg, items = cfg3
    P = lf.LF_PREC_MIXED if prec == "mixed" else lf.LF_PREC_FP64
    b = lf.Batch(ctx, items, mode, P, autotune=True)
    outs = b.run()
    torch.cuda.synchronize()
    info = b.info()
    assert info["n_tiles"] >= len(items)
    for (m, c, p, S), (chi, fl) in zip(items, outs):
        ref, rfl, _ = ctx.chi2_batch(m, p, S, c, mode, P)
        torch.cuda.synchronize()
        assert torch.equal(chi, ref) or torch.equal(torch.isnan(chi), torch.isnan(ref)) and \
            torch.equal(chi[~torch.isnan(chi)], ref[~torch.isnan(ref)])
        assert torch.equal(fl, rfl)
    b.release()


def test_batch_graph_replays_track_new_parameters(ctx, lf, cfg3):
    import torch
    cfg, items = cfg3
    b = lf.Batch(ctx, items, 0, lf.LF_PREC_MIXED, autotune=True)
    rng = np.random.default_rng(0)
    for rep in range(3):
        for m, c, p, S in items:      # eager work between replays: new sample contents
            p.mul_(torch.as_tensor(1 + 1e-3 * rng.normal(size=tuple(p.shape)), device="cuda"))
        torch.cuda.synchronize()
        outs = b.run()
        torch.cuda.synchronize()
        for (m, c, p, S), (chi, fl) in zip(items, outs):
            ref, _, _ = ctx.chi2_batch(m, p, S, c, 0, lf.LF_PREC_MIXED)
            torch.cuda.synchronize()
            assert torch.equal(chi, ref)
    b.release()


def test_batch_items_against_oracle(ctx, lf, orc, cfg3):
    import torch
    cfg, items = cfg3
    b = lf.Batch(ctx, items, 0, lf.LF_PREC_FP64, autotune=False)
    outs = b.run()
    torch.cuda.synchronize()
    for k in (0, 5):
        m = cfg["models"][k]
        p = items[k][2].cpu().numpy()
        tabs = orc.expand_batch(m["model"], p)
        cons = _cons(m, orc.adis)
        o = orc.chi2_batch(tabs, cons)
        g = outs[k][0].cpu().numpy()
        a = cons["a_fam"][cons["family"]]
        mu = np.zeros(len(tabs))
        for s, t in enumerate(tabs):
            mm = orc.maps(t, cons["theta"][:, 0], cons["theta"][:, 1], 1.0)
            det = (1 - a * mm["p11"]) * (1 - a * mm["p22"]) - a * a * mm["p12"] ** 2
            mu[s] = np.max(np.abs(1 / det))
        tol = 1e-9 + 1e-15 * mu ** 2
        assert np.all(np.abs(g - o["chi2_src"]) <= tol * np.abs(o["chi2_src"]) + tol)
    b.release()


def test_autotune_cache_is_reused(ctx, lf, cfg3):
    cfg, items = cfg3
    b1 = lf.Batch(ctx, items, 0, lf.LF_PREC_MIXED, autotune=True)
    path = os.environ["LF_AUTOTUNE_CACHE"]
    lines = open(path).read().splitlines()
    b2 = lf.Batch(ctx, items, 0, lf.LF_PREC_MIXED, autotune=True)
    assert open(path).read().splitlines() == lines          # no new tuning entry
    assert b1.info() == b2.info()
    b1.release()
    b2.release()
