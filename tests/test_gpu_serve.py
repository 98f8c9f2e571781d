"""Serving runtime: continuous batching with HBM-budget admission.  Each result is the same
(bit-identical) alone and in a mix with other chi^2 requests and maps; requests that do not fit
wait for memory; an over-budget request fails alone; a bad request does not affect others."""
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
def env(lf):
    ctx = lf.Context(0)
    cfg = W.config2(n_samples=512)
    m = ctx.upload_model(cfg["model"])
    cons = ctx.upload_constraints(lensdata.cluster_constraints())
    c3 = W.config3(n_models=2, walkers_per_model=64)["models"][1]
    m2 = ctx.upload_model(c3["model"])
    a = np.array([ctx.adis(0.5, z) for z in c3["z_fam"]])
    n = c3["n_img"]
    cons2 = ctx.upload_constraints({"theta": c3["theta"], "family": c3["family"], "sig1": np.full(n, 0.5),
                                    "sig2": np.full(n, 0.5), "phi": np.zeros(n), "a_fam": a})
    yield ctx, cfg, m, cons, c3, m2, cons2
    ctx.close()


def _requests(cfg, c3):
    rng = np.random.default_rng(3)
    reqs = []
    for k in range(10):
        S = int(rng.integers(1, 120))
        lo = int(rng.integers(0, 512 - S))
        if k % 3 == 2:
            reqs.append(("chi2b", c3["params"][:S], int(rng.integers(0, 2))))
        else:
            reqs.append(("chi2", cfg["params"][lo:lo + S], int(rng.integers(0, 2))))
    grid = {"x0": -50.0, "y0": -50.0, "h": 100.0 / 384, "nx": 384, "ny": 300}
    reqs.insert(3, ("mu", grid, 0.6))
    reqs.insert(7, ("sing", grid, 0.4))
    return reqs


def _submit(srv, lf, env, rq):
    ctx, cfg, m, cons, c3, m2, cons2 = env
    kind = rq[0]
    if kind == "chi2":
        return srv.submit_chi2(m, cons, rq[1], rq[2], lf.LF_PREC_MIXED)
    if kind == "chi2b":
        return srv.submit_chi2(m2, cons2, rq[1], rq[2], lf.LF_PREC_MIXED)
    k = lf.LF_REQ_MU_MAP if kind == "mu" else lf.LF_REQ_SING_MAP
    t, out = srv.submit_map(m, cfg["params"][0], rq[1], rq[2], k, lf.LF_PREC_MIXED)
    return t, out, None


def test_same_alone_and_in_the_mix(lf, env):
    reqs = _requests(env[1], env[4])
    srv = lf.Server(env[0], 2 << 30, n_streams=3, map_chunk_rows=64)
    alone = []
    for rq in reqs:
        t, out, fl = _submit(srv, lf, env, rq)
        st, lat = srv.wait(t)
        assert st == 1 and lat > 0
        alone.append((out.clone(), None if fl is None else fl.clone()))
    tickets = [_submit(srv, lf, env, rq) for rq in reqs]       # all at once: batched and overlapped
    for (t, out, fl), (a_out, a_fl) in zip(tickets, alone):
        st, _ = srv.wait(t)
        assert st == 1
        assert np.array_equal(out.numpy(), a_out.numpy(), equal_nan=True)
        if fl is not None:
            assert np.array_equal(fl.numpy(), a_fl.numpy())
    s = srv.stats()
    assert s["count"] == 2 * len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0
    assert srv.stats(lf.LF_REQ_CHI2)["count"] == 2 * (len(reqs) - 2)
    srv.stop()


def test_served_maps_equal_direct_maps(lf, env):
    import torch
    ctx, cfg, m = env[0], env[1], env[2]
    grid = {"x0": -50.0, "y0": -50.0, "h": 100.0 / 384, "nx": 384, "ny": 300}
    srv = lf.Server(ctx, 1 << 30, n_streams=2, map_chunk_rows=37)       # ragged last chunk
    t, out = srv.submit_map(m, cfg["params"][0], grid, 0.6, lf.LF_REQ_MU_MAP, lf.LF_PREC_MIXED)
    t2, out2 = srv.submit_map(m, cfg["params"][0], grid, 0.4, lf.LF_REQ_SING_MAP, lf.LF_PREC_MIXED)
    assert srv.wait(t)[0] == 1 and srv.wait(t2)[0] == 1
    srv.stop()
    p = torch.as_tensor(cfg["params"][:1], device="cuda")
    d = ctx.lens_maps(m, p, 1, grid, 0.6, lf.LF_PREC_MIXED, outputs=("mu",))
    d2 = ctx.lens_maps(m, p, 1, grid, 0.4, lf.LF_PREC_MIXED, outputs=lf.SING_PLANES)
    torch.cuda.synchronize()
    assert np.array_equal(out.numpy()[0], d["mu"].cpu().numpy()[0])
    for k, name in enumerate(lf.SING_PLANES):
        assert np.array_equal(out2.numpy()[k], d2[name].cpu().numpy()[0]), name


def test_device_resident_map_results(lf, env):
    """Maps served into caller-owned device memory (no copy to the host; their output planes are
    not charged to the budget) equal the host-copied results bit for bit, beside chi^2 requests;
    a request with both or neither output is refused."""
    import torch
    ctx, cfg, m, cons = env[0], env[1], env[2], env[3]
    grid = {"x0": -50.0, "y0": -50.0, "h": 100.0 / 384, "nx": 384, "ny": 300}
    P = grid["nx"] * grid["ny"]
    # 1 MB of planes per singularity map, beyond a budget that holds the rest of the request
    srv = lf.Server(ctx, 6 << 20, n_streams=3, map_chunk_rows=41)
    dev = torch.full((6, P), np.nan, dtype=torch.float64, device="cuda")
    dmu = torch.full((1, P), np.nan, dtype=torch.float64, device="cuda")
    c = srv.submit_chi2(m, cons, cfg["params"][:64], 0)
    t1, _ = srv.submit_map(m, cfg["params"][0], grid, 0.4, lf.LF_REQ_SING_MAP, lf.LF_PREC_MIXED, out=dev)
    t2, _ = srv.submit_map(m, cfg["params"][0], grid, 0.6, lf.LF_REQ_MU_MAP, lf.LF_PREC_FP64, out=dmu)
    assert srv.wait(t1)[0] == 1 and srv.wait(t2)[0] == 1 and srv.wait(c[0])[0] == 1
    srv.stop()
    srv = lf.Server(ctx, 1 << 30, n_streams=2, map_chunk_rows=41)
    h1 = srv.submit_map(m, cfg["params"][0], grid, 0.4, lf.LF_REQ_SING_MAP, lf.LF_PREC_MIXED)
    h2 = srv.submit_map(m, cfg["params"][0], grid, 0.6, lf.LF_REQ_MU_MAP, lf.LF_PREC_FP64)
    assert srv.wait(h1[0])[0] == 1 and srv.wait(h2[0])[0] == 1
    req = lf.lf_request(lf.LF_REQ_MU_MAP, 1, m.handle.value, None, None, 0, lf.LF_PREC_MIXED,
                        lf.lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"]), 0.6,
                        h2[1].data_ptr(), None, dmu.data_ptr(), None)
    with pytest.raises(lf.LfError):
        srv._submit(req, None)
    srv.stop()
    torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), h1[1].numpy())
    assert np.array_equal(dmu.cpu().numpy(), h2[1].numpy())


def test_budget_admission_and_errors(lf, env):
    ctx, cfg, m, cons = env[0], env[1], env[2], env[3]
    # ~4.3 MB per 256-sample request against a 12 MB budget: requests queue and all finish
    srv = lf.Server(ctx, 12 << 20, n_streams=2)
    subs = [srv.submit_chi2(m, cons, cfg["params"][k * 32:k * 32 + 256], 0) for k in range(8)]
    bad_params = cfg["params"][:5].copy()
    bad_params[2, 4] = np.nan
    bad = srv.submit_chi2(m, cons, bad_params, 0)
    huge = srv.submit_chi2(m, cons, np.repeat(cfg["params"][:1], 4000, 0), 0)   # > budget
    for t, out, fl in subs:
        assert srv.wait(t)[0] == 1
        assert np.all(np.isfinite(out.numpy()))
    assert srv.wait(bad[0])[0] == 1
    assert np.isnan(bad[1].numpy()[2]) and bad[2].numpy()[2] & lf.FLAG_INVALID
    assert np.all(np.isfinite(bad[1].numpy()[[0, 1, 3, 4]]))
    assert srv.wait(huge[0])[0] == lf.LF_E_OUT_OF_BUDGET
    srv.stop()
    # a malformed request is refused at submission
    srv = lf.Server(ctx, 1 << 30, n_streams=2)
    with pytest.raises(lf.LfError):
        srv.submit_chi2(m, cons, np.zeros((0, 14)), 0)
    srv.stop()
