"""The allocation-free chi^2 entry point (lf_chi2_batch_noalloc) against lf_chi2_batch: the same
kernels on the same layouts, so every output must be bit-identical, for calls in a row that
reuse the static scratch (a large call, then smaller ones); the context allocates nothing during
those calls; a workspace larger than the scratch is rejected before anything runs."""
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


def _run(fn, m, params, S, c, mode, prec):
    import torch
    pp = torch.as_tensor(params, device="cuda") if params is not None else None
    chi, fl, bm = fn(m, pp, S, c, mode, prec, want_beta=True)
    torch.cuda.synchronize()
    return chi.cpu().numpy(), fl.cpu().numpy(), bm.cpu().numpy()


def _same(a, b):
    for x, y in zip(a, b):
        assert np.array_equal(x, y, equal_nan=True)


def test_noalloc_matches_chi2_batch(lf):
    cfg = W.config2(n_samples=1024)
    cluster = lensdata.cluster_constraints()
    small_model, truth, small_cons = lensdata.small_constraints(41)
    rng = np.random.default_rng(7)
    small_params = np.repeat(truth[None], 37, 0)
    small_params[1:] *= 1 + 0.003 * rng.normal(size=(36, truth.size))
    ctx = lf.Context(0)
    try:
        mc, cc = ctx.upload_model(cfg["model"]), ctx.upload_constraints(cluster)
        ms, cs = ctx.upload_model(small_model), ctx.upload_constraints(small_cons)
        # calls in a row on the shared scratch: the full cluster case, then smaller ones
        cases = [(mc, cfg["params"], 1024, cc, 0, lf.LF_PREC_MIXED),
                 (ms, small_params, 37, cs, 1, lf.LF_PREC_FP64),
                 (mc, cfg["params"][:200], 200, cc, 1, lf.LF_PREC_MIXED),
                 (ms, small_params[:5], 5, cs, 0, lf.LF_PREC_MIXED)]
        before = ctx.device_bytes
        got = [_run(ctx.chi2_batch_noalloc, *k) for k in cases]
        assert ctx.device_bytes == before           # no workspace was allocated
        with pytest.raises(lf.LfError) as ei:         # 4096 x 150 (sample, image) pairs > 32 MiB
            big = np.repeat(cfg["params"], 4, 0)
            _run(ctx.chi2_batch_noalloc, mc, big, big.shape[0], cc, 0, lf.LF_PREC_MIXED)
        assert ei.value.status == lf.LF_E_OUT_OF_BUDGET and "scratch" in str(ei.value)
        assert ctx.device_bytes == before
        ref = [_run(ctx.chi2_batch, *k) for k in cases]
        for g, r in zip(got, ref):
            _same(g, r)
        assert np.all(np.isfinite(got[0][0])) and np.all(np.isfinite(got[1][0]))
        # and again after the existing entry point has run (the scratch keeps older contents)
        again = _run(ctx.chi2_batch_noalloc, *cases[2])
        _same(again, ref[2])
        for h in (cc, cs):
            h.release()
        for h in (mc, ms):
            h.release()
    finally:
        ctx.close()
