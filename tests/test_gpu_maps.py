"""GPU parity of lf_lens_maps against the FP64 oracle.

Bar: FP64 path within ~1e-10 relative (bug detector); MIXED path |d alpha| <= 1e-5",
relative mu error <= 1e-4 where |mu| < 100 (tolerances of the hot-path specification).
"""
import numpy as np
import pytest

from paper_2609_08649_amd import workloads as W

pytestmark = pytest.mark.gpu

OR2GPU = {"ax": "alpha_x", "ay": "alpha_y", "p11": "psi11", "p12": "psi12", "p22": "psi22", "kappa": "kappa",
          "gamma1": "gamma1", "gamma2": "gamma2", "detA": "detA", "mu": "mu", "beta_x": "beta_x",
          "beta_y": "beta_y", "e1": "e1", "e2": "e2", "p111": "psi111", "p112": "psi112", "p122": "psi122",
          "p222": "psi222", "f1": "f1", "f2": "f2"}
BASE = ("alpha_x", "alpha_y", "psi11", "psi12", "psi22", "kappa", "gamma1", "gamma2", "detA", "mu", "beta_x",
        "beta_y", "e1", "e2")
D3 = ("psi111", "psi112", "psi122", "psi222", "f1", "f2")


@pytest.fixture(scope="module")
def lf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2609_08649_amd import lensfield
    return lensfield


@pytest.fixture(scope="module")
def ctx(lf):
    c = lf.Context(0)
    yield c
    c.close()


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def check(gpu, orc_out, prec, d3=False, sl=slice(None), a_dis=None, a=None):
    """Compare GPU planes (numpy) with oracle columns at tolerances of the precision.  With
    a_dis given, relative mu errors are divided by the condition number of det A,
    (|A11 A22| + A12^2) / |det A| (near a singular centre det A ~ 1e9 from terms ~ 1e18).  The
    MIXED det A check needs the distance ratio of the maps (a, or a_dis)."""
    ax, ay = gpu["alpha_x"][sl], gpu["alpha_y"][sl]
    dal = np.hypot(ax - orc_out["ax"], ay - orc_out["ay"])
    amag = np.hypot(orc_out["ax"], orc_out["ay"])
    mu_o = orc_out["mu"]
    mask = np.abs(mu_o) < 100
    rel_mu = np.abs(gpu["mu"][sl][mask] - mu_o[mask]) / np.abs(mu_o[mask])
    if a_dis is not None:
        A11, A22, A12 = 1 - a_dis * orc_out["p11"], 1 - a_dis * orc_out["p22"], -a_dis * orc_out["p12"]
        cond = (np.abs(A11 * A22) + A12 * A12) / np.abs(orc_out["detA"])
        rel_mu = rel_mu / cond[mask]
    if prec == "fp64":
        assert np.max(dal / (1 + amag)) < 1e-10, np.max(dal)
        # e1, e2 = kappa -+ |gamma| are conditioned by kappa and |gamma| (they cancel near a
        # singular centre, where both exceed 1e8 while e2 stays O(1))
        eig_scale = 1 + np.abs(orc_out["kappa"]) + np.hypot(orc_out["gamma1"], orc_out["gamma2"])
        for k in ("p11", "p12", "p22", "kappa", "gamma1", "gamma2", "e1", "e2"):
            g, o = gpu[OR2GPU[k]][sl], orc_out[k]
            scale = eig_scale if k in ("e1", "e2") else 1 + np.abs(o)
            assert np.max(np.abs(g - o) / scale) < 1e-9, k
        assert np.max(rel_mu) < 1e-8
        bx = orc_out["beta_x"]
        assert np.max(np.abs(gpu["beta_x"][sl] - bx) / (1 + np.abs(bx))) < 1e-9
        if d3:
            for k in ("p111", "p112", "p122", "p222"):
                g, o = gpu[OR2GPU[k]][sl], orc_out[k]
                assert np.max(np.abs(g - o) / (1 + np.abs(o))) < 1e-7, k
            for k in ("f1", "f2"):
                g, o = gpu[k][sl], orc_out[k]
                assert np.max(np.abs(np.abs(g) - np.abs(o)) / (1 + np.abs(o))) < 1e-6, k
    else:
        assert np.max(dal) <= 1e-5, np.max(dal)
        assert np.max(rel_mu) <= 1e-4, np.max(rel_mu)
        for k in ("p11", "p12", "p22", "kappa", "gamma1", "gamma2"):
            g, o = gpu[OR2GPU[k]][sl], orc_out[k]
            assert np.max(np.abs(g - o) / (1 + np.abs(o))) < 1e-5, k
        # beta = theta - a alpha: |d beta| = a |d alpha|
        if "beta_x" in gpu:
            db = np.hypot(gpu["beta_x"][sl] - orc_out["beta_x"], gpu["beta_y"][sl] - orc_out["beta_y"])
            assert np.max(db) <= 1e-5, np.max(db)
        # det A = A11 A22 - A12^2 with A = I - a psi: first-order propagation of the psi bound
        # d psi <= 1e-5 (1 + |psi|)
        a = a if a is not None else a_dis
        if a is not None:
            A11, A22, A12 = 1 - a * orc_out["p11"], 1 - a * orc_out["p22"], -a * orc_out["p12"]
            dpsi = 1e-5 * (1 + np.maximum(np.maximum(np.abs(orc_out["p11"]), np.abs(orc_out["p22"])),
                                          np.abs(orc_out["p12"])))
            bound = a * (np.abs(A11) + np.abs(A22) + 2 * np.abs(A12)) * dpsi + 1e-12
            assert np.max(np.abs(gpu["detA"][sl] - orc_out["detA"]) / bound) <= 1.0
        # e1,2 = kappa +- |gamma|
        if "e1" in gpu:
            gm = np.hypot(orc_out["gamma1"], orc_out["gamma2"])
            scale = 1 + np.abs(orc_out["kappa"]) + gm
            for k in ("e1", "e2"):
                assert np.max(np.abs(gpu[k][sl] - orc_out[k]) / scale) < 2e-5, k
        if d3:
            for k in ("p111", "p112", "p122", "p222"):
                g, o = gpu[OR2GPU[k]][sl], orc_out[k]
                assert np.max(np.abs(g - o) / (1 + np.abs(o))) < 1e-4, k
            check_fields(gpu, orc_out, sl, 1e-4)


def check_fields(gpu, o, sl, tol):
    """Signed A3-line fields f1, f2 where they are well conditioned: |gamma| > 0.05 (the
    eigenvectors turn as d gamma / |gamma|) and the eigenvector sign rule (positive x component)
    is not ambiguous (|x component| > 1e-3).  Error scale: the third derivatives the field is
    made of, 1 + |f| + max |psi_ijk|."""
    g1, g2 = o["gamma1"], o["gamma2"]
    gm = np.hypot(g1, g2)
    vax, vay, vbx, vby = g1 + gm, g2, g2, gm - g1
    na, nb = np.hypot(vax, vay), np.hypot(vbx, vby)
    use_a = na >= nb
    vx = np.where(use_a, vax / np.where(na > 0, na, 1), vbx / np.where(nb > 0, nb, 1))
    vy = np.where(use_a, vay / np.where(na > 0, na, 1), vby / np.where(nb > 0, nb, 1))
    t3 = np.max(np.abs(np.stack([o["p111"], o["p112"], o["p122"], o["p222"]])), axis=0)
    for k, comp in (("f1", np.abs(vx)), ("f2", np.abs(vy))):
        ok = (gm > 0.05) & (comp > 1e-3)
        assert ok.sum() > 0.5 * ok.size, k
        err = np.abs(gpu[k][sl] - o[k]) / (1 + np.abs(o[k]) + t3)
        assert np.max(err[ok]) < tol, (k, np.max(err[ok]))


def _run(ctx, lf, model, params, S, pts, a, prec, outputs=BASE):
    m = ctx.upload_model(model)
    pp = _dev(params) if params is not None and model.get("n_free", 0) > 0 else None
    if not isinstance(pts, dict):
        pts = (_dev(pts[0]), _dev(pts[1]))
    res = ctx.lens_maps(m, pp, S, pts, a, lf.LF_PREC_FP64 if prec == "fp64" else lf.LF_PREC_MIXED,
                        outputs=outputs)
    import torch
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in res.items()}
    m.release()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("seed,types,ell", [(31, None, False), (32, [2, 3], True), (33, [5, 4, 0, 1], False)])
def test_maps_mixed_profiles_explicit_points(ctx, lf, orc, prec, seed, types, ell):
    model, _ = W.tiny_model(seed, n_main=6 if types is None else len(types), n_mem=37,
                            elliptical_members=ell, types=types)
    x, y = W.random_points(seed, 3001, 25.0)           # several tiles and a ragged tail
    g = _run(ctx, lf, model, None, 1, (x, y), 0.63, prec)
    o = orc.maps(orc.expand(model), x, y, 0.63)
    check({k: v[0] for k, v in g.items()}, o, prec, a=0.63)
    assert np.array_equal(g["flags"][0] & 1, o["flags"] & 1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_maps_third_derivatives_and_singularity_fields(ctx, lf, orc, prec):
    model, _ = W.tiny_model(34, n_main=2, n_mem=23, types=[2, 3], elliptical_members=True)
    model["main"].append(W._comp(W.SIS, x=W.fixed(3.0), y=W.fixed(-4.0), b=W.fixed(1.5)))
    model["main"].append(W._comp(W.POINT, x=W.fixed(-6.0), y=W.fixed(2.0), b=W.fixed(0.7)))
    model["main"].append(W._comp(W.NFW, x=W.fixed(1.0), y=W.fixed(1.0), b=W.fixed(0.2), s=W.fixed(12.0)))
    x, y = W.random_points(7, 1500, 20.0)
    g = _run(ctx, lf, model, None, 1, (x, y), 0.45, prec, outputs=BASE + D3)
    o = orc.maps(orc.expand(model), x, y, 0.45)
    check({k: v[0] for k, v in g.items()}, o, prec, d3=True, a=0.45)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_maps_many_samples_with_free_parameters(ctx, lf, orc, prec):
    model, truth = W.tiny_model(35, n_main=2, n_mem=29, types=[3, 2], free_params=True)
    rng = np.random.default_rng(1)
    S = 5
    params = np.repeat(truth[None], S, 0) * (1 + 0.01 * rng.normal(size=(S, truth.size)))
    x, y = W.random_points(8, 700, 15.0)
    g = _run(ctx, lf, model, params, S, (x, y), 0.7, prec)
    for s in range(S):
        o = orc.maps(orc.expand(model, params[s]), x, y, 0.7)
        check({k: v[s] for k, v in g.items()}, o, prec, a=0.7)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_maps_config1_grid(ctx, lf, orc, prec):
    cfg = W.config1()
    g = _run(ctx, lf, cfg["model"], None, 1, cfg["grid"], 0.6354, prec)
    x, y = W.grid_points(cfg["grid"])
    o = orc.maps(orc.expand(cfg["model"]), x, y, 0.6354)
    check({k: v[0] for k, v in g.items()}, o, prec, a=0.6354)


def test_profile_only_times_one_kernel(lf):
    """lf_profile_only: with a kernel name only that kernel's launches are timed; with NULL every
    launch again."""
    import ctypes as C
    c = lf.Context(0)
    try:
        cfg = W.config1()
        L = lf.lib()

        def counts():
            out = {}
            for k in ("maps_lean", "maps_heavy", "expand"):
                t, n = C.c_double(), C.c_int64()
                assert L.lf_profile_read(c.handle, k.encode(), C.byref(t), C.byref(n)) == 0
                out[k] = n.value
            return out

        assert L.lf_profile_only(None, b"maps_lean") != 0
        L.lf_profile_reset(c.handle)
        assert L.lf_profile_only(c.handle, b"maps_lean") == 0
        L.lf_profile_enable(c.handle, 1)
        _run(c, lf, cfg["model"], None, 1, cfg["grid"], 0.6354, "mixed")
        one = counts()
        assert one["maps_lean"] >= 1 and one["maps_heavy"] == 0 and one["expand"] == 0
        L.lf_profile_reset(c.handle)
        assert L.lf_profile_only(c.handle, None) == 0
        _run(c, lf, cfg["model"], None, 1, cfg["grid"], 0.6354, "mixed")
        every = counts()
        assert every["maps_lean"] >= 1 and every["expand"] >= 1
        L.lf_profile_enable(c.handle, 0)
    finally:
        c.close()


def test_maps_config2_full_grid(ctx, lf, orc):
    """Full 2048^2 cluster map (2 elliptical dPIE + 300 members) in the benchmark's launch
    configuration, compared with the oracle at every one of the 4.2M points."""
    cfg = W.config2(n_samples=1)
    g = _run(ctx, lf, cfg["model"], cfg["params"][:1], 1, cfg["grid"], 0.7, "mixed")
    x, y = W.grid_points(cfg["grid"])
    o = orc.maps(orc.expand(cfg["model"], cfg["params"][0]), x, y, 0.7)
    check({k: v[0] for k, v in g.items()}, o, "mixed", a=0.7)


def test_maps_edge_cases(ctx, lf, orc):
    model, _ = W.tiny_model(36, n_main=1, n_mem=3, types=[1])
    tab = orc.expand(model)
    # a point exactly on the SIS centre is flagged and its term is zero; a single point works
    x = np.array([tab[0, 1]])
    y = np.array([tab[0, 2]])
    g = _run(ctx, lf, model, None, 1, (x, y), 0.5, "fp64")
    o = orc.maps(tab, x, y, 0.5)
    assert g["flags"][0, 0] & lf.FLAG_SINGULAR and o["flags"][0] & 1
    assert abs(g["alpha_x"][0, 0] - o["ax"][0]) < 1e-12
    # a model with members only and one with main components only
    m2, _ = W.tiny_model(37, n_main=0, n_mem=12)
    xx, yy = W.random_points(9, 257, 10.0)
    check({k: v[0] for k, v in _run(ctx, lf, m2, None, 1, (xx, yy), 0.5, "fp64").items()},
          orc.maps(orc.expand(m2), xx, yy, 0.5), "fp64")
    m3, _ = W.tiny_model(38, n_main=3, n_mem=0, types=[2, 3, 0])
    check({k: v[0] for k, v in _run(ctx, lf, m3, None, 1, (xx, yy), 0.5, "mixed").items()},
          orc.maps(orc.expand(m3), xx, yy, 0.5), "mixed")


def test_maps_errors(ctx, lf):
    import torch
    model, _ = W.tiny_model(39, n_main=1, n_mem=2, types=[5])
    m = ctx.upload_model(model)
    with pytest.raises(lf.LfError) as e:
        ctx.lens_maps(m, None, 1, {"x0": 0, "y0": 0, "h": 1.0, "nx": 4, "ny": 4}, 0.5, outputs=(), flags=False)
    assert e.value.status == lf.LF_E_INVALID_ARG
    with pytest.raises(lf.LfError) as e:
        ctx.lens_maps(m, None, 1, {"x0": 0, "y0": 0, "h": -1.0, "nx": 4, "ny": 4}, 0.5)
    assert e.value.status == lf.LF_E_INVALID_ARG
    torch.cuda.synchronize()
    m.release()


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_maps_member_centres_and_near_field(ctx, lf, orc, prec):
    """Points on and around member centres: singular centres (s = 0) are flagged with a zero
    term, and the near-field region (< 3 b/q, evaluated in FP64 by the MIXED path) and its
    edge agree with the oracle for every member profile."""
    rng = np.random.default_rng(41)
    types = np.array([W.PJE, W.PJE, W.SIE, W.SIE, W.SIS, W.POINT, W.PJE, W.SIE], np.int32)
    n = types.size
    b0 = rng.uniform(0.3, 2.0, n)
    s0 = np.array([0.0, 0.08, 0.0, 0.1, 0.0, 0.0, 0.05, 0.2])
    a0 = np.array([6.0, 9.0, 0.0, 0.0, 0.0, 0.0, 7.0, 0.0])
    q = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.7, 0.6])
    pa = rng.uniform(0, np.pi, n)
    mx, my = rng.uniform(-20, 20, n), rng.uniform(-20, 20, n)
    mem = {"type": types, "x": mx, "y": my, "q": q, "pa": pa, "b0": b0, "s0": s0, "a0": a0,
           "bmul": W.fixed(1.0), "smul": W.fixed(1.0), "amul": W.fixed(1.0)}
    main = [W._comp(W.SIE, x=W.fixed(1.0), y=W.fixed(-2.0), b=W.fixed(8.0), q=W.fixed(0.8),
                    pa=W.fixed(0.3), s=W.fixed(0.5))]
    model = {"z_d": 0.5, "H0": 70.0, "Om": 0.3, "main": main, "members": mem, "n_free": 0}
    px, py = [], []
    for i in range(n):
        rn = 3.0 * b0[i] / q[i]
        for d in (0.0, 1e-9, 1e-6, 1e-3, 0.05, 0.5, 0.999 * rn, 1.001 * rn, 10.0):
            t = rng.uniform(0, 2 * np.pi)
            px.append(mx[i] + d * np.cos(t))
            py.append(my[i] + d * np.sin(t))
    px, py = np.array(px), np.array(py)
    g = _run(ctx, lf, model, None, 1, (px, py), 0.6, prec)
    o = orc.maps(orc.expand(model), px, py, 0.6)
    gg = {k: v[0] for k, v in g.items()}
    assert np.array_equal(gg["flags"] & 1, o["flags"] & 1)
    assert (o["flags"] & 1).sum() == 4          # exact centres of the s = 0 SIS/PJE/SIE and the point mass
    ok = (o["flags"] & 1) == 0
    check({k: v[ok] for k, v in gg.items()}, {k: v[ok] for k, v in o.items()}, prec, a_dis=0.6)


def _cluster_window_grid(cfg, i0, j0, n):
    g = cfg["grid"]
    return {"x0": g["x0"] + i0 * g["h"], "y0": g["y0"] + j0 * g["h"], "h": g["h"], "nx": n, "ny": n - 3}


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_maps_third_derivatives_cluster_grid(ctx, lf, orc, prec):
    """Third derivatives and A3-line fields of the cluster model (2 elliptical dPIE + 300 circular
    dPIE members: the circular members' FP32 run sums with third derivatives) on grid windows of
    the 2048^2 map: one at the cluster centre (member near fields and their edges), one at the
    field edge (members far away), with ragged block edges (n x (n - 3) vertices)."""
    cfg = W.config2(n_samples=1)
    tab = orc.expand(cfg["model"], cfg["params"][0])
    for i0, j0, n in ((900, 920, 61), (60, 1900, 45)):
        grid = _cluster_window_grid(cfg, i0, j0, n)
        g = _run(ctx, lf, cfg["model"], cfg["params"][:1], 1, grid, 0.5, prec, outputs=BASE + D3)
        x, y = W.grid_points(grid)
        o = orc.maps(tab, x, y, 0.5)
        check({k: v[0] for k, v in g.items()}, o, prec, d3=True, a=0.5)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_maps_third_derivatives_cluster_points(ctx, lf, orc, prec):
    """The same at explicit points: 3000 random points of the cluster field and 1200 points
    around member centres at the near-field radius 3 b/q and its edges."""
    cfg = W.config2(n_samples=1)
    tab = orc.expand(cfg["model"], cfg["params"][0])
    mem = tab[2:]
    rng = np.random.default_rng(43)
    x, y = W.random_points(43, 3000, 100.0)
    k = rng.integers(0, mem.shape[0], 1200)
    rn = 3.0 * mem[k, 3] / mem[k, 4]
    d = rn * rng.choice([0.5, 0.999, 1.001, 1.5, 3.0], 1200)
    t = rng.uniform(0, 2 * np.pi, 1200)
    x = np.concatenate([x, mem[k, 1] + d * np.cos(t)])
    y = np.concatenate([y, mem[k, 2] + d * np.sin(t)])
    g = _run(ctx, lf, cfg["model"], cfg["params"][:1], 1, (x, y), 0.5, prec, outputs=BASE + D3)
    o = orc.maps(tab, x, y, 0.5)
    check({k: v[0] for k, v in g.items()}, o, prec, d3=True, a=0.5)


def test_maps_local_expansion_members(ctx, lf, orc):
    """MIXED grid maps where most (block, member) pairs are summed by the blocks' local expansion
    (far circular dPIE members at least eight block radii from a 16 x 8 block centre): 150
    members of varied cut radius in several batches of 64, a ragged 200 x 120 grid, against the
    oracle at every point.  Besides the stated bounds, |d alpha| stays below 2e-6 arcsec (the
    truncation of the expansion is ~1e-9, its FP32 rounding ~3e-7)."""
    rng = np.random.default_rng(52)
    n = 150
    mem = {"type": np.full(n, W.PJE, np.int32), "x": rng.uniform(-40, 40, n), "y": rng.uniform(-40, 40, n),
           "q": np.ones(n), "pa": np.zeros(n), "b0": rng.uniform(0.2, 1.5, n), "s0": rng.uniform(0.0, 0.2, n),
           "a0": np.exp(rng.uniform(np.log(0.5), np.log(20.0), n)),
           "bmul": W.fixed(1.0), "smul": W.fixed(1.0), "amul": W.fixed(1.0)}
    main = [W._comp(W.SIE, x=W.fixed(0.5), y=W.fixed(-0.5), b=W.fixed(5.0), q=W.fixed(0.8),
                    pa=W.fixed(0.4), s=W.fixed(0.3))]
    model = {"z_d": 0.5, "H0": 70.0, "Om": 0.3, "main": main, "members": mem, "n_free": 0}
    grid = {"x0": -10.0, "y0": -6.0, "h": 0.1, "nx": 200, "ny": 120}
    # share of pairs that take the expansion (cut radius a = a0, near radius 3 b)
    h = grid["h"]
    bx = grid["x0"] + h * (np.arange((grid["nx"] + 15) // 16) * 16 + 8)
    by = grid["y0"] + h * (np.arange(grid["ny"] // 8) * 8 + 4)
    BX, BY = np.meshgrid(bx, by)
    hwx, hwy = 7.5 * h, 3.5 * h
    dx, dy = mem["x"][:, None] - BX.ravel()[None], mem["y"][:, None] - BY.ravel()[None]
    e = np.hypot(np.maximum(np.abs(dx) - hwx, 0), np.maximum(np.abs(dy) - hwy, 0))
    ex = (e >= 5 * mem["a0"][:, None]) & (e >= 3 * mem["b0"][:, None]) & (np.hypot(dx, dy) >= 8 * np.hypot(hwx, hwy))
    assert 0.3 < ex.mean() < 0.95, ex.mean()
    g = _run(ctx, lf, model, None, 1, grid, 0.6, "mixed")
    x, y = W.grid_points(grid)
    o = orc.maps(orc.expand(model), x, y, 0.6)
    gg = {k: v[0] for k, v in g.items()}
    check(gg, o, "mixed", a=0.6)
    assert np.max(np.hypot(gg["alpha_x"] - o["ax"], gg["alpha_y"] - o["ay"])) < 2e-6


def test_maps_grid_many_samples_mixed(ctx, lf, orc):
    """MIXED grid maps of several samples in one call (free parameters): each sample's member
    table, its structure-of-arrays block and its blocks' local expansions, against the oracle
    at every point of every sample."""
    model, truth = W.tiny_model(35, n_main=2, n_mem=90, types=[3, 2], free_params=True)
    rng = np.random.default_rng(3)
    S = 3
    params = np.repeat(truth[None], S, 0) * (1 + 0.02 * rng.normal(size=(S, truth.size)))
    grid = {"x0": -25.0, "y0": -18.0, "h": 0.2, "nx": 250, "ny": 180}
    g = _run(ctx, lf, model, params, S, grid, 0.7, "mixed")
    x, y = W.grid_points(grid)
    for s in range(S):
        o = orc.maps(orc.expand(model, params[s]), x, y, 0.7)
        check({k: v[s] for k, v in g.items()}, o, "mixed", a=0.7)
