"""Test inputs derived from the seeded workloads with the oracle (never with the GPU path):
image constraints are the oracle's images of selected sources plus seeded noise."""
import functools

import numpy as np

from paper_2609_08649_amd import workloads as W


def select_sources(orc, tab, grid, cand, zs, zd, n_src, min_img=2, max_img=7, H0=70.0, Om=0.3, mu_min=0.5):
    """First n_src candidates (in generation order) with min_img..max_img oracle images; only
    images with |mu| >= mu_min (observable ones) are kept as constraints."""
    out = []
    k = 0
    while len(out) < n_src and k < len(cand):
        batch = cand[k:k + 64]
        zb = zs[k:k + 64] if np.ndim(zs) else np.full(len(batch), zs)
        a = np.array([orc.adis(zd, z, H0, Om) for z in zb])
        fi = orc.find_images(tab, grid, batch, a, max_img=16)
        for j in range(len(batch)):
            n = fi["count"][j]
            keep = np.abs(fi["mu"][j, :n]) >= mu_min
            if min_img <= keep.sum() <= max_img and n <= 16 and not fi["flags"][j]:
                out.append((batch[j], zb[j], a[j], fi["theta"][j, :n][keep].copy(), fi["mu"][j, :n][keep].copy()))
                if len(out) == n_src:
                    break
        k += 64
    return out


def constraints_from_sources(srcs, n_img_total, noise, sigma):
    """Two images per family, then extra images in generation order up to n_img_total."""
    th, fam = [], []
    for f, s in enumerate(srcs):
        for t in s[3][:2]:
            th.append(t)
            fam.append(f)
    for f, s in enumerate(srcs):
        for t in s[3][2:]:
            if len(th) >= n_img_total:
                break
            th.append(t)
            fam.append(f)
    src_img = []
    for f, s in enumerate(srcs):
        src_img += [(f, k) for k in range(min(2, len(s[3])))]
    for f, s in enumerate(srcs):
        for k in range(2, len(s[3])):
            if len(src_img) >= n_img_total:
                break
            src_img.append((f, k))
    th = np.array(th) + noise[:len(th)]
    n = len(th)
    return {"theta": th, "family": np.array(fam, np.int32), "sig1": np.full(n, sigma),
            "sig2": np.full(n, sigma), "phi": np.zeros(n), "a_fam": np.array([s[2] for s in srcs]),
            "src_img": np.array(src_img, np.int32)}


def observables(orc, tab, srcs, cons, zd, seed, sig_mag=0.15, sig_dt=1.0, H0=70.0, Om=0.3):
    """Flux and delay data for a constraint set: magnitudes m0_f - 2.5 log10|mu| and delays
    T_f (|theta - beta|^2 / 2 - a psi) + t0_f at each image's true (noise-free) position, plus
    seeded Gaussian noise; about one image in six has no magnitude and one in three no delay."""
    rng = np.random.default_rng(seed)
    nf = len(srcs)
    m0 = rng.uniform(22.0, 26.0, nf)
    t0 = rng.uniform(-500.0, 500.0, nf)
    T = np.array([orc.tdscale(zd, s[1], H0, Om) for s in srcs])
    n = cons["theta"].shape[0]
    mag, dt = np.zeros(n), np.zeros(n)
    for i, (f, k) in enumerate(cons["src_img"]):
        th, mu = srcs[f][3][k], srcs[f][4][k]
        psi = orc.potential(tab, th[:1], th[1:])[0][0]
        d = th - srcs[f][0]
        mag[i] = m0[f] - 2.5 * np.log10(abs(mu))
        dt[i] = T[f] * (0.5 * d @ d - srcs[f][2] * psi) + t0[f]
    smag = np.where(rng.uniform(size=n) < 1 / 6, 0.0, sig_mag)
    sdt = np.where(rng.uniform(size=n) < 1 / 3, -1.0, sig_dt)
    return dict(cons, mag=mag + rng.normal(0, sig_mag, n), sig_mag=smag, dt=dt + rng.normal(0, sig_dt, n),
                sig_dt=sdt, tscale=T)


@functools.lru_cache(maxsize=None)
def cluster_constraints(seed=2611):
    from oracle import oracle as orc
    cfg = W.config2(seed=seed, n_samples=1)
    tab = orc.expand(cfg["model"], cfg["truth"])
    grid = {"x0": -60.0, "y0": -60.0, "h": 0.25, "nx": 480, "ny": 480}
    srcs = select_sources(orc, tab, grid, cfg["src_cand"], cfg["zs_cand"], cfg["model"]["z_d"], cfg["n_src"])
    return constraints_from_sources(srcs, cfg["n_img"], cfg["noise"], cfg["sigma_img"])


@functools.lru_cache(maxsize=None)
def cluster_observables(seed=2611):
    """The cluster constraints with flux and delay data of their sources."""
    from oracle import oracle as orc
    cfg = W.config2(seed=seed, n_samples=1)
    tab = orc.expand(cfg["model"], cfg["truth"])
    grid = {"x0": -60.0, "y0": -60.0, "h": 0.25, "nx": 480, "ny": 480}
    srcs = select_sources(orc, tab, grid, cfg["src_cand"], cfg["zs_cand"], cfg["model"]["z_d"], cfg["n_src"])
    cons = constraints_from_sources(srcs, cfg["n_img"], cfg["noise"], cfg["sigma_img"])
    return observables(orc, tab, srcs, cons, cfg["model"]["z_d"], seed + 1)


@functools.lru_cache(maxsize=None)
def _small(seed, n_src):
    from oracle import oracle as orc
    model, truth = W.tiny_model(seed, n_main=2, n_mem=25, types=[2, 3], free_params=True)
    tab = orc.expand(model, truth)
    rng = np.random.default_rng(seed)
    cand = rng.uniform(-3, 3, (400, 2))
    zs = rng.uniform(1.0, 6.0, 400)
    grid = {"x0": -30.0, "y0": -30.0, "h": 0.2, "nx": 300, "ny": 300}
    srcs = select_sources(orc, tab, grid, cand, zs, model["z_d"], n_src)
    cons = constraints_from_sources(srcs, 10 ** 6, rng.normal(0, 0.03, (200, 2)), 0.3)
    cons["sig2"] = cons["sig1"] * rng.uniform(0.5, 1.0, cons["sig1"].size)   # elliptical errors
    cons["phi"] = rng.uniform(0, np.pi, cons["sig1"].size)
    return model, truth, cons, tab, srcs


def small_constraints(seed, n_src=4):
    model, truth, cons, _, _ = _small(seed, n_src)
    return model, truth, cons


@functools.lru_cache(maxsize=None)
def small_observables(seed, n_src=4):
    """small_constraints(seed) with flux and delay data."""
    from oracle import oracle as orc
    model, truth, cons, tab, srcs = _small(seed, n_src)
    return model, truth, observables(orc, tab, srcs, cons, model["z_d"], seed + 7)


def margin_ok(orc, tab, grid, beta, a, d=1e-4):
    """Caustic-margin filter: the oracle's image count of a source is unchanged when the source
    moves by d in four directions (bit-exact counts are well posed only away from caustics)."""
    shifts = np.array([[d, 0], [-d, 0], [0, d], [0, -d]])
    base = orc.find_images(tab, grid, beta[None], np.array([a]))["count"][0]
    pert = orc.find_images(tab, grid, beta[None] + shifts, np.full(4, a))["count"]
    return bool(np.all(pert == base))


@functools.lru_cache(maxsize=None)
def config1_sources(seed=2610):
    """Config 1: five sources at z_s = 2 with 3-5 images each, away from caustics."""
    from oracle import oracle as orc
    cfg = W.config1(seed)
    tab = orc.expand(cfg["model"])
    a = orc.adis(cfg["model"]["z_d"], cfg["zs"])
    out = []
    for b in cfg["src_cand"]:
        n = orc.find_images(tab, cfg["grid"], b[None], np.array([a]))["count"][0]
        if 3 <= n <= 5 and margin_ok(orc, tab, cfg["grid"], b, a):
            out.append(b)
            if len(out) == cfg["n_src"]:
                break
    return np.array(out), a


@functools.lru_cache(maxsize=None)
def cluster_sources(seed=2611):
    """The 60 cluster sources behind the chi^2 constraints, with their distance ratios."""
    from oracle import oracle as orc
    cfg = W.config2(seed=seed, n_samples=1)
    tab = orc.expand(cfg["model"], cfg["truth"])
    grid = {"x0": -60.0, "y0": -60.0, "h": 0.25, "nx": 480, "ny": 480}
    srcs = select_sources(orc, tab, grid, cfg["src_cand"], cfg["zs_cand"], cfg["model"]["z_d"], cfg["n_src"])
    return np.array([s[0] for s in srcs]), np.array([s[1] for s in srcs]), np.array([s[2] for s in srcs])


def mu_max(orc, tabs, cons):
    """Largest |mu| over the observed images of each sample (conditioning of W = mu^T S^-1 mu)."""
    a = cons["a_fam"][cons["family"]]
    out = np.zeros(len(tabs))
    for s, t in enumerate(tabs):
        m = orc.maps(t, cons["theta"][:, 0], cons["theta"][:, 1], 1.0)
        det = (1 - a * m["p11"]) * (1 - a * m["p22"]) - a * a * m["p12"] ** 2
        out[s] = np.max(np.abs(1 / det))
    return out


def stable_image_plane(orc, tabs, cons, ref, eps=1e-5):
    """Samples whose image-plane chi^2 is well posed: in the oracle every image's Newton solve
    converges and is accepted, and the result moves by less than 1e-4 (relative) when every
    observed position is shifted by eps in three directions.  Newton basins have fractal
    boundaries; where an image does not converge within the step budget, or a 1e-5" shift
    changes which root it reaches, two correct implementations may legitimately disagree."""
    base = orc.chi2_batch(tabs, cons, img_mode=True)
    ok = (base["flags"] & 12) == 0            # every image converged and was accepted
    for d in ((eps, 0.0), (0.0, eps), (-eps, eps)):
        r = orc.chi2_batch(tabs, dict(cons, theta=cons["theta"] + np.array(d)), img_mode=True)
        ok &= np.abs(r["chi2_img"] - ref) <= 1e-4 * np.abs(ref) + 1e-4
    return ok


def mu_images(orc, tabs, cons):
    """mu at every observed image of every sample, [S, n_img]."""
    a = cons["a_fam"][cons["family"]]
    out = np.zeros((len(tabs), a.size))
    for s, t in enumerate(tabs):
        m = orc.maps(t, cons["theta"][:, 0], cons["theta"][:, 1], 1.0)
        out[s] = 1 / ((1 - a * m["p11"]) * (1 - a * m["p22"]) - a * a * m["p12"] ** 2)
    return out


def key_map(r, grid):
    """Crossings of a singularity map keyed by (row, column, edge direction, family) of their
    grid edge, so that maps of different windows of the same vertices can be matched."""
    out = {}
    for n, (p, k) in enumerate(zip(r["cross"]["pos"], r["cross"]["k"])):
        fi = (p[0] - grid["x0"]) / grid["h"] - 0.5
        fj = (p[1] - grid["y0"]) / grid["h"] - 0.5
        if abs(fj - round(fj)) < 1e-7:
            key = (int(round(fj)), int(np.floor(fi + 1e-9)), 0, int(k))
        else:
            key = (int(np.floor(fj + 1e-9)), int(round(fi)), 1, int(k))
        out[key] = n
    return out


def ainv_norm(orc, tabs, cons, theta):
    """Spectral norm of A^-1 = (I - a psi)^-1 at positions theta [S, n_img, 2] (each image at its
    family's distance ratio): how far an error in beta moves a root of the lens equation."""
    a = cons["a_fam"][cons["family"]]
    out = np.zeros(theta.shape[:2])
    for s, t in enumerate(tabs):
        m = orc.maps(t, theta[s, :, 0], theta[s, :, 1], 1.0)
        A11, A12, A22 = 1 - a * m["p11"], -a * m["p12"], 1 - a * m["p22"]
        # eigenvalues of the symmetric A: the smallest |lambda| sets the norm of A^-1
        h, d = 0.5 * (A11 + A22), np.hypot(0.5 * (A11 - A22), A12)
        out[s] = 1 / np.minimum(np.abs(h - d), np.abs(h + d))
    return out
