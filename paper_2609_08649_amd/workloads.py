"""Seeded synthetic workloads for the lens-equation hot path.

This module only draws random numbers and lays them out; it performs none of
the lensing arithmetic (no unit conversion, no deflection, no distance).  Both
the FP64 CPU oracle and the GPU library consume what it returns, each through
its own code.  Physical quantities are handed over in the units the workload
recipe states (km/s, kpc, Msun, degrees) together with a transform code that
tells the consumer how to turn them into lensing units.

Recipes follow the paper's workloads: cluster lenses made of a few main halos
plus hundreds of member galaxies on the scaling relations of Sec. 3.4
(Eq. scaling, exponents (0.25, 0.5, 0.5) as in Sec. 4.1 and Sec. 5), source
families at z_s between 1 and 9, circular positional errors of 0.5 arcsec
(Sec. 4.1), and samplers that evaluate many jittered parameter sets (Sec. 3.5).
The paper's own catalogs are not available; these synthetic inputs stand in
for them.
"""
from __future__ import annotations

import numpy as np

# Profile codes (shared vocabulary of the model description).
POINT, SIS, SIE, PJE, NFW, ENFW, SHEAR, MPOLE3 = 0, 1, 2, 3, 4, 5, 6, 7
PROFILE_NAMES = {POINT: "point", SIS: "sis", SIE: "sie", PJE: "pje", NFW: "nfw", ENFW: "enfw"}

# Transform codes: how a bound raw value becomes a lensing-unit field.
XF_NONE = 0        # already in lensing units (arcsec, radians, axis ratio)
XF_SIGMA_TO_B = 1  # velocity dispersion [km/s] -> isothermal strength b [arcsec]
XF_KPC = 2         # proper length at the lens redshift [kpc] -> arcsec
XF_EPS_TO_Q = 3    # ellipticity (1-q)/(1+q) -> axis ratio q
XF_DEG = 4         # degrees -> radians
XF_M200 = 5        # NFW M200 [Msun] (b slot); needs XF_C200 in the s slot
XF_C200 = 6        # NFW concentration c200 (s slot)

FIELDS = ("x", "y", "b", "q", "pa", "s", "a")

# Recipe constant: distance ratio used to turn a requested Einstein radius into a
# strength for the small single-plane workload (z_d=0.5, z_s=2 in flat LCDM with
# H0=70, Om=0.3).  It only sets the scale of the synthetic lens.
A_REF = 0.635


def fixed(v, xf=XF_NONE):
    return ("fixed", float(v), int(xf))


def free(i, xf=XF_NONE):
    return ("free", int(i), int(xf))


def _comp(t, **kw):
    c = {"type": int(t)}
    for f in FIELDS:
        c[f] = kw.get(f, fixed(0.0 if f not in ("q",) else 1.0))
    return c


def _members(rng, n, center, spread, field_half, lum=None, exps=(0.25, 0.5, 0.5)):
    """Circular PJE member galaxies with log-normal luminosities."""
    x = rng.normal(center[0], spread, n)
    y = rng.normal(center[1], spread, n)
    x = np.clip(x, -field_half, field_half)
    y = np.clip(y, -field_half, field_half)
    if lum is None:
        lum = np.exp(rng.normal(-1.0, 0.8, n))
        lum = np.minimum(lum, 5.0)
    return {
        "type": np.full(n, PJE, np.int32),
        "x": x.astype(np.float64), "y": y.astype(np.float64),
        "q": np.ones(n), "pa": np.zeros(n),
        "lum": lum.astype(np.float64), "exps": tuple(float(e) for e in exps),
        "b0": None, "s0": None, "a0": None,
    }


def config1(seed: int = 2610):
    """Small single-plane FP64 case: one cored SIE (theta_E = 10") plus ten
    circular truncated isothermal galaxies; 256^2 grid over 60"; five point
    sources at z_s = 2."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(0.6, 0.9)
    pa = rng.uniform(0.0, np.pi)
    b_main = 10.0 / (A_REF * np.sqrt(q))
    main = [_comp(SIE, x=fixed(0.0), y=fixed(0.0), b=fixed(b_main), q=fixed(q),
                  pa=fixed(pa), s=fixed(0.2))]
    n = 10
    thE = rng.uniform(0.3, 1.0, n)
    mem = {
        "type": np.full(n, PJE, np.int32),
        "x": rng.uniform(-30, 30, n), "y": rng.uniform(-30, 30, n),
        "q": np.ones(n), "pa": np.zeros(n),
        "lum": None, "exps": (0.0, 0.0, 0.0),
        "b0": thE / A_REF, "s0": np.zeros(n), "a0": rng.uniform(3.0, 10.0, n),
    }
    mem.update({"bmul": fixed(1.0), "smul": fixed(1.0), "amul": fixed(1.0)})
    model = {"z_d": 0.5, "H0": 70.0, "Om": 0.3, "main": main, "members": mem, "n_free": 0}
    grid = {"x0": -30.0, "y0": -30.0, "h": 60.0 / 256, "nx": 256, "ny": 256}
    # candidate sources for rejection sampling (uniform inside the caustic scale)
    cand = rng.uniform(-3.0, 3.0, (400, 2))
    return {"model": model, "params": np.zeros((1, 0)), "grid": grid,
            "src_cand": cand, "zs": 2.0, "n_src": 5, "sigma_img": 0.05,
            "noise": rng.normal(0.0, 0.05, (64, 2))}


def _cluster_model(rng, n_members, field_half=100.0, z_d=0.5, free_offset=0):
    """Two elliptical dPIE halos with free parameters + scaled members.

    Free parameter layout per main halo: x, y, sigma[km/s], s[kpc], q, pa[deg];
    then v* [km/s] and theta*_cut [arcsec] of the scaling relations."""
    truth = []
    main = []
    k = free_offset
    for _ in range(2):
        cx, cy = rng.uniform(-20, 20, 2)
        sig = rng.uniform(600, 1200)
        core = rng.uniform(5, 50)
        q = rng.uniform(0.6, 0.9)
        pa = rng.uniform(0.0, 180.0)
        main.append(_comp(PJE, x=free(k), y=free(k + 1), b=free(k + 2, XF_SIGMA_TO_B),
                          s=free(k + 3, XF_KPC), q=free(k + 4), pa=free(k + 5, XF_DEG),
                          a=fixed(1500.0, XF_KPC)))
        truth += [cx, cy, sig, core, q, pa]
        k += 6
    center = (np.mean([truth[0], truth[6]]), np.mean([truth[1], truth[7]]))
    mem = _members(rng, n_members, center, 40.0, field_half)
    mem.update({"bmul": free(k, XF_SIGMA_TO_B), "smul": fixed(0.05), "amul": free(k + 1)})
    truth += [220.0, 8.0]
    k += 2
    model = {"z_d": z_d, "H0": 70.0, "Om": 0.3, "main": main, "members": mem,
             "n_free": k}
    return model, np.array(truth)


def cluster_prior():
    """Uniform prior box of the cluster model's free parameters (layout of _cluster_model):
    per main halo x, y in [-30, 30]", sigma in [500, 1300] km/s, s in [2, 60] kpc, q in
    [0.5, 0.99], PA in [0, 180] deg; v* in [150, 300] km/s, theta*_cut in [2, 20]"."""
    lo = np.array([-30.0, -30.0, 500.0, 2.0, 0.5, 0.0] * 2 + [150.0, 2.0])
    hi = np.array([30.0, 30.0, 1300.0, 60.0, 0.99, 180.0] * 2 + [300.0, 20.0])
    return lo, hi


def jitter(rng, truth, n_samples):
    """Gaussian ball around the truth (the AIES start of Sec. 3.5): 1% relative on
    velocity dispersions, cores, v* and cut radius; 0.2" on positions; 0.02 on q;
    1 degree on PA.  Row 0 is the truth itself."""
    n = len(truth)
    out = np.repeat(truth[None, :], n_samples, axis=0).astype(np.float64)
    nmain = (n - 2) // 6
    for h in range(nmain):
        o = 6 * h
        out[1:, o + 0] += rng.normal(0, 0.2, n_samples - 1)
        out[1:, o + 1] += rng.normal(0, 0.2, n_samples - 1)
        out[1:, o + 2] *= 1 + rng.normal(0, 0.01, n_samples - 1)
        out[1:, o + 3] *= 1 + rng.normal(0, 0.01, n_samples - 1)
        out[1:, o + 4] = np.clip(out[1:, o + 4] + rng.normal(0, 0.02, n_samples - 1), 0.3, 0.99)
        out[1:, o + 5] += rng.normal(0, 1.0, n_samples - 1)
    out[1:, n - 2] *= 1 + rng.normal(0, 0.01, n_samples - 1)
    out[1:, n - 1] *= 1 + rng.normal(0, 0.01, n_samples - 1)
    return out


def config2(seed: int = 2611, n_samples: int = 1024, n_members: int = 300, grid_n: int = 2048):
    """Cluster scale, single plane: 2 elliptical dPIE + 300 circular dPIE members;
    2048^2 grid over 200"; 60 sources z~U[1,8]; 150 images; sigma_img = 0.5";
    1024 parameter samples."""
    rng = np.random.default_rng(seed)
    model, truth = _cluster_model(rng, n_members)
    params = jitter(rng, truth, n_samples)
    grid = {"x0": -100.0, "y0": -100.0, "h": 200.0 / grid_n, "nx": grid_n, "ny": grid_n}
    cand = rng.uniform(-25.0, 25.0, (4000, 2))
    zs = rng.uniform(1.0, 8.0, 4000)
    return {"model": model, "params": params, "truth": truth, "grid": grid,
            "src_cand": cand, "zs_cand": zs, "n_src": 60, "n_img": 150,
            "sigma_img": 0.5, "noise": rng.normal(0.0, 0.05, (4096, 2))}


def config3(seed: int = 2612, n_models: int = 8, walkers_per_model: int = 512):
    """Uneven batch: 8 cluster models with 50-800 halos and 40-400 image
    constraints each; 512 walkers per model."""
    rng = np.random.default_rng(seed)
    models = []
    for m in range(n_models):
        h = int(rng.integers(50, 801))
        p = int(rng.integers(40, 401))
        model, truth = _cluster_model(rng, h - 2)
        params = jitter(rng, truth, walkers_per_model)
        n_fam = int(np.ceil(p / 2.5))
        cand = rng.uniform(-25.0, 25.0, (6 * n_fam + 400, 2))
        zs = rng.uniform(1.0, 8.0, 6 * n_fam + 400)
        # constraint set: p positions in n_fam families (>= 2 images each), circular 0.5" errors,
        # one source redshift per family
        fam = np.concatenate([np.repeat(np.arange(n_fam), 2),
                              rng.integers(0, n_fam, max(0, p - 2 * n_fam))])[:p].astype(np.int32)
        theta = rng.uniform(-40.0, 40.0, (p, 2))
        models.append({"model": model, "params": params, "truth": truth,
                       "n_img": p, "n_fam": n_fam, "src_cand": cand, "zs_cand": zs,
                       "sigma_img": 0.5, "noise": rng.normal(0.0, 0.05, (p + 64, 2)),
                       "theta": theta, "family": fam, "z_fam": rng.uniform(1.0, 8.0, n_fam)})
    return {"models": models}


def config4(seed: int = 2613, grid_n: int = 4096, members=(298, 59, 39)):
    """Multi-plane: planes at z = 0.3, 0.6, 1.2 with eNFW halos plus dPIE members
    (300/60/40 halos); flat LCDM H0=70, Om=0.3; grid 4096^2 over 200"."""
    rng = np.random.default_rng(seed)
    zp = [0.3, 0.6, 1.2]
    n_nfw = [2, 1, 1]
    mranges = [(3e14, 1.5e15), (5e13, 2e14), (2e13, 1e14)]
    planes = []
    for j in range(3):
        off = rng.uniform(-30, 30, 2) if j > 0 else np.zeros(2)
        main = []
        for _ in range(n_nfw[j]):
            lo, hi = mranges[j]
            m200 = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
            c200 = rng.uniform(4.0, 7.0)
            q = rng.uniform(0.6, 0.9)
            pa = rng.uniform(0.0, np.pi)
            cx, cy = off + rng.uniform(-15, 15, 2)
            main.append(_comp(ENFW, x=fixed(cx), y=fixed(cy), b=fixed(m200, XF_M200),
                              s=fixed(c200, XF_C200), q=fixed(q), pa=fixed(pa)))
        mem = _members(rng, members[j], off, 40.0, 100.0)
        mem.update({"bmul": fixed(220.0 if j == 0 else 180.0, XF_SIGMA_TO_B),
                    "smul": fixed(0.05), "amul": fixed(8.0)})
        planes.append({"z_d": zp[j], "H0": 70.0, "Om": 0.3, "main": main,
                       "members": mem, "n_free": 0})
    grid = {"x0": -100.0, "y0": -100.0, "h": 200.0 / grid_n, "nx": grid_n, "ny": grid_n}
    cand = rng.uniform(-25.0, 25.0, (4000, 2))
    zs = rng.uniform(1.5, 9.0, 4000)
    return {"planes": planes, "z_planes": np.array(zp), "grid": grid,
            "zs_maps": np.array([1.5, 3.0, 6.0, 9.0]), "src_cand": cand, "zs_cand": zs,
            "n_src": 60}


def config5_requests(seed: int = 2614, rate: float = 100.0, duration: float = 10.0,
                     n_models: int = 8):
    """Serving mix: Poisson arrivals; 80% chi^2 requests (S ~ U{1..256}) on one
    of n_models resident cluster models, 15% magnification maps 2048^2, 5%
    singularity maps 4096^2 (a_dis <= 0.5)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        u = rng.uniform()
        if u < 0.80:
            reqs.append({"t": t, "kind": "chi2", "model": int(rng.integers(n_models)),
                         "S": int(rng.integers(1, 257)), "seed": int(rng.integers(1 << 31))})
        elif u < 0.95:
            reqs.append({"t": t, "kind": "mu_map", "model": int(rng.integers(n_models)),
                         "n": 2048, "a_dis": float(rng.uniform(0.3, 0.9))})
        else:
            reqs.append({"t": t, "kind": "sing_map", "model": int(rng.integers(n_models)),
                         "n": 4096, "a_dis": float(rng.uniform(0.2, 0.5))})
    return reqs


def tiny_model(seed: int, n_main: int = 2, n_mem: int = 6, elliptical_members: bool = False,
               types=None, free_params: bool = False):
    """Small mixed-profile single-plane models for CPU tests and fast parity cases."""
    rng = np.random.default_rng(seed)
    main = []
    truth = []
    k = 0
    types = types if types is not None else [SIE, PJE, ENFW, NFW, SIS, POINT]
    for i in range(n_main):
        t = types[i % len(types)]
        cx, cy = rng.uniform(-8, 8, 2)
        q = rng.uniform(0.55, 0.95)
        pa = rng.uniform(0, np.pi)
        if t == POINT:
            c = _comp(POINT, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(1, 3)))
        elif t == SIS:
            c = _comp(SIS, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(1, 4)))
        elif t == SIE:
            c = _comp(SIE, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(4, 12)), q=fixed(q),
                      pa=fixed(pa), s=fixed(rng.uniform(0.1, 2.0)))
        elif t == PJE:
            c = _comp(PJE, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(3, 10)), q=fixed(q),
                      pa=fixed(pa), s=fixed(rng.uniform(0.2, 2.0)), a=fixed(rng.uniform(15, 60)))
        elif t == SHEAR:
            c = _comp(SHEAR, b=fixed(rng.uniform(0.02, 0.1)), pa=fixed(pa))
        elif t == MPOLE3:
            c = _comp(MPOLE3, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(0.01, 0.05)), pa=fixed(pa))
        elif t == NFW:
            c = _comp(NFW, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(0.1, 0.4)),
                      s=fixed(rng.uniform(10, 40)))
        else:
            c = _comp(ENFW, x=fixed(cx), y=fixed(cy), b=fixed(rng.uniform(0.1, 0.4)), q=fixed(q),
                      pa=fixed(pa), s=fixed(rng.uniform(10, 40)))
        if free_params and t in (SIE, PJE):
            vals = [cx, cy, c["b"][1], c["q"][1], c["pa"][1]]
            c["x"], c["y"], c["b"], c["q"], c["pa"] = (free(k), free(k + 1), free(k + 2),
                                                       free(k + 3), free(k + 4))
            truth += vals
            k += 5
        main.append(c)
    mem = _members(rng, n_mem, (0.0, 0.0), 10.0, 30.0)
    if elliptical_members:
        mem["q"] = rng.uniform(0.6, 0.95, n_mem)
        mem["pa"] = rng.uniform(0, np.pi, n_mem)
    if free_params:
        mem.update({"bmul": free(k, XF_SIGMA_TO_B), "smul": fixed(0.05), "amul": free(k + 1)})
        truth += [200.0, 6.0]
        k += 2
    else:
        mem.update({"bmul": fixed(200.0, XF_SIGMA_TO_B), "smul": fixed(0.05), "amul": fixed(6.0)})
    model = {"z_d": 0.5, "H0": 70.0, "Om": 0.3, "main": main, "members": mem, "n_free": k}
    return model, np.array(truth, dtype=np.float64)


def grid_points(grid):
    """Pixel-centre coordinates of a grid spec: x0 + (i + 1/2) h (row-major, y outer)."""
    xs = grid["x0"] + (np.arange(grid["nx"]) + 0.5) * grid["h"]
    ys = grid["y0"] + (np.arange(grid["ny"]) + 0.5) * grid["h"]
    X, Y = np.meshgrid(xs, ys)
    return X.ravel().copy(), Y.ravel().copy()


def random_points(seed: int, n: int, half: float):
    rng = np.random.default_rng(seed)
    return rng.uniform(-half, half, n), rng.uniform(-half, half, n)
