"""ctypes wrapper around the FP64 CPU oracle (lf_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lf_oracle.cpp")
# LF_ORACLE_SANITIZE=1: a separate build with AddressSanitizer and UndefinedBehaviorSanitizer
# (run the Python process with the sanitizer runtimes preloaded, see sanitize.sh)
_SAN = os.environ.get("LF_ORACLE_SANITIZE") == "1"
_SO = os.path.join(_HERE, "liblf_oracle_san.so" if _SAN else "liblf_oracle.so")
_lib = None

FIELDS = ("x", "y", "b", "q", "pa", "s", "a")
F_SINGULAR, F_GSING, F_NOCONV, F_REJECT, F_MERGED, F_OVERFLOW, F_UMBILIC = 1, 2, 4, 8, 16, 32, 64
MAP_COLS = ("ax", "ay", "p11", "p12", "p22", "p111", "p112", "p122", "p222", "kappa", "gamma1",
            "gamma2", "detA", "mu", "beta_x", "beta_y", "e1", "e2", "f1", "f2")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (IEEE double, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
               "-g"] if _SAN else []
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off"] + san + ["-o", tmp, _SRC, "-lpthread"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        d, i, dp, ip = C.c_double, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc_dist.restype = d
        L.orc_dist.argtypes = [d, d, d, d]
        L.orc_comoving.restype = d
        L.orc_comoving.argtypes = [d, d, d, d]
        L.orc_adis.restype = d
        L.orc_adis.argtypes = [d, d, d, d]
        L.orc_sigma_to_b.restype = d
        L.orc_sigma_to_b.argtypes = [d]
        L.orc_orient.restype = i
        L.orc_orient.argtypes = [d] * 6
        L.orc_tdscale.restype = d
        L.orc_tdscale.argtypes = [d, d, d, d]
        _lib = L
    return _lib


def _p(a, ct=C.c_double):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def nthreads_default():
    """Worker threads: the CPUs this process may use, at most its CPU share (OMP_NUM_THREADS, or 16
    where that is unset: one GPU's share of a GPU host)."""
    share = int(os.environ.get("OMP_NUM_THREADS") or 16)
    return max(1, min(share, len(os.sched_getaffinity(0))))


# --------------------------------------------------------------------------- cosmology
def dist(z1, z2, H0=70.0, Om=0.3):
    return lib().orc_dist(z1, z2, H0, Om)


def comoving(z1, z2, H0=70.0, Om=0.3):
    return lib().orc_comoving(z1, z2, H0, Om)


def adis(zd, zs, H0=70.0, Om=0.3):
    return lib().orc_adis(zd, zs, H0, Om)


def sigma_to_b(sigma):
    return lib().orc_sigma_to_b(sigma)


def nfw_params(H0, Om, zd, m200, c200):
    ks, rs = C.c_double(), C.c_double()
    lib().orc_nfw_params(C.c_double(H0), C.c_double(Om), C.c_double(zd), C.c_double(m200),
                         C.c_double(c200), C.byref(ks), C.byref(rs))
    return ks.value, rs.value


# --------------------------------------------------------------------------- model expansion
def _bind(b):
    kind, v, xf = b
    if kind == "fixed":
        return (0, 0, int(xf)), float(v)
    return (1, int(v), int(xf)), 0.0


def expand(model, params_row=None):
    """Halo table [H, 8] (type, x, y, b, q, pa, s, a) for one parameter sample."""
    main = model["main"]
    mem = model["members"]
    nm = len(main)
    mt = _i32([c["type"] for c in main]) if nm else np.zeros(1, np.int32)
    mb = np.zeros(max(1, nm * 7 * 3), np.int32)
    mv = np.zeros(max(1, nm * 7), np.float64)
    for m, c in enumerate(main):
        for k, f in enumerate(FIELDS):
            t, v = _bind(c[f])
            mb[(m * 7 + k) * 3:(m * 7 + k) * 3 + 3] = t
            mv[m * 7 + k] = v
    n = len(mem["x"])
    mtyp = _i32(mem["type"])
    mx, my = _f64(mem["x"]), _f64(mem["y"])
    mq = _f64(mem["q"]) if mem.get("q") is not None else np.ones(n)
    mpa = _f64(mem["pa"]) if mem.get("pa") is not None else np.zeros(n)
    lum = mem.get("lum")
    exps = _f64(mem.get("exps", (0, 0, 0)))
    if lum is not None:
        lum = _f64(lum)
        b0 = s0 = a0 = np.zeros(max(1, n))
    else:
        b0, s0, a0 = _f64(mem["b0"]), _f64(mem["s0"]), _f64(mem["a0"])
    ub = np.zeros(9, np.int32)
    uv = np.zeros(3)
    for k, key in enumerate(("bmul", "smul", "amul")):
        t, v = _bind(mem[key])
        ub[3 * k:3 * k + 3] = t
        uv[k] = v
    nf = int(model.get("n_free", 0))
    pr = _f64(params_row if params_row is not None and nf > 0 else np.zeros(max(1, nf)))
    out = np.zeros((nm + n, 8))
    rc = lib().orc_expand(
        C.c_int(nm), _p(mt, C.c_int), _p(mb, C.c_int), _p(mv), C.c_int(n), _p(mtyp, C.c_int),
        _p(mx), _p(my), _p(mq), _p(mpa), _p(lum) if lum is not None else None, _p(exps),
        _p(b0), _p(s0), _p(a0), _p(ub, C.c_int), _p(uv), C.c_double(model["z_d"]),
        C.c_double(model["H0"]), C.c_double(model["Om"]), _p(pr), C.c_int(nf), _p(out))
    if rc != 0:
        raise ValueError("oracle expand failed (%d)" % rc)
    return out


def expand_batch(model, params):
    return np.stack([expand(model, params[s]) for s in range(params.shape[0])])


# --------------------------------------------------------------------------- maps
def maps(tab, px, py, a_dis, nthreads=None):
    tab = _f64(tab)
    px, py = _f64(px), _f64(py)
    P = px.size
    out = np.zeros((P, 20))
    fl = np.zeros(P, np.int32)
    lib().orc_maps(_p(tab), C.c_int(tab.shape[0]), _p(px), _p(py), C.c_int(P), C.c_double(a_dis),
                   _p(out), _p(fl, C.c_int), C.c_int(nthreads or nthreads_default()))
    d = {k: out[:, i].copy() for i, k in enumerate(MAP_COLS)}
    d["flags"] = fl
    return d


def alpha(tab, px, py, nthreads=None):
    tab = _f64(tab)
    px, py = _f64(px), _f64(py)
    ax, ay = np.zeros(px.size), np.zeros(px.size)
    lib().orc_alpha(_p(tab), C.c_int(tab.shape[0]), _p(px), _p(py), C.c_int(px.size), _p(ax), _p(ay),
                    C.c_int(nthreads or nthreads_default()))
    return ax, ay


# --------------------------------------------------------------------------- multi-plane
def _plane_ptrs(tabs):
    tabs = [_f64(t) for t in tabs]
    arr = (C.POINTER(C.c_double) * len(tabs))(*[_p(t) for t in tabs])
    Hs = _i32([t.shape[0] for t in tabs])
    return tabs, arr, Hs


def multiplane(tabs, zp, zs, px, py, H0=70.0, Om=0.3, nthreads=None, want_planes=False):
    tabs, arr, Hs = _plane_ptrs(tabs)
    zp, zs = _f64(zp), _f64(np.atleast_1d(zs))
    px, py = _f64(px), _f64(py)
    P, nz, N = px.size, zs.size, len(tabs)
    beta = np.zeros((nz, P, 2))
    A = np.zeros((nz, P, 4))
    mu = np.zeros((nz, P))
    alp = np.zeros((N, P, 2)) if want_planes else None
    fl = np.zeros(P, np.int32)
    lib().orc_multiplane(C.c_int(N), arr, _p(Hs, C.c_int), _p(zp), C.c_double(H0), C.c_double(Om),
                         _p(zs), C.c_int(nz), _p(px), _p(py), C.c_int(P), _p(beta), _p(A), _p(mu),
                         _p(alp) if want_planes else None, _p(fl, C.c_int),
                         C.c_int(nthreads or nthreads_default()))
    out = {"beta": beta, "A": A, "mu": mu, "flags": fl}
    if want_planes:
        out["alpha_planes"] = alp
    return out


# --------------------------------------------------------------------------- chi^2
def chi2_batch(tabs, cons, img_mode=False, newton_tol=1e-9, nthreads=None):
    """tabs: [S, H, 8]; cons: dict(theta [n,2], family [n], sig1, sig2, phi [n], a_fam [n_fam])."""
    tabs = _f64(tabs)
    S, H = tabs.shape[0], tabs.shape[1]
    th = _f64(cons["theta"])
    fam = _i32(cons["family"])
    s1, s2, phi = _f64(cons["sig1"]), _f64(cons["sig2"]), _f64(cons["phi"])
    afam = _f64(cons["a_fam"])
    n, nf = fam.size, afam.size
    cs, ci = np.zeros(S), np.zeros(S)
    fl = np.zeros(S, np.int32)
    bm = np.zeros((S, nf, 2))
    tm = np.zeros((S, n, 2))
    ifl = np.zeros((S, n), np.int32)
    lib().orc_chi2_batch(_p(tabs), C.c_int(S), C.c_int(H), _p(th), _p(fam, C.c_int), _p(s1), _p(s2),
                         _p(phi), C.c_int(n), _p(afam), C.c_int(nf), C.c_int(1 if img_mode else 0),
                         C.c_double(newton_tol), _p(cs), _p(ci), _p(fl, C.c_int), _p(bm), _p(tm),
                         _p(ifl, C.c_int), C.c_int(nthreads or nthreads_default()))
    return {"chi2_src": cs, "chi2_img": ci if img_mode else None, "flags": fl,
            "beta_model": bm, "theta_model": tm, "img_flags": ifl if img_mode else None}


def potential(tab, px, py, nthreads=None):
    """Lensing potential psi (a_dis-free; each profile up to its own constant) at points."""
    tab = _f64(tab)
    px, py = _f64(px), _f64(py)
    P = px.size
    pot = np.zeros(P)
    fl = np.zeros(P, np.int32)
    lib().orc_potential(_p(tab), C.c_int(tab.shape[0]), _p(px), _p(py), C.c_int(P), _p(pot), _p(fl, C.c_int),
                        C.c_int(nthreads or nthreads_default()))
    return pot, fl


def tdscale(zd, zs, H0=70.0, Om=0.3):
    """(1+z_d)/c D_d D_s/D_ds (1 arcsec)^2 in days per arcsec^2."""
    return lib().orc_tdscale(C.c_double(zd), C.c_double(zs), C.c_double(H0), C.c_double(Om))


def chi2_obs(tabs, cons, img_mode=False, newton_tol=1e-9, nthreads=None):
    """Position, flux and time-delay chi^2 terms: cons may carry mag, sig_mag (per image),
    dt, sig_dt (per image) and tscale (per family); an image enters a term where its error is
    positive."""
    tabs = _f64(tabs)
    S, H = tabs.shape[0], tabs.shape[1]
    th = _f64(cons["theta"])
    fam = _i32(cons["family"])
    s1, s2, phi = _f64(cons["sig1"]), _f64(cons["sig2"]), _f64(cons["phi"])
    afam = _f64(cons["a_fam"])
    n, nf = fam.size, afam.size
    opt = lambda k: _f64(cons[k]) if cons.get(k) is not None else None
    mag, smag, dt, sdt, tsc = opt("mag"), opt("sig_mag"), opt("dt"), opt("sig_dt"), opt("tscale")
    cp, cf, ct = np.zeros(S), np.zeros(S), np.zeros(S)
    fl = np.zeros(S, np.int32)
    lib().orc_chi2_obs(_p(tabs), C.c_int(S), C.c_int(H), _p(th), _p(fam, C.c_int), _p(s1), _p(s2), _p(phi),
                       C.c_int(n), _p(afam), C.c_int(nf), C.c_int(1 if img_mode else 0), C.c_double(newton_tol),
                       _p(mag) if mag is not None else None, _p(smag) if smag is not None else None,
                       _p(dt) if dt is not None else None, _p(sdt) if sdt is not None else None,
                       _p(tsc) if tsc is not None else None, _p(cp), _p(cf), _p(ct), _p(fl, C.c_int),
                       C.c_int(nthreads or nthreads_default()))
    return {"pos": cp, "flux": cf, "td": ct, "total": cp + cf + ct, "flags": fl}


# --------------------------------------------------------------------------- image finder
def _finder_out(n_src, max_img, max_cand):
    return (np.zeros((n_src, max_img, 2)), np.zeros((n_src, max_img)), np.zeros(n_src, np.int32),
            np.zeros(n_src, np.int32), np.zeros(max_cand, np.int32), np.zeros(max_cand, np.int32),
            np.zeros(max_cand, np.int32), C.c_int(0))


def find_images(tab, grid, beta, a_src, max_img=16, max_cand=100000, nthreads=None):
    tab = _f64(tab)
    beta = _f64(beta).reshape(-1, 2)
    a_src = _f64(np.broadcast_to(a_src, (beta.shape[0],)))
    ns = beta.shape[0]
    th, mu, cnt, fl, cs, ct, cst, nc = _finder_out(ns, max_img, max_cand)
    lib().orc_find_images(_p(tab), C.c_int(tab.shape[0]), C.c_double(grid["x0"]), C.c_double(grid["y0"]),
                          C.c_double(grid["h"]), C.c_int(grid["nx"]), C.c_int(grid["ny"]), _p(beta),
                          _p(a_src), C.c_int(ns), C.c_int(max_img), _p(th), _p(mu), _p(cnt, C.c_int),
                          _p(fl, C.c_int), _p(cs, C.c_int), _p(ct, C.c_int), _p(cst, C.c_int),
                          C.c_int(max_cand), C.byref(nc), C.c_int(nthreads or nthreads_default()))
    k = min(nc.value, max_cand)
    return {"theta": th, "mu": mu, "count": cnt, "flags": fl,
            "cand_src": cs[:k], "cand_tri": ct[:k], "cand_status": cst[:k], "n_cand": nc.value}


def find_images_mp(tabs, zp, grid, beta, zs, H0=70.0, Om=0.3, max_img=16, max_cand=100000, nthreads=None):
    tabs, arr, Hs = _plane_ptrs(tabs)
    zp = _f64(zp)
    beta = _f64(beta).reshape(-1, 2)
    zs = _f64(np.broadcast_to(zs, (beta.shape[0],)))
    ns = beta.shape[0]
    th, mu, cnt, fl, cs, ct, cst, nc = _finder_out(ns, max_img, max_cand)
    lib().orc_find_images_mp(C.c_int(len(tabs)), arr, _p(Hs, C.c_int), _p(zp), C.c_double(H0),
                             C.c_double(Om), C.c_double(grid["x0"]), C.c_double(grid["y0"]),
                             C.c_double(grid["h"]), C.c_int(grid["nx"]), C.c_int(grid["ny"]), _p(beta),
                             _p(zs), C.c_int(ns), C.c_int(max_img), _p(th), _p(mu), _p(cnt, C.c_int),
                             _p(fl, C.c_int), _p(cs, C.c_int), _p(ct, C.c_int), _p(cst, C.c_int),
                             C.c_int(max_cand), C.byref(nc), C.c_int(nthreads or nthreads_default()))
    k = min(nc.value, max_cand)
    return {"theta": th, "mu": mu, "count": cnt, "flags": fl,
            "cand_src": cs[:k], "cand_tri": ct[:k], "cand_status": cst[:k], "n_cand": nc.value}


def vertex_beta(tab, grid, a):
    tab = _f64(tab)
    n = grid["nx"] * grid["ny"]
    bx, by = np.zeros(n), np.zeros(n)
    lib().orc_vertex_beta(_p(tab), C.c_int(tab.shape[0]), C.c_double(grid["x0"]), C.c_double(grid["y0"]),
                          C.c_double(grid["h"]), C.c_int(grid["nx"]), C.c_int(grid["ny"]), C.c_double(a),
                          _p(bx), _p(by))
    return bx, by


def orient(a, b, c):
    return lib().orc_orient(float(a[0]), float(a[1]), float(b[0]), float(b[1]), float(c[0]), float(c[1]))


def tri_contains(B, s):
    B = _f64(B).ravel()
    return bool(lib().orc_tri_contains(_p(B), C.c_double(s[0]), C.c_double(s[1])))


# --------------------------------------------------------------------------- singularity maps
def sing_map(tab, grid, refine=True, tol=1e-10, cap=200000, nthreads=None):
    """A3 crossings, segments, umbilics (D4) and swallowtails (A4) of a single-plane lens on
    the vertex grid x0 + (i + 1/2) h (Sec. 6)."""
    tab = _f64(tab)
    cx, ck, ce, cg, cfl = np.zeros(2 * cap), np.zeros(cap, np.int32), np.zeros(cap), np.zeros(cap), \
        np.zeros(cap, np.int32)
    sa, sb, sk = np.zeros(cap, np.int32), np.zeros(cap, np.int32), np.zeros(cap, np.int32)
    ux, ukap, ust = np.zeros(2 * cap), np.zeros(cap), np.zeros(cap, np.int32)
    wx, wk, we, wseg = np.zeros(2 * cap), np.zeros(cap, np.int32), np.zeros(cap), np.zeros(cap, np.int32)
    wst = np.zeros(cap, np.int32)
    cnt = np.zeros(6, np.int32)
    I = C.c_int
    lib().orc_sing_map(_p(tab), I(tab.shape[0]), C.c_double(grid["x0"]), C.c_double(grid["y0"]),
                       C.c_double(grid["h"]), I(grid["nx"]), I(grid["ny"]), I(1 if refine else 0), C.c_double(tol),
                       I(cap), _p(cx), _p(ck, I), _p(ce), _p(cg), _p(cfl, I), _p(sa, I), _p(sb, I), _p(sk, I),
                       _p(ux), _p(ukap), _p(ust, I), _p(wx), _p(wk, I), _p(we), _p(wseg, I), _p(wst, I), _p(cnt, I),
                       I(nthreads or nthreads_default()))
    nx_, ns, nu, nw = (min(int(c), cap) for c in cnt[:4])
    return {"cross": {"pos": cx[:2 * nx_].reshape(-1, 2), "k": ck[:nx_], "e": ce[:nx_], "g": cg[:nx_],
                      "flags": cfl[:nx_]},
            "seg": {"a": sa[:ns], "b": sb[:ns], "k": sk[:ns]},
            "umb": {"pos": ux[:2 * nu].reshape(-1, 2), "kappa": ukap[:nu], "status": ust[:nu]},
            "swt": {"pos": wx[:2 * nw].reshape(-1, 2), "k": wk[:nw], "e": we[:nw], "seg": wseg[:nw],
                    "status": wst[:nw]},
            "counts": cnt.copy()}


def find_images_ms(tab, grid, beta, a_src, max_img=16, polish=False, nthreads=None):
    """The contour-intersection finder of Sec. 2.3 (marching squares on both components of
    beta - theta + a alpha); polish: FP64 Newton from each intersection."""
    tab = _f64(tab)
    beta = _f64(beta).reshape(-1, 2)
    a_src = _f64(np.broadcast_to(a_src, (beta.shape[0],)))
    ns = beta.shape[0]
    th, mu = np.zeros((ns, max_img, 2)), np.zeros((ns, max_img))
    cnt, fl = np.zeros(ns, np.int32), np.zeros(ns, np.int32)
    lib().orc_find_images_ms(_p(tab), C.c_int(tab.shape[0]), C.c_double(grid["x0"]), C.c_double(grid["y0"]),
                             C.c_double(grid["h"]), C.c_int(grid["nx"]), C.c_int(grid["ny"]), _p(beta), _p(a_src),
                             C.c_int(ns), C.c_int(max_img), C.c_int(1 if polish else 0), _p(th), _p(mu),
                             _p(cnt, C.c_int), _p(fl, C.c_int), C.c_int(nthreads or nthreads_default()))
    return {"theta": th, "mu": mu, "count": cnt, "flags": fl}
