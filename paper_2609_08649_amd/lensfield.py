"""Thin ctypes binding of the lensfield C ABI (include/lensfield.h).

Functions named like the C entry points marshal arguments only; every step of the
hot path runs in the HIP library.  PyTorch provides device memory and streams.
The library is loaded after torch so that both use the same HIP runtime; if it
cannot be loaded the import fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import build as _build

LF_OK, LF_E_INVALID_ARG, LF_E_UNSUPPORTED, LF_E_OUT_OF_BUDGET, LF_E_DEVICE, LF_E_OVERFLOW, LF_E_NOT_READY = \
    0, -1, -2, -3, -4, -5, -6
LF_PREC_FP64, LF_PREC_MIXED = 0, 1
FLAG_SINGULAR, FLAG_GSING, FLAG_NOCONV, FLAG_REJECT, FLAG_MERGED, FLAG_OVERFLOW, FLAG_UMBILIC, FLAG_INVALID = \
    1, 2, 4, 8, 16, 32, 64, 128
FIELDS = ("x", "y", "b", "q", "pa", "s", "a")


class LfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("lensfield error %d: %s" % (status, msg))
        self.status = status


class lf_binding(C.Structure):
    _fields_ = [("kind", C.c_int32), ("index", C.c_int32), ("xform", C.c_int32), ("pad", C.c_int32),
                ("value", C.c_double)]


class lf_component(C.Structure):
    _fields_ = [("type", C.c_int32), ("pad", C.c_int32), ("f", lf_binding * 7)]


class lf_members(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad", C.c_int32), ("type", C.POINTER(C.c_int32)),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)), ("q", C.POINTER(C.c_double)),
                ("pa", C.POINTER(C.c_double)), ("lum", C.POINTER(C.c_double)), ("lam", C.c_double),
                ("bet", C.c_double), ("alp", C.c_double), ("b0", C.POINTER(C.c_double)),
                ("s0", C.POINTER(C.c_double)), ("a0", C.POINTER(C.c_double)), ("bmul", lf_binding),
                ("smul", lf_binding), ("amul", lf_binding)]


class lf_cosmo(C.Structure):
    _fields_ = [("H0", C.c_double), ("Om", C.c_double)]


class lf_grid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("h", C.c_double), ("nx", C.c_int32), ("ny", C.c_int32)]


class lf_points(C.Structure):
    _fields_ = [("grid", lf_grid), ("px", C.c_void_p), ("py", C.c_void_p), ("n", C.c_int64)]


SING_FIELDS = ("cross_pos", "cross_k", "cross_e", "cross_g", "cross_flags", "seg_a", "seg_b", "seg_k", "umb_pos",
               "umb_kappa", "umb_status", "swt_pos", "swt_k", "swt_e", "swt_seg", "swt_status", "counts")


class lf_sing_out(C.Structure):
    _fields_ = [("cap", C.c_int32)] + [(k, C.c_void_p) for k in SING_FIELDS]


MAP_FIELDS = ("alpha_x", "alpha_y", "psi11", "psi12", "psi22", "kappa", "gamma1", "gamma2", "detA", "mu",
              "beta_x", "beta_y", "psi111", "psi112", "psi122", "psi222", "e1", "e2", "f1", "f2")


class lf_maps(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in MAP_FIELDS] + [("flags", C.c_void_p)]


_lib = None
P, I32, I64, D, VP = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_void_p
PP = C.POINTER(C.c_void_p)


def lib():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        L = C.CDLL(path, mode=C.RTLD_GLOBAL)
        sig = {
            "lf_init": (I32, [PP, I32, C.c_size_t]),
            "lf_shutdown": (I32, [P]),
            "lf_last_error": (C.c_char_p, [P]),
            "lf_device_bytes": (C.c_size_t, [P]),
            "lf_cosmo_dist": (I32, [C.POINTER(lf_cosmo), D, D, C.POINTER(D)]),
            "lf_cosmo_adis": (I32, [C.POINTER(lf_cosmo), D, D, C.POINTER(D)]),
            "lf_cosmo_tdscale": (I32, [C.POINTER(lf_cosmo), D, D, C.POINTER(D)]),
            "lf_nfw_params": (I32, [C.POINTER(lf_cosmo), D, D, D, C.POINTER(D), C.POINTER(D)]),
            "lf_model_upload": (I32, [P, C.POINTER(lf_component), I32, C.POINTER(lf_members), D,
                                      C.POINTER(lf_cosmo), I32, PP]),
            "lf_model_release": (I32, [P, P]),
            "lf_model_n_halos": (I32, [P]),
            "lf_constraints_upload": (I32, [P, P, P, P, P, P, I32, P, I32, PP]),
            "lf_constraints_release": (I32, [P, P]),
            "lf_constraints_observables": (I32, [P, P, P, P, P, P, P]),
            "lf_lens_maps": (I32, [P, P, P, I32, C.POINTER(lf_points), D, I32, C.POINTER(lf_maps), P]),
            "lf_chi2_batch": (I32, [P, P, P, I32, P, I32, I32, P, P, P, P]),
            "lf_chi2_terms": (I32, [P, P, P, I32, P, I32, I32, P, P, P, P, P]),
            "lf_chi2_batch_noalloc": (I32, [P, P, P, I32, P, I32, I32, P, P, P, P]),
            "lf_chi2_images": (I32, [P, P, P, I32, P, I32, P, P, P, P, P, P]),
            "lf_find_images": (I32, [P, P, P, P, P, I32, C.POINTER(lf_grid), I32, I32, P, P, P, P, P]),
            "lf_find_images_alpha": (I32, [P, P, P, P, P, P, P, I32, C.POINTER(lf_grid), I32, I32, P, P, P, P, P]),
            "lf_find_images_ms": (I32, [P, P, P, P, P, I32, C.POINTER(lf_grid), I32, I32, I32, P, P, P, P, P]),
            "lf_multiplane_trace": (I32, [P, P, P, I32, C.POINTER(lf_cosmo), P, I32, C.POINTER(lf_points), I32,
                                          P, P, P, P]),
            "lf_aies_run": (I32, [P, P, P, I32, I32, I32, P, P, I32, P, P, D, C.c_uint64, I64, I32, P, P, P, P]),
            "lf_nelder_mead_run": (I32, [P, P, P, I32, I32, I32, P, P, P, P, I32, P, P]),
            "lf_singularity_map": (I32, [P, P, P, C.POINTER(lf_grid), I32, I32, D, C.POINTER(lf_sing_out), P]),
            "lf_find_images_mp": (I32, [P, P, P, I32, C.POINTER(lf_cosmo), P, P, I32, C.POINTER(lf_grid), I32,
                                        I32, P, P, P, P, P]),
            "lf_profile_enable": (I32, [P, I32]),
            "lf_batch_create": (I32, [P, P, I32, I32, I32, I32, PP]),
            "lf_batch_run": (I32, [P, P]),
            "lf_batch_info": (I32, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)]),
            "lf_batch_release": (I32, [P]),
            "lf_serve_start": (I32, [P, P, PP]),
            "lf_serve_submit": (I32, [P, P, C.POINTER(I64)]),
            "lf_serve_poll": (I32, [P, I64, C.POINTER(I32), C.POINTER(D)]),
            "lf_serve_wait": (I32, [P, I64, C.POINTER(I32), C.POINTER(D)]),
            "lf_serve_stats": (I32, [P, I32, C.POINTER(I64), C.POINTER(D), C.POINTER(D), C.POINTER(D)]),
            "lf_serve_stop": (I32, [P]),
            "lf_profile_read": (I32, [P, C.c_char_p, C.POINTER(D), C.POINTER(I64)]),
            "lf_profile_reset": (I32, [P]),
            "lf_profile_only": (I32, [P, C.c_char_p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols():
    """Names of the functions declared in include/lensfield.h."""
    import re
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lensfield.h")
    txt = open(hdr).read()
    decl = re.compile(r"^(?:lf_status|const char\*|size_t|int32_t|void)\s+(lf_[a-z0-9_]+)\s*\(", re.M)
    return sorted(set(decl.findall(txt)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _bind(b):
    kind, v, xf = b
    if kind == "fixed":
        return lf_binding(0, 0, int(xf), 0, float(v))
    return lf_binding(1, int(v), int(xf), 0, 0.0)


def _f64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Model:
    def __init__(self, ctx, handle, model, keep):
        self.ctx, self.handle, self.desc, self._keep = ctx, handle, model, keep
        self.n_free = int(model.get("n_free", 0))

    @property
    def n_halos(self):
        return lib().lf_model_n_halos(self.handle)

    def release(self):
        if self.handle:
            lib().lf_model_release(self.ctx.handle, self.handle)
            self.handle = None


class Constraints:
    def __init__(self, ctx, handle, n_img, n_fam):
        self.ctx, self.handle, self.n_img, self.n_fam = ctx, handle, n_img, n_fam

    def release(self):
        if self.handle:
            lib().lf_constraints_release(self.ctx.handle, self.handle)
            self.handle = None


class Context:
    """An lf_ctx on one HIP device."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        L = lib()
        h = C.c_void_p()
        st = L.lf_init(C.byref(h), int(device), C.c_size_t(hbm_budget))
        if st != LF_OK:
            raise LfError(st, "lf_init failed")
        self.handle = h
        self.device = torch.device("cuda", device)

    def close(self):
        if self.handle:
            lib().lf_shutdown(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, st):
        if st != LF_OK:
            raise LfError(st, lib().lf_last_error(self.handle).decode())

    @property
    def device_bytes(self):
        return lib().lf_device_bytes(self.handle)

    # ---------------------------------------------------------------- helpers
    @staticmethod
    def cosmo(H0=70.0, Om=0.3):
        return lf_cosmo(H0, Om)

    def dist(self, z1, z2, H0=70.0, Om=0.3):
        out = C.c_double()
        c = lf_cosmo(H0, Om)
        self.check(lib().lf_cosmo_dist(C.byref(c), z1, z2, C.byref(out)))
        return out.value

    def adis(self, zd, zs, H0=70.0, Om=0.3):
        out = C.c_double()
        c = lf_cosmo(H0, Om)
        self.check(lib().lf_cosmo_adis(C.byref(c), zd, zs, C.byref(out)))
        return out.value

    def tdscale(self, zd, zs, H0=70.0, Om=0.3):
        """(1+z_d)/c D_d D_s/D_ds theta_0^2 in days per arcsec^2."""
        out = C.c_double()
        c = lf_cosmo(H0, Om)
        self.check(lib().lf_cosmo_tdscale(C.byref(c), zd, zs, C.byref(out)))
        return out.value

    def nfw_params(self, zd, m200, c200, H0=70.0, Om=0.3):
        ks, rs = C.c_double(), C.c_double()
        c = lf_cosmo(H0, Om)
        self.check(lib().lf_nfw_params(C.byref(c), zd, m200, c200, C.byref(ks), C.byref(rs)))
        return ks.value, rs.value

    # ---------------------------------------------------------------- models
    def upload_model(self, model) -> Model:
        main = model["main"]
        comps = (lf_component * max(1, len(main)))()
        for i, c in enumerate(main):
            comps[i].type = int(c["type"])
            for k, f in enumerate(FIELDS):
                comps[i].f[k] = _bind(c[f])
        mem = model["members"]
        n = len(mem["x"])
        keep = []

        def arr(a, dt=np.float64):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=dt)
            keep.append(a)
            return a

        ms = lf_members()
        ms.n = n
        t = arr(mem["type"], np.int32)
        ms.type = t.ctypes.data_as(C.POINTER(C.c_int32))
        for k in ("x", "y", "q", "pa", "lum", "b0", "s0", "a0"):
            a = arr(mem.get(k))
            setattr(ms, k, _f64p(a) if a is not None else None)
        ex = mem.get("exps", (0.0, 0.0, 0.0))
        ms.lam, ms.bet, ms.alp = float(ex[0]), float(ex[1]), float(ex[2])
        ms.bmul, ms.smul, ms.amul = _bind(mem["bmul"]), _bind(mem["smul"]), _bind(mem["amul"])
        cos = lf_cosmo(model["H0"], model["Om"])
        h = C.c_void_p()
        self.check(lib().lf_model_upload(self.handle, comps, len(main), C.byref(ms), float(model["z_d"]),
                                         C.byref(cos), int(model.get("n_free", 0)), C.byref(h)))
        return Model(self, h, model, keep)

    def upload_constraints(self, cons) -> Constraints:
        th = np.ascontiguousarray(cons["theta"], np.float64).reshape(-1, 2)
        fam = np.ascontiguousarray(cons["family"], np.int32)
        s1 = np.ascontiguousarray(cons["sig1"], np.float64)
        s2 = np.ascontiguousarray(cons["sig2"], np.float64)
        ph = np.ascontiguousarray(cons["phi"], np.float64)
        af = np.ascontiguousarray(cons["a_fam"], np.float64)
        h = C.c_void_p()
        self.check(lib().lf_constraints_upload(self.handle, th.ctypes.data, fam.ctypes.data, s1.ctypes.data,
                                               s2.ctypes.data, ph.ctypes.data, fam.size, af.ctypes.data, af.size,
                                               C.byref(h)))
        c = Constraints(self, h, fam.size, af.size)
        has_mag, has_dt = cons.get("mag") is not None, cons.get("dt") is not None
        if has_mag or has_dt:
            def f64(k):
                return np.ascontiguousarray(cons[k], np.float64) if cons.get(k) is not None else None
            arrs = [f64("mag") if has_mag else None, f64("sig_mag") if has_mag else None,
                    f64("dt") if has_dt else None, f64("sig_dt") if has_dt else None,
                    f64("tscale") if has_dt else None]
            ptrs = [None if a is None else a.ctypes.data for a in arrs]
            try:
                self.check(lib().lf_constraints_observables(self.handle, h, *ptrs))
            except Exception:
                c.release()
                raise
        return c

    # ---------------------------------------------------------------- hot path
    def lens_maps(self, model: Model, params, S, points, a_dis, prec=LF_PREC_FP64,
                  outputs=("alpha_x", "alpha_y", "psi11", "psi12", "psi22", "kappa", "gamma1", "gamma2",
                           "detA", "mu", "beta_x", "beta_y"), flags=True, stream=None, out=None):
        """points: grid dict (x0, y0, h, nx, ny) or (px, py) device tensors."""
        pts = lf_points()
        keep = []
        if isinstance(points, dict):
            pts.grid = lf_grid(points["x0"], points["y0"], points["h"], points["nx"], points["ny"])
            pts.px = pts.py = None
            P = points["nx"] * points["ny"]
        else:
            px, py = points
            keep += [px, py]
            pts.px, pts.py, pts.n = px.data_ptr(), py.data_ptr(), px.numel()
            P = px.numel()
        res = {} if out is None else dict(out)
        m = lf_maps()
        for k in outputs:
            if k not in res:
                res[k] = torch.empty((S, P), dtype=torch.float64, device=self.device)
            setattr(m, k, res[k].data_ptr())
        if flags:
            if "flags" not in res:
                res["flags"] = torch.empty((S, P), dtype=torch.int32, device=self.device)
            m.flags = res["flags"].data_ptr()
        pp = None
        if params is not None:
            pp = C.c_void_p(params.data_ptr())
        self.check(lib().lf_lens_maps(self.handle, model.handle, pp, int(S), C.byref(pts), float(a_dis), int(prec),
                                      C.byref(m), _stream(stream)))
        return res


def _chi2(self, model: Model, params, S, cons: Constraints, mode=0, prec=LF_PREC_FP64, want_beta=False,
          stream=None, out=None):
    """chi^2 per sample (device tensors): returns (chi2 [S] f64, flags [S] i32, beta_model or None)."""
    dev = self.device
    chi2 = out["chi2"] if out else torch.empty(S, dtype=torch.float64, device=dev)
    flags = out["flags"] if out else torch.empty(S, dtype=torch.int32, device=dev)
    bm = torch.empty((S, cons.n_fam, 2), dtype=torch.float64, device=dev) if want_beta else None
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_chi2_batch(self.handle, model.handle, pp, int(S), cons.handle, int(mode), int(prec),
                                   C.c_void_p(chi2.data_ptr()), C.c_void_p(flags.data_ptr()),
                                   C.c_void_p(bm.data_ptr()) if bm is not None else None, _stream(stream)))
    return chi2, flags, bm


Context.chi2_batch = _chi2


def _chi2_noalloc(self, model: Model, params, S, cons: Constraints, mode=0, prec=LF_PREC_FP64, want_beta=False,
                  stream=None, out=None):
    """chi^2 per sample through the allocation-free entry point (workspace in the library's static
    device scratch); same outputs as chi2_batch."""
    dev = self.device
    chi2 = out["chi2"] if out else torch.empty(S, dtype=torch.float64, device=dev)
    flags = out["flags"] if out else torch.empty(S, dtype=torch.int32, device=dev)
    bm = torch.empty((S, cons.n_fam, 2), dtype=torch.float64, device=dev) if want_beta else None
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_chi2_batch_noalloc(self.handle, model.handle, pp, int(S), cons.handle, int(mode),
                                           int(prec), C.c_void_p(chi2.data_ptr()), C.c_void_p(flags.data_ptr()),
                                           C.c_void_p(bm.data_ptr()) if bm is not None else None,
                                           _stream(stream)))
    return chi2, flags, bm


Context.chi2_batch_noalloc = _chi2_noalloc


def _chi2_terms(self, model: Model, params, S, cons: Constraints, mode=0, prec=LF_PREC_FP64, want_beta=False,
                stream=None, out=None):
    """Total chi^2 with the flux and delay terms: (chi2 [S], flags [S], terms [S,3], beta_model or None)."""
    dev = self.device
    chi2 = out["chi2"] if out else torch.empty(S, dtype=torch.float64, device=dev)
    flags = out["flags"] if out else torch.empty(S, dtype=torch.int32, device=dev)
    terms = out["terms"] if out else torch.empty((S, 3), dtype=torch.float64, device=dev)
    bm = torch.empty((S, cons.n_fam, 2), dtype=torch.float64, device=dev) if want_beta else None
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_chi2_terms(self.handle, model.handle, pp, int(S), cons.handle, int(mode), int(prec),
                                   C.c_void_p(chi2.data_ptr()), C.c_void_p(flags.data_ptr()),
                                   C.c_void_p(bm.data_ptr()) if bm is not None else None,
                                   C.c_void_p(terms.data_ptr()), _stream(stream)))
    return chi2, flags, terms, bm


Context.chi2_terms = _chi2_terms


def _chi2_images(self, model: Model, params, S, cons: Constraints, prec=LF_PREC_FP64, stream=None):
    """Image-plane chi^2 with per-image results (device tensors): chi2 [S], flags [S],
    beta_model [S, n_fam, 2], theta_model [S, n_img, 2] and img_flags [S, n_img] in the constraint
    order."""
    dev = self.device
    n = cons.n_img
    r = {"chi2": torch.empty(S, dtype=torch.float64, device=dev),
         "flags": torch.empty(S, dtype=torch.int32, device=dev),
         "beta_model": torch.empty((S, cons.n_fam, 2), dtype=torch.float64, device=dev),
         "theta_model": torch.empty((S, n, 2), dtype=torch.float64, device=dev),
         "img_flags": torch.empty((S, n), dtype=torch.int32, device=dev)}
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_chi2_images(self.handle, model.handle, pp, int(S), cons.handle, int(prec),
                                    *[C.c_void_p(r[k].data_ptr()) for k in
                                      ("chi2", "flags", "beta_model", "theta_model", "img_flags")],
                                    _stream(stream)))
    return r


Context.chi2_images = _chi2_images


def _find(self, model: Model, params, beta, a_src, grid, max_img=16, prec=LF_PREC_FP64, stream=None, out=None):
    """Images of n_src sources (beta [n,2], a_src [n] device f64 tensors) on a grid."""
    n = beta.shape[0]
    dev = self.device
    if out is None:
        out = {"theta": torch.zeros((n, max_img, 2), dtype=torch.float64, device=dev),
               "mu": torch.zeros((n, max_img), dtype=torch.float64, device=dev),
               "count": torch.zeros(n, dtype=torch.int32, device=dev),
               "flags": torch.zeros(n, dtype=torch.int32, device=dev)}
    th, mu, cnt, fl = out["theta"], out["mu"], out["count"], out["flags"]
    g = lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"])
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_find_images(self.handle, model.handle, pp, C.c_void_p(beta.data_ptr()),
                                    C.c_void_p(a_src.data_ptr()), int(n), C.byref(g), int(max_img), int(prec),
                                    C.c_void_p(th.data_ptr()), C.c_void_p(mu.data_ptr()),
                                    C.c_void_p(cnt.data_ptr()), C.c_void_p(fl.data_ptr()), _stream(stream)))
    return {"theta": th, "mu": mu, "count": cnt, "flags": fl}


def _find_alpha(self, model: Model, params, alpha_x, alpha_y, beta, a_src, grid, max_img=16, prec=LF_PREC_FP64,
                stream=None, out=None):
    """Images of n_src sources on a grid whose vertex deflections alpha_x, alpha_y (device f64,
    nx * ny each, e.g. lens_maps outputs on that grid) are already computed."""
    n = beta.shape[0]
    dev = self.device
    if out is None:
        out = {"theta": torch.zeros((n, max_img, 2), dtype=torch.float64, device=dev),
               "mu": torch.zeros((n, max_img), dtype=torch.float64, device=dev),
               "count": torch.zeros(n, dtype=torch.int32, device=dev),
               "flags": torch.zeros(n, dtype=torch.int32, device=dev)}
    th, mu, cnt, fl = out["theta"], out["mu"], out["count"], out["flags"]
    assert alpha_x.numel() == grid["nx"] * grid["ny"] and alpha_y.numel() == alpha_x.numel()
    g = lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"])
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_find_images_alpha(self.handle, model.handle, pp, C.c_void_p(alpha_x.data_ptr()),
                                          C.c_void_p(alpha_y.data_ptr()), C.c_void_p(beta.data_ptr()),
                                          C.c_void_p(a_src.data_ptr()), int(n), C.byref(g), int(max_img), int(prec),
                                          C.c_void_p(th.data_ptr()), C.c_void_p(mu.data_ptr()),
                                          C.c_void_p(cnt.data_ptr()), C.c_void_p(fl.data_ptr()), _stream(stream)))
    return {"theta": th, "mu": mu, "count": cnt, "flags": fl}


def _planes_arg(planes, z_planes, H0, Om):
    arr = (C.c_void_p * len(planes))(*[p.handle.value for p in planes])
    zp = np.ascontiguousarray(z_planes, np.float64)
    return arr, zp, lf_cosmo(H0, Om)


def _mp_trace(self, planes, z_planes, z_src, points, prec=LF_PREC_FP64, H0=70.0, Om=0.3, stream=None,
              outputs=("beta", "A", "mu")):
    arr, zp, cos = _planes_arg(planes, z_planes, H0, Om)
    zs = np.ascontiguousarray(np.atleast_1d(z_src), np.float64)
    pts = lf_points()
    keep = []
    if isinstance(points, dict):
        pts.grid = lf_grid(points["x0"], points["y0"], points["h"], points["nx"], points["ny"])
        P = points["nx"] * points["ny"]
    else:
        px, py = points
        keep += [px, py]
        pts.px, pts.py, pts.n = px.data_ptr(), py.data_ptr(), px.numel()
        P = px.numel()
    dev = self.device
    res = {}
    if "beta" in outputs:
        res["beta"] = torch.empty((zs.size, P, 2), dtype=torch.float64, device=dev)
    if "A" in outputs:
        res["A"] = torch.empty((zs.size, P, 4), dtype=torch.float64, device=dev)
    if "mu" in outputs:
        res["mu"] = torch.empty((zs.size, P), dtype=torch.float64, device=dev)
    ptr = lambda k: C.c_void_p(res[k].data_ptr()) if k in res else None
    self.check(lib().lf_multiplane_trace(self.handle, arr, zp.ctypes.data, len(planes), C.byref(cos),
                                         zs.ctypes.data, zs.size, C.byref(pts), int(prec), ptr("beta"), ptr("A"),
                                         ptr("mu"), _stream(stream)))
    return res


def _find_mp(self, planes, z_planes, beta, z_src, grid, max_img=16, prec=LF_PREC_FP64, H0=70.0, Om=0.3,
             stream=None):
    arr, zp, cos = _planes_arg(planes, z_planes, H0, Om)
    zs = np.ascontiguousarray(z_src, np.float64)
    n = beta.shape[0]
    dev = self.device
    th = torch.zeros((n, max_img, 2), dtype=torch.float64, device=dev)
    mu = torch.zeros((n, max_img), dtype=torch.float64, device=dev)
    cnt = torch.zeros(n, dtype=torch.int32, device=dev)
    fl = torch.zeros(n, dtype=torch.int32, device=dev)
    g = lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"])
    self.check(lib().lf_find_images_mp(self.handle, arr, zp.ctypes.data, len(planes), C.byref(cos),
                                       C.c_void_p(beta.data_ptr()), zs.ctypes.data, int(n), C.byref(g),
                                       int(max_img), int(prec), C.c_void_p(th.data_ptr()),
                                       C.c_void_p(mu.data_ptr()), C.c_void_p(cnt.data_ptr()),
                                       C.c_void_p(fl.data_ptr()), _stream(stream)))
    return {"theta": th, "mu": mu, "count": cnt, "flags": fl}


Context.find_images = _find
Context.find_images_alpha = _find_alpha


def _find_ms(self, model: Model, params, beta, a_src, grid, max_img=16, prec=LF_PREC_FP64, polish=True,
             stream=None):
    """Contour-intersection finder (Sec. 2.3) for n_src sources (device tensors beta [n,2], a_src [n])."""
    n = beta.shape[0]
    dev = self.device
    out = {"theta": torch.zeros((n, max_img, 2), dtype=torch.float64, device=dev),
           "mu": torch.zeros((n, max_img), dtype=torch.float64, device=dev),
           "count": torch.zeros(n, dtype=torch.int32, device=dev),
           "flags": torch.zeros(n, dtype=torch.int32, device=dev)}
    g = lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"])
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_find_images_ms(self.handle, model.handle, pp, _ptr(beta), _ptr(a_src), int(n), C.byref(g),
                                       int(max_img), int(prec), 1 if polish else 0, _ptr(out["theta"]),
                                       _ptr(out["mu"]), _ptr(out["count"]), _ptr(out["flags"]), _stream(stream)))
    return out


Context.find_images_ms = _find_ms


def sing_buffers(device, cap):
    """Device output lists for lf_singularity_map (reusable across calls)."""
    f64 = lambda *sh: torch.zeros(sh, dtype=torch.float64, device=device)
    i32 = lambda *sh: torch.zeros(sh, dtype=torch.int32, device=device)
    return {"cross_pos": f64(cap, 2), "cross_k": i32(cap), "cross_e": f64(cap), "cross_g": f64(cap),
            "cross_flags": i32(cap), "seg_a": i32(cap), "seg_b": i32(cap), "seg_k": i32(cap), "umb_pos": f64(cap, 2),
            "umb_kappa": f64(cap), "umb_status": i32(cap), "swt_pos": f64(cap, 2), "swt_k": i32(cap),
            "swt_e": f64(cap), "swt_seg": i32(cap), "swt_status": i32(cap), "counts": i32(6)}


def _sing_map(self, model: Model, params, grid, prec=LF_PREC_FP64, refine=True, tol=1e-10, cap=1 << 18,
              stream=None, out=None, finish=True):
    """Singularity map of a single-plane lens (A3 crossings and segments, umbilics, swallowtails);
    device tensors cut to the true counts (or to cap).  out: buffers from sing_buffers (their
    capacity is used); finish=False returns the raw buffers without synchronising."""
    t = out if out is not None else sing_buffers(self.device, cap)
    cap = t["cross_k"].numel()
    o = lf_sing_out()
    o.cap = int(cap)
    for k in SING_FIELDS:
        setattr(o, k, t[k].data_ptr())
    g = lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"])
    pp = C.c_void_p(params.data_ptr()) if params is not None else None
    self.check(lib().lf_singularity_map(self.handle, model.handle, pp, C.byref(g), int(prec), 1 if refine else 0,
                                        float(tol), C.byref(o), _stream(stream)))
    if not finish:
        return t
    (stream or torch.cuda.current_stream()).synchronize()
    cnt = t["counts"].cpu()
    n = [min(int(c), cap) for c in cnt[:4]]
    return {"cross": {"pos": t["cross_pos"][:n[0]], "k": t["cross_k"][:n[0]], "e": t["cross_e"][:n[0]],
                      "g": t["cross_g"][:n[0]], "flags": t["cross_flags"][:n[0]]},
            "seg": {"a": t["seg_a"][:n[1]], "b": t["seg_b"][:n[1]], "k": t["seg_k"][:n[1]]},
            "umb": {"pos": t["umb_pos"][:n[2]], "kappa": t["umb_kappa"][:n[2]], "status": t["umb_status"][:n[2]]},
            "swt": {"pos": t["swt_pos"][:n[3]], "k": t["swt_k"][:n[3]], "e": t["swt_e"][:n[3]],
                    "seg": t["swt_seg"][:n[3]], "status": t["swt_status"][:n[3]]},
            "counts": cnt.numpy()}


Context.singularity_map = _sing_map


def _aies(self, model: Model, cons: Constraints, X, lp, lo, hi, n_steps, seed, step0=0, a=2.0, mode=0,
          prec=LF_PREC_MIXED, init_lp=False, chain=None, lp_chain=None, n_accept=None, stream=None):
    """AIES steps on device tensors X [K, D] and lp [K] (updated in place)."""
    K = X.shape[0]
    self.check(lib().lf_aies_run(self.handle, model.handle, cons.handle, int(mode), int(prec), int(K),
                                 _ptr(X), _ptr(lp), 1 if init_lp else 0, _ptr(lo), _ptr(hi), float(a),
                                 C.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(step0), int(n_steps), _ptr(chain),
                                 _ptr(lp_chain), _ptr(n_accept), _stream(stream)))


def _nelder_mead(self, model: Model, cons: Constraints, simplex, lo, hi, n_rounds, mode=0, prec=LF_PREC_MIXED,
                 fvals=None, n_evals=None, stream=None):
    """Nelder-Mead rounds on device simplices [R, D+1, D] (updated in place, sorted); returns f."""
    R, V, D = simplex.shape
    f = fvals if fvals is not None else torch.empty((R, V), dtype=torch.float64, device=simplex.device)
    self.check(lib().lf_nelder_mead_run(self.handle, model.handle, cons.handle, int(mode), int(prec), int(R),
                                        _ptr(simplex), _ptr(f), _ptr(lo), _ptr(hi), int(n_rounds), _ptr(n_evals),
                                        _stream(stream)))
    return f


Context.aies = _aies
Context.nelder_mead = _nelder_mead
Context.multiplane_trace = _mp_trace
Context.find_images_mp = _find_mp


class lf_batch_item(C.Structure):
    _fields_ = [("model", C.c_void_p), ("cons", C.c_void_p), ("params", C.c_void_p), ("S", C.c_int32),
                ("pad", C.c_int32), ("chi2", C.c_void_p), ("flags", C.c_void_p)]


class Batch:
    """A planned uneven chi^2 batch (persistent launch captured in a hipGraph)."""

    def __init__(self, ctx, items, mode=0, prec=LF_PREC_MIXED, autotune=True):
        """items: list of (Model, Constraints, params tensor [S, n_free] or None, S)."""
        self.ctx = ctx
        dev = ctx.device
        self.outputs = []
        arr = (lf_batch_item * len(items))()
        self._keep = []
        for k, (m, c, p, S) in enumerate(items):
            chi = torch.empty(S, dtype=torch.float64, device=dev)
            fl = torch.empty(S, dtype=torch.int32, device=dev)
            self.outputs.append((chi, fl))
            self._keep.append(p)
            arr[k] = lf_batch_item(m.handle.value, c.handle.value, p.data_ptr() if p is not None else None,
                                   int(S), 0, chi.data_ptr(), fl.data_ptr())
        h = C.c_void_p()
        ctx.check(lib().lf_batch_create(ctx.handle, C.cast(arr, C.c_void_p), len(items), int(mode), int(prec),
                                        1 if autotune else 0, C.byref(h)))
        self.handle = h

    def run(self, stream=None):
        self.ctx.check(lib().lf_batch_run(self.handle, _stream(stream)))
        return self.outputs

    def info(self):
        v = [C.c_int32() for _ in range(4)]
        self.ctx.check(lib().lf_batch_info(self.handle, *[C.byref(x) for x in v]))
        return {"block": v[0].value, "grid": v[1].value, "tile_lanes": v[2].value, "n_tiles": v[3].value}

    def release(self):
        if self.handle:
            lib().lf_batch_release(self.handle)
            self.handle = None


LF_REQ_CHI2, LF_REQ_MU_MAP, LF_REQ_SING_MAP = 0, 1, 2
SING_PLANES = ("kappa", "detA", "e1", "e2", "f1", "f2")


class lf_serve_config(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("n_streams", C.c_int32), ("max_batch_samples", C.c_int32),
                ("map_chunk_rows", C.c_int32)]


class lf_request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("S", C.c_int32), ("model", C.c_void_p), ("cons", C.c_void_p),
                ("params", C.c_void_p), ("mode", C.c_int32), ("prec", C.c_int32), ("grid", lf_grid),
                ("a_dis", C.c_double), ("out_host", C.c_void_p), ("flags_host", C.c_void_p),
                ("out_device", C.c_void_p), ("flags_device", C.c_void_p)]


class Server:
    """Continuous-batching server (C++ scheduler thread) on a context."""

    def __init__(self, ctx, hbm_budget, n_streams=3, max_batch_samples=0, map_chunk_rows=0):
        self.ctx = ctx
        cfg = lf_serve_config(int(hbm_budget), int(n_streams), int(max_batch_samples), int(map_chunk_rows))
        h = C.c_void_p()
        ctx.check(lib().lf_serve_start(ctx.handle, C.byref(cfg), C.byref(h)))
        self.handle = h
        self._keep = {}

    def _submit(self, req, keep):
        t = C.c_int64()
        st = lib().lf_serve_submit(self.handle, C.byref(req), C.byref(t))
        if st != LF_OK:
            raise LfError(st, "submit rejected")
        self._keep[t.value] = keep
        return t.value

    def submit_chi2(self, model, cons, params, mode=0, prec=LF_PREC_MIXED, out=None, flags=None):
        """params: host float64 [S, n_free] (copied at submit).  Returns (ticket, chi2, flags) with
        pinned host outputs that are valid once the ticket is done."""
        p = np.ascontiguousarray(params, np.float64)
        S = p.shape[0]
        out = out if out is not None else torch.empty(S, dtype=torch.float64, pin_memory=True)
        flags = flags if flags is not None else torch.empty(S, dtype=torch.int32, pin_memory=True)
        req = lf_request(LF_REQ_CHI2, S, model.handle.value, cons.handle.value, p.ctypes.data if p.size else None,
                         int(mode), int(prec), lf_grid(0, 0, 1, 1, 1), 1.0, out.data_ptr(), flags.data_ptr(), None,
                         None)
        return self._submit(req, (p, out, flags)), out, flags

    def submit_map(self, model, params, grid, a_dis, kind=LF_REQ_MU_MAP, prec=LF_PREC_MIXED, out=None):
        """out: pinned host [planes, P] (allocated when None), or a device tensor of that shape to
        keep the result on the device (no copy to the host)."""
        planes = 6 if kind == LF_REQ_SING_MAP else 1
        P = grid["nx"] * grid["ny"]
        out = out if out is not None else torch.empty((planes, P), dtype=torch.float64, pin_memory=True)
        on_dev = out.is_cuda
        p = np.ascontiguousarray(params, np.float64) if params is not None else None
        req = lf_request(int(kind), 1, model.handle.value, None, p.ctypes.data if p is not None else None, 0, int(prec),
                         lf_grid(grid["x0"], grid["y0"], grid["h"], grid["nx"], grid["ny"]), float(a_dis),
                         None if on_dev else out.data_ptr(), None, out.data_ptr() if on_dev else None, None)
        return self._submit(req, (p, out)), out

    def poll(self, ticket):
        st, lat = C.c_int32(), C.c_double()
        self.ctx.check(lib().lf_serve_poll(self.handle, int(ticket), C.byref(st), C.byref(lat)))
        return st.value, lat.value

    def wait(self, ticket):
        st, lat = C.c_int32(), C.c_double()
        self.ctx.check(lib().lf_serve_wait(self.handle, int(ticket), C.byref(st), C.byref(lat)))
        self._keep.pop(ticket, None)
        return st.value, lat.value

    def stats(self, kind=-1):
        n, p50, p99, mean = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        self.ctx.check(lib().lf_serve_stats(self.handle, int(kind), C.byref(n), C.byref(p50), C.byref(p99),
                                            C.byref(mean)))
        return {"count": n.value, "p50_ms": p50.value, "p99_ms": p99.value, "mean_ms": mean.value}

    def stop(self):
        if self.handle:
            lib().lf_serve_stop(self.handle)
            self.handle = None
