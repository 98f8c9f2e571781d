"""Inference layer of Sec. 3.5 in plain numpy: the affine-invariant ensemble sampler (AIES,
Goodman & Weare 2010) and the Nelder-Mead downhill simplex, driven by the oracle's chi^2.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU-baseline leg; the
product library never imports it.  Plain and slow on purpose: one step at a time, in the
order the algorithms are stated.

Readings (the paper names the methods and the workflow -- many Nelder-Mead runs started within
the priors, then AIES walkers jittered around the best fit -- but no parameters):
  * AIES: the stretch move with scale a (g(z) ~ 1/sqrt(z) on [1/a, a]); walkers update in two
    halves, each half using the other as its complementary ensemble, so a half can move in
    parallel (the paper runs walkers on parallel threads).  Acceptance with probability
    min(1, z^(D-1) p(Y) / p(X)).  log p = -chi^2 / 2 inside the uniform prior box, -inf
    outside it or where chi^2 is undefined.
  * Random numbers: uniform u(seed, n) = (SplitMix64 output n of the stream seeded with seed)
    / 2^64 truncated to 53 bits; draw n = ((t * 2 + half) * K + k) * 3 + d for step t, walker k
    and draw d (0: complementary walker, 1: stretch factor, 2: acceptance).
  * Nelder-Mead: the standard coefficients (reflection 1, expansion 2, contraction 1/2,
    shrink 1/2) and the rules of Lagarias, Reeds, Wright & Wright (1998), with vertices kept
    sorted by f (a new vertex goes after those with equal f; after a shrink all are re-sorted
    stably).  f = chi^2, +inf outside the prior box or where chi^2 is undefined.  One function
    evaluation per run and round (a shrink takes D rounds)."""
from __future__ import annotations

import numpy as np

from . import oracle as orc

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    """Output n (0-based) of the SplitMix64 generator seeded with seed (Steele, Lea & Flood
    2014): state seed + (n + 1) gamma, then the mixing function."""
    with np.errstate(over="ignore"):
        z = np.uint64(np.uint64(seed) & np.uint64(0xFFFFFFFFFFFFFFFF)) + \
            (np.asarray(n, dtype=np.uint64) + np.uint64(1)) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, n):
    """u in [0, 1): the top 53 bits of output n."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ------------------------------------------------------------------------------------- AIES
def aies(logp, X, lp, a, seed, step0, n_steps):
    """n_steps stretch-move steps of K walkers X [K, D] with log-probabilities lp [K].
    Returns (X, lp, accepted [K], chain [n_steps, K, D], lp_chain [n_steps, K])."""
    X = np.array(X, dtype=np.float64)
    lp = np.array(lp, dtype=np.float64)
    K, D = X.shape
    H = K // 2
    acc = np.zeros(K, np.int64)
    chain, lpc = [], []
    for t in range(step0, step0 + n_steps):
        for h in (0, 1):
            S = np.arange(h * H, (h + 1) * H)
            comp = np.arange((1 - h) * H, (2 - h) * H)
            base = ((np.uint64(t) * np.uint64(2) + np.uint64(h)) * np.uint64(K) + S.astype(np.uint64)) * np.uint64(3)
            u0, u1, u2 = uniform(seed, base), uniform(seed, base + np.uint64(1)), uniform(seed, base + np.uint64(2))
            j = comp[np.minimum((u0 * H).astype(np.int64), H - 1)]
            z = ((a - 1.0) * u1 + 1.0) ** 2 / a
            Y = X[j] + z[:, None] * (X[S] - X[j])
            lpY = logp(Y)
            with np.errstate(divide="ignore", invalid="ignore"):
                take = np.log(u2) < (D - 1) * np.log(z) + lpY - lp[S]
            X[S[take]] = Y[take]
            lp[S[take]] = lpY[take]
            acc[S[take]] += 1
        chain.append(X.copy())
        lpc.append(lp.copy())
    return X, lp, acc, np.array(chain), np.array(lpc)


# ------------------------------------------------------------------------------ Nelder-Mead
class _Run:
    def __init__(self, simplex, f):
        order = np.argsort(f, kind="stable")
        self.x = np.array(simplex, dtype=np.float64)[order]
        self.f = np.array(f, dtype=np.float64)[order]
        self.state, self.i = 0, 0
        self.xr, self.fr = None, None
        self.pending = self._reflection()

    def _centroid(self):
        D = self.x.shape[1]
        return np.sum(self.x[:D], axis=0) / D

    def _reflection(self):
        c = self._centroid()
        return c + (c - self.x[-1])

    def _insert(self, x, f):
        """Replace the worst vertex by (x, f), placed after the vertices with f <= its f."""
        xs, fs = self.x[:-1], self.f[:-1]
        k = int(np.searchsorted(fs, f, side="right"))
        self.x = np.concatenate([xs[:k], x[None], xs[k:]])
        self.f = np.concatenate([fs[:k], [f], fs[k:]])

    def step(self, fp):
        """Consume f at the pending point and set the next pending point."""
        D = self.x.shape[1]
        c = self._centroid()
        p = self.pending
        if self.state == 0:                        # reflection evaluated
            if self.f[0] <= fp < self.f[D - 1]:
                self._insert(p, fp)
            elif fp < self.f[0]:
                self.xr, self.fr = p, fp
                self.state, self.pending = 1, c + 2.0 * (p - c)
                return
            elif fp < self.f[D]:
                self.xr, self.fr = p, fp
                self.state, self.pending = 2, c + 0.5 * (p - c)
                return
            else:
                self.state, self.pending = 3, c + 0.5 * (self.x[D] - c)
                return
        elif self.state == 1:                      # expansion
            if fp < self.fr:
                self._insert(p, fp)
            else:
                self._insert(self.xr, self.fr)
        elif self.state == 2:                      # outside contraction
            if fp <= self.fr:
                self._insert(p, fp)
            else:
                self.state, self.i = 4, 1
                self.pending = self.x[0] + 0.5 * (self.x[1] - self.x[0])
                return
        elif self.state == 3:                      # inside contraction
            if fp < self.f[D]:
                self._insert(p, fp)
            else:
                self.state, self.i = 4, 1
                self.pending = self.x[0] + 0.5 * (self.x[1] - self.x[0])
                return
        else:                                      # shrink: vertex i evaluated
            self.x[self.i] = p
            self.f[self.i] = fp
            if self.i < D:
                self.i += 1
                self.pending = self.x[0] + 0.5 * (self.x[self.i] - self.x[0])
                return
            order = np.argsort(self.f, kind="stable")
            self.x, self.f = self.x[order], self.f[order]
        self.state = 0
        self.pending = self._reflection()


def nelder_mead(fun, simplices, n_rounds):
    """R runs from initial simplices [R, D+1, D]: the vertices are evaluated together, then
    n_rounds rounds of one evaluation per run.  fun maps points [n, D] to f [n].  Returns the
    sorted simplices [R, D+1, D] and f [R, D+1]."""
    S = np.asarray(simplices, dtype=np.float64)
    R, V, D = S.shape
    f0 = fun(S.reshape(R * V, D)).reshape(R, V)
    runs = [_Run(S[r], f0[r]) for r in range(R)]
    for _ in range(n_rounds):
        P = np.stack([r.pending for r in runs])
        fp = fun(P)
        for r, v in zip(runs, fp):
            r.step(v)
    return np.stack([r.x for r in runs]), np.stack([r.f for r in runs])


# --------------------------------------------------------------------------- lens likelihood
def lens_chi2(model, cons, lo, hi, img_mode=False):
    """f(P [n, D]) = chi^2 of each parameter row; +inf outside [lo, hi] or where the model is
    invalid or chi^2 undefined."""
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)

    def f(P):
        P = np.atleast_2d(P)
        out = np.full(P.shape[0], np.inf)
        inside = np.all((P >= lo) & (P <= hi), axis=1)
        idx = np.nonzero(inside)[0]
        tabs, keep = [], []
        for s in idx:
            try:
                tabs.append(orc.expand(model, P[s]))
                keep.append(s)
            except ValueError:
                pass
        if keep:
            r = orc.chi2_batch(np.stack(tabs), cons, img_mode=img_mode)
            c = r["chi2_img"] if img_mode else r["chi2_src"]
            c = np.where(np.isfinite(c), c, np.inf)
            out[np.array(keep)] = c
        return out
    return f


def lens_logp(model, cons, lo, hi, img_mode=False):
    f = lens_chi2(model, cons, lo, hi, img_mode)
    return lambda P: -0.5 * f(P)
