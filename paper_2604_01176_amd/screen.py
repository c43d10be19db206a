"""Learned gradient screen around the native ADAPT driver.

Per screened ADAPT iteration (every call below is one C-ABI entry point;
the arithmetic runs in the library's kernels):
  state psi -> <n_q> occupations -> feature rows -> MLP scores -> descending
  order -> candidates = the top K_t, the band of the next audit/2 ranks, and
  audit/2 positions drawn uniformly from the ranks below the band (a generator
  seeded by (seed, iteration), on the host) -> exact gradients of the
  candidates -> fallback to the full sweep when the largest |g| outside the
  top K_t reaches RHO of the largest inside it (the ranking does not separate
  the leaders from the rest at this state) -> selection + BFGS -> g_prev /
  age update -> one online Adam step on the freshly computed (feature,
  target) rows.
Every judge_every-th iteration (iteration 0 included) runs the full sweep.
After every full sweep the rank that the network gave the true argmax is
recorded and K_t widens to keep GROW times that rank inside the top (at most
half the pool), so a ranking that drifts costs more exact gradients rather
than a wrong selection.

Scores are residual: an operator's score is its base, the floored log of
its last exact gradient max(log10(|g_prev| + 1e-12), T_FLOOR), plus the
network's output, which is trained on the change of the floored log gradient
since that value (an untrained network ranks like |g_prev|).  The floor keeps
the regression on the large gradients that decide the selection rather than
the many near-zero ones.  Offline training keeps, per exact sweep, the rows
within BAND decades of the sweep's largest floored target plus REST_FRAC of
the others.
"""
from __future__ import annotations

import ctypes

import time

import numpy as np

from . import _lib
from ._lib import check
from . import _dev_ptr, _stream, _torch, _dtype_code, Adapt, Sector

N_FEAT = 32
RHO = 0.5      # fallback when |g| outside the top K_t reaches RHO of the top's largest
GROW = 1.5     # K_t keeps GROW x the worst rank of a true argmax seen at a full sweep
T_FLOOR = -4.0
BAND = 2.0
REST_FRAC = 0.1
N_PARAM = 256 * 32 + 256 + 256 * 256 + 256 + 256 + 1


class MLP:
    """hyp_mlp: the screen's network, parameters on the device."""

    def __init__(self, init_params, max_rows: int):
        p = np.ascontiguousarray(init_params, dtype=np.float32)
        if p.size != N_PARAM:
            raise ValueError(f"expected {N_PARAM} parameters")
        h = ctypes.c_void_p()
        check(_lib.load().hyp_mlp_create(p.ctypes.data, int(max_rows), ctypes.byref(h)))
        self._h = h
        self.max_rows = int(max_rows)

    def params(self) -> np.ndarray:
        out = np.empty(N_PARAM, dtype=np.float32)
        check(_lib.load().hyp_mlp_params(self._h, out.ctypes.data))
        return out

    def state(self) -> np.ndarray:
        """Parameters, Adam moments and step count (3 N_PARAM + 1 floats)."""
        out = np.empty(3 * N_PARAM + 1, dtype=np.float32)
        check(_lib.load().hyp_mlp_get_state(self._h, out.ctypes.data))
        return out

    def load_state(self, st):
        st = np.ascontiguousarray(st, dtype=np.float32)
        if st.size != 3 * N_PARAM + 1:
            raise ValueError(f"expected {3 * N_PARAM + 1} floats")
        check(_lib.load().hyp_mlp_set_state(self._h, st.ctypes.data))

    def clone(self, max_rows=None) -> "MLP":
        """An independent network with the same parameters and optimiser state."""
        c = MLP(self.params(), self.max_rows if max_rows is None else max_rows)
        c.load_state(self.state())
        return c

    def grads(self) -> np.ndarray:
        out = np.empty(N_PARAM, dtype=np.float32)
        check(_lib.load().hyp_mlp_grads(self._h, out.ctypes.data))
        return out

    def forward(self, X, y=None):
        torch = _torch()
        n = X.shape[0]
        if y is None:
            y = torch.empty(n, dtype=torch.float32, device=X.device)
        check(_lib.load().hyp_mlp_forward(self._h, _dev_ptr(X, n * N_FEAT, "X"), n,
                                          _dev_ptr(y, n, "y"), _stream()))
        return y

    def train_step(self, X, t, lr=1e-3, y=None):
        torch = _torch()
        B = X.shape[0]
        if y is None:
            y = torch.empty(B, dtype=torch.float32, device=X.device)
        check(_lib.load().hyp_mlp_train_step(self._h, _dev_ptr(X, B * N_FEAT, "X"), _dev_ptr(t, B, "t"),
                                             B, ctypes.c_float(lr), _dev_ptr(y, B, "y"), _stream()))
        return y

    def rank(self, y, base=None, order=None):
        """Operator indices by descending y + base (base None: y)."""
        torch = _torch()
        n = y.shape[0]
        if order is None:
            order = torch.empty(n, dtype=torch.int32, device=y.device)
        bp = _dev_ptr(base, n, "base") if base is not None else None
        check(_lib.load().hyp_rank_scores(self._h, _dev_ptr(y, n, "y"), bp, n, _dev_ptr(order, n, "order"),
                                          _stream()))
        return order

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().hyp_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def static_features(n_orb, cre, ann, cls, h, g):
    """(stat [n][32] float32, qidx [n][4] int32) from hyp_screen_static."""
    n = len(cre)
    pool = (_lib.HypExc * n)()
    for i, (c_, a_) in enumerate(zip(np.asarray(cre).tolist(), np.asarray(ann).tolist())):
        pool[i].cre, pool[i].ann = int(c_), int(a_)
    cls = np.ascontiguousarray(cls, dtype=np.uint8)
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    stat = np.empty((n, N_FEAT), dtype=np.float32)
    qidx = np.empty((n, 4), dtype=np.int32)
    check(_lib.load().hyp_screen_static(int(n_orb), pool, cls.ctypes.data, n, h.ctypes.data, g.ctypes.data,
                                        stat.ctypes.data, qidx.ctypes.data))
    return stat, qidx


class FeatureState:
    """Device buffers of one problem's features: static rows, g_prev, age."""

    def __init__(self, sector: Sector, stat, qidx, dtype="f64"):
        torch = _torch()
        self.sector = sector
        self.n = stat.shape[0]
        self.stat = torch.from_numpy(stat).cuda()
        self.qidx = torch.from_numpy(qidx).cuda()
        self.gprev = torch.zeros(self.n, dtype=torch.float64, device="cuda")
        self.age = torch.full((self.n,), 50, dtype=torch.int32, device="cuda")
        self.occ = torch.zeros(2 * sector.n_orb, dtype=torch.float64, device="cuda")
        db = int(round(sector.dim / _comb(sector.n_orb, sector.n_alpha)))
        self.work = torch.zeros(db * 17, dtype=torch.float64, device="cuda")
        self.X = torch.empty((self.n, N_FEAT), dtype=torch.int16, device="cuda")
        self.base = torch.empty(self.n, dtype=torch.float32, device="cuda")
        self.gdev = torch.empty(self.n, dtype=torch.float64, device="cuda")
        self.qidx_host = np.ascontiguousarray(qidx, dtype=np.int32)
        self.last = np.full(4, -1, dtype=np.int32)  # the last selected operator (qidx layout)
        self.last_g = 0.0

    def features(self, psi):
        """Feature rows and base scores of the current state (from g_prev as
        it stands before this iteration's exact gradients)."""
        L = _lib.load()
        check(L.hyp_occupations(self.sector.handle, _dtype_code(psi), _dev_ptr(psi, self.sector.dim, "psi"),
                                _dev_ptr(self.occ, None), _dev_ptr(self.work, None), _stream()))
        check(L.hyp_features(_dev_ptr(self.stat, None), _dev_ptr(self.qidx, None), _dev_ptr(self.occ, None),
                             _dev_ptr(self.gprev, None), _dev_ptr(self.age, None), self.n,
                             int(self.sector.n_orb), self.last.ctypes.data, float(self.last_g),
                             _dev_ptr(self.X, None), _stream()))
        check(L.hyp_screen_base(_dev_ptr(self.gprev, None), self.n, ctypes.c_float(T_FLOOR),
                                _dev_ptr(self.base, None), _stream()))
        return self.X

    def update(self, g_host):
        """Record exact gradients (NaN = not computed) as g_prev / age."""
        torch = _torch()
        self.gdev.copy_(torch.from_numpy(np.ascontiguousarray(g_host, dtype=np.float64)))
        check(_lib.load().hyp_screen_update(_dev_ptr(self.gdev, None), self.n, _dev_ptr(self.gprev, None),
                                            _dev_ptr(self.age, None), _stream()))

    def note_selected(self, k: int, g_sel: float):
        """After operator k was appended (selected with |g| = g_sel) and the
        parameters re-optimised: it becomes the last selection of the
        features, and its own pool gradient is known exactly, since at the
        optimum it equals dE/dtheta of its newly appended parameter (zero up
        to the optimiser's tolerance)."""
        self.last = self.qidx_host[int(k)].copy()
        self.last_g = float(abs(g_sel))
        self.gprev[int(k)] = 0.0
        self.age[int(k)] = 0

    def rows(self, idx, t_floor=T_FLOOR, residual=True):
        """(X rows, targets max(log10(|g| + 1e-12), t_floor) - base) of the
        operators idx, from gdev (no base subtracted if residual is False)."""
        torch = _torch()
        idx_d = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
        m = idx_d.shape[0]
        Xo = torch.empty((m, N_FEAT), dtype=torch.int16, device="cuda")
        t = torch.empty(m, dtype=torch.float32, device="cuda")
        check(_lib.load().hyp_screen_batch(_dev_ptr(self.X, None), _dev_ptr(self.gdev, None),
                                           _dev_ptr(idx_d, None), m, ctypes.c_float(t_floor),
                                           _dev_ptr(self.base, None) if residual else None,
                                           _dev_ptr(Xo, None), _dev_ptr(t, None), _stream()))
        return Xo, t


def _comb(n, k):
    import math
    return math.comb(n, k)


def audit_ranks(n_rest: int, n_audit: int, seed: int, iteration: int):
    """Audit positions among the operators ranked below the top-K: a uniform
    sample without replacement from a generator seeded by (seed, iteration)."""
    rng = np.random.default_rng([seed, iteration])
    m = min(n_audit, n_rest)
    return np.sort(rng.choice(n_rest, m, replace=False)) if m > 0 else np.zeros(0, dtype=np.int64)


def candidate_ranks(n: int, k_top: int, audit: int, seed: int, iteration: int):
    """Rank positions (into the descending score order) of one screened
    iteration's candidates: the top k_top, the band of the next audit // 2
    ranks (a true argmax ranked just past the top is the likeliest miss), and
    audit - audit // 2 uniform positions below the band."""
    k_top = min(k_top, n)
    band = min(audit // 2, n - k_top)
    below = n - k_top - band
    aud = k_top + band + audit_ranks(below, audit - audit // 2, seed, iteration)
    return np.arange(k_top), np.arange(k_top, k_top + band), aud


def widen_top(k_now: int, true_rank: int, n: int, k_min: int) -> int:
    """Top size after a full sweep whose true argmax the network ranked at
    true_rank: wide enough to hold GROW x that rank (multiple of 64), never
    narrower than before, at most half the pool."""
    want = int(np.ceil(GROW * (true_rank + 1) / 64.0)) * 64
    return int(min(max(k_now, k_min, want), max(k_min, n // 2)))


class Screen:
    """Screened ADAPT iterations for one problem."""

    def __init__(self, adapt: Adapt, sector: Sector, stat, qidx, mlp: MLP, K=512, audit=256,
                 judge_every=10, seed=42, lr=1e-3, online=False, cost_policy=True):
        """online: one Adam step per iteration on the freshly computed rows (off
        by default: on the held-out 16-qubit run it pulled the network's
        ranking back toward |g_prev| and cost a selection).
        cost_policy: besides the judge iterations, take the exact full sweep
        whenever the last full sweep's gradient phase took no longer than the
        last screened one (near Hartree-Fock the support-restricted sweep is
        cheaper than scoring the pool; the screen pays once the state fills)."""
        self.adapt = adapt
        self.fs = FeatureState(sector, stat, qidx)
        self.mlp = mlp
        self.K, self.audit, self.judge_every, self.seed, self.lr = K, audit, judge_every, seed, lr
        self.k_top = K  # K_t: widened by widen_top after full sweeps
        self.online = online
        self.cost_policy = cost_policy
        self.full_ms = None
        self.screen_ms = None
        self.n = stat.shape[0]
        self.psi = None
        self.log = []

    def iterate(self, it: int, shadow: bool = False) -> dict:
        """One screened iteration.  shadow=True also runs the full sweep on
        the same state first (not used for the selection) and reports its
        largest |g| and whether the screened pick lies in its tie set."""
        torch = _torch()
        n = self.n
        judge = (it % self.judge_every == 0) or n <= self.K + self.audit
        cheaper = (self.cost_policy and not judge and self.full_ms is not None and self.screen_ms is not None
                   and self.full_ms <= self.screen_ms)
        full = judge or cheaper
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.psi = self.adapt.state(self.psi)
        X = self.fs.features(self.psi)
        if shadow:
            self._base_host = self.fs.base.cpu().numpy()  # diagnostic: the |g_prev| ranking
        info = {"iteration": it, "judge": judge, "cheaper_full": cheaper, "fallback": False}
        g_shadow = None
        if shadow and not full:
            torch.cuda.synchronize()
            ts = time.perf_counter()
            self.adapt.gradients(None)
            g_shadow = np.abs(self.adapt.last_gradients())
            torch.cuda.synchronize()
            shadow_ms = (time.perf_counter() - ts) * 1e3
        order = None
        info["k_top"] = self.k_top
        if full:
            if judge and not cheaper:
                # the judge also ranks the pool, to see where the network put the argmax
                y = self.mlp.forward(X)
                order = self.mlp.rank(y, self.fs.base).cpu().numpy()
            rec = self.adapt.gradients(None)
            cand = np.arange(n)
        else:
            y = self.mlp.forward(X)
            order = self.mlp.rank(y, self.fs.base).cpu().numpy()
            r_top, r_band, r_aud = candidate_ranks(n, self.k_top, self.audit, self.seed, it)
            top = order[r_top]
            out = order[np.concatenate([r_band, r_aud])]
            cand = np.concatenate([top, out]).astype(np.int32)
            rec = self.adapt.gradients(cand)
            g = self.adapt.last_gradients()
            if out.size and np.nanmax(np.abs(g[out])) >= RHO * np.nanmax(np.abs(g[top])):
                info["fallback"] = True
                rec = self.adapt.gradients(None)
                cand = np.arange(n)
        if order is not None and cand.size == n:
            # a full sweep on a ranked iteration: the rank of the true argmax
            ga = np.abs(self.adapt.last_gradients())
            true_rank = int(np.nonzero(order == int(np.argmax(ga)))[0][0])
            info["true_rank"] = true_rank
            self.k_top = widen_top(self.k_top, true_rank, n, self.K)
        torch.cuda.synchronize()
        phase_ms = (time.perf_counter() - t0) * 1e3
        if g_shadow is not None:
            phase_ms -= shadow_ms
        if full:
            self.full_ms = phase_ms
        elif not info["fallback"]:
            self.screen_ms = phase_ms
        info["grad_phase_ms"] = phase_ms
        g = self.adapt.last_gradients()
        self.fs.update(g)
        if self.online:
            m = (cand.size // 16) * 16
            if m >= 16:
                pick = cand[:m] if m == cand.size else np.sort(
                    np.random.default_rng([self.seed, it, 1]).choice(cand, m, replace=False))
                for lo in range(0, m, self.mlp.max_rows // 16 * 16):
                    sl = pick[lo: lo + self.mlp.max_rows // 16 * 16]
                    Xb, tb = self.fs.rows(sl)
                    self.mlp.train_step(Xb, tb, self.lr)
        rec2 = self.adapt.select_optimize()
        if rec2["selected"] >= 0:
            self.fs.note_selected(rec2["selected"], g[rec2["selected"]])
        info.update(rec2)
        info["n_exact"] = int(np.count_nonzero(~np.isnan(g)))
        if g_shadow is not None:
            gm = float(g_shadow.max())
            kstar = int(np.argmax(g_shadow))
            info["shadow_gmax"] = gm
            info["shadow_agree"] = bool(rec2["selected"] >= 0 and g_shadow[rec2["selected"]] >= gm * (1 - 1e-6))
            info["shadow_argmax"] = kstar
            info["shadow_in_candidates"] = bool(np.isin(kstar, cand))
            if not full and not info["fallback"]:
                info["shadow_rank"] = int(np.nonzero(order == kstar)[0][0])
                base_h = self._base_host
                info["shadow_rank_heuristic"] = int(np.nonzero(np.argsort(-base_h, kind="stable") == kstar)[0][0])
        elif full:
            info["shadow_agree"] = True
        self.log.append(info)
        torch.cuda.synchronize()
        return info


def training_rows(t, rng, band=BAND, rest_frac=REST_FRAC):
    """Rows of one exact sweep kept for training: every operator whose target
    lies within `band` decades of the sweep's largest, plus a uniform sample
    of `rest_frac` of the others (at least one).  Sorted indices."""
    t = np.asarray(t)
    top = np.nonzero(t >= t.max() - band)[0]
    rest = np.setdiff1d(np.arange(t.size), top)
    m = min(rest.size, max(1, int(rest.size * rest_frac)))
    pick = rng.choice(rest, m, replace=False) if m > 0 else np.zeros(0, dtype=np.int64)
    return np.sort(np.concatenate([top, pick]))


def collect_rows(adapt: Adapt, fs: FeatureState, n_iter: int, seed: int = 0, select: bool = True):
    """Plain ADAPT with full sweeps; after each sweep the feature rows (built
    before the sweep) and the floored log targets, thinned by training_rows
    (all rows if select is False).  Returns host arrays (X int16 bit patterns
    [rows][32], t float32 [rows])."""
    Xs, ts = [], []
    psi = None
    for it in range(n_iter):
        psi = adapt.state(psi)
        X = fs.features(psi)
        rec = adapt.gradients(None)
        g = adapt.last_gradients()
        fs.update(g)
        Xr, tr = fs.rows(np.arange(fs.n))
        Xh, th = Xr.cpu().numpy(), tr.cpu().numpy()
        if select:
            absolute = th + fs.base.cpu().numpy()
            keep = training_rows(absolute, np.random.default_rng([seed, it]))
            Xh, th = Xh[keep], th[keep]
        Xs.append(Xh)
        ts.append(th)
        r2 = adapt.select_optimize()
        if r2["selected"] < 0:
            break
        fs.note_selected(r2["selected"], g[r2["selected"]])
        del X, rec
    return np.concatenate(Xs), np.concatenate(ts)


def train(mlp: MLP, X, t, epochs=3, batch=1024, lr=1e-3, seed=0):
    """Shuffled mini-batch Adam on host arrays (X int16 [rows][32], t float32)."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    n = (X.shape[0] // batch) * batch
    losses = []
    Xd = torch.from_numpy(X).cuda()
    td = torch.from_numpy(t).cuda()
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(X.shape[0])[:n].astype(np.int64)).cuda()
        tot = 0.0
        for b in range(0, n, batch):
            idx = perm[b: b + batch]
            Xb = Xd.index_select(0, idx).contiguous()
            tb = td.index_select(0, idx).contiguous()
            y = mlp.train_step(Xb, tb, lr)
            d = y.cpu().numpy().astype(np.float64) - tb.cpu().numpy()
            tot += float(np.mean(d * d))
        losses.append(tot / max(1, n // batch))
    return losses
