"""Learned surrogate of the Vecchia conditional densities (binding and
driver of include/vecchia_surrogate.h).

* ``MLP``          device-resident network: FP32 parameters with their BF16
                   copy and Adam moments; forward, loss/gradient and Adam
                   steps run in the library's kernels.
* ``training_set`` neighbourhoods solved exactly by the FP64 kernel
                   (vec_kriging_weights): inputs from vec_surrogate_features,
                   targets = kriging weights and scaled log variance.
* ``train``        mini-batch Adam over a training set on the device.
* ``SurrogateLoglik`` the profile log-likelihood of a problem with the
                   network serving the neighbourhoods it can and the exact
                   kernel the ones it hands back (vec_loglik_sums_at), then
                   the combine step (vec_combine_loglik).

Host code only marshals arguments and loops; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import synthetic as S
from . import vecchia as V

M = 30
IN, HID, OUT = 64, 256, 32
_VP = ctypes.c_void_p


def _lib():
    L = V.lib()
    if not getattr(L, "_surrogate_ready", False):
        pp = ctypes.POINTER(V.Problem)
        L.vec_mlp_param_count.restype = ctypes.c_int64
        L.vec_mlp_param_count.argtypes = []
        L.vec_mlp_workspace_bytes.restype = ctypes.c_size_t
        L.vec_mlp_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
        L.vec_mlp_forward.restype = ctypes.c_int
        L.vec_mlp_forward.argtypes = [ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t,
                                      _VP]
        L.vec_mlp_loss_grad.restype = ctypes.c_int
        L.vec_mlp_loss_grad.argtypes = [ctypes.c_int64, _VP, _VP, _VP, ctypes.c_float, _VP, _VP,
                                        _VP, _VP, _VP, ctypes.c_size_t, _VP]
        L.vec_mlp_adam.restype = ctypes.c_int
        L.vec_mlp_adam.argtypes = [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP]
        L.vec_mlp_to_bf16.restype = ctypes.c_int
        L.vec_mlp_to_bf16.argtypes = [_VP, _VP, _VP]
        L.vec_surrogate_features.restype = ctypes.c_int
        L.vec_surrogate_features.argtypes = [pp, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_float, ctypes.c_float, _VP, _VP, _VP]
        L.vec_surrogate_workspace_bytes.restype = ctypes.c_size_t
        L.vec_surrogate_workspace_bytes.argtypes = [pp]
        L.vec_surrogate_sums.restype = ctypes.c_int
        L.vec_surrogate_sums.argtypes = [pp, _VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int64,
                                         _VP, _VP, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, _VP, ctypes.c_int32, _VP,
                                         _VP, _VP, ctypes.c_size_t, _VP]
        L.vec_loglik_sums_at.restype = ctypes.c_int
        L.vec_loglik_sums_at.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP,
                                         _VP, ctypes.c_size_t, _VP, _VP]
        L.vec_combine_loglik.restype = ctypes.c_int
        L.vec_combine_loglik.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP]
        L._surrogate_ready = True
    return L


def _check(rc, where):
    if rc != V.VEC_OK:
        raise V.VecchiaError(rc, where)


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _pad32(n: int) -> int:
    return (n + 31) // 32 * 32


class MLP:
    """Network parameters on the device (FP32 master, BF16 copy) and the
    output scaling of the log variance."""

    def __init__(self, seed: int = 0, device: str = "cuda", params: np.ndarray | None = None,
                 lv_shift: float = 0.0, lv_scale: float = 1.0):
        L = _lib()
        self.n = int(L.vec_mlp_param_count())
        if params is None:
            params = init_params(seed)
        assert params.size == self.n
        self.device = torch.device(device)
        self.p32 = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        self.p16 = torch.empty(self.n, dtype=torch.bfloat16, device=self.device)
        self.m1 = torch.zeros_like(self.p32)
        self.m2 = torch.zeros_like(self.p32)
        self.grad = torch.zeros_like(self.p32)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.step = 0
        self.lv_shift, self.lv_scale = float(lv_shift), float(lv_scale)
        self._ws = {}
        _check(L.vec_mlp_to_bf16(self.p32.data_ptr(), self.p16.data_ptr(), _stream()),
               "vec_mlp_to_bf16")

    def _work(self, rows: int, training: bool) -> torch.Tensor:
        key = (rows, training)
        if key not in self._ws:
            nb = _lib().vec_mlp_workspace_bytes(rows, int(training))
            if nb == 0:
                raise V.VecchiaError(V.VEC_EINVAL, "vec_mlp_workspace_bytes")
            self._ws = {key: torch.empty(nb, dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def forward(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        rows = x.shape[0]
        if y is None:
            y = torch.empty(rows, OUT, dtype=torch.float32, device=self.device)
        ws = self._work(rows, False)
        _check(_lib().vec_mlp_forward(rows, x.data_ptr(), self.p32.data_ptr(),
                                      self.p16.data_ptr(), y.data_ptr(), ws.data_ptr(),
                                      ws.numel(), _stream()), "vec_mlp_forward")
        return y

    def loss_grad(self, x, targets, colw, scale: float) -> torch.Tensor:
        rows = x.shape[0]
        ws = self._work(rows, True)
        _check(_lib().vec_mlp_loss_grad(rows, x.data_ptr(), targets.data_ptr(), colw.data_ptr(),
                                        float(scale), self.p32.data_ptr(), self.p16.data_ptr(),
                                        self.grad.data_ptr(), self.loss.data_ptr(),
                                        ws.data_ptr(), ws.numel(), _stream()),
               "vec_mlp_loss_grad")
        return self.loss

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        _check(_lib().vec_mlp_adam(self.grad.data_ptr(), self.p32.data_ptr(),
                                   self.p16.data_ptr(), self.m1.data_ptr(), self.m2.data_ptr(),
                                   self.step, float(lr), float(beta1), float(beta2), float(eps),
                                   _stream()), "vec_mlp_adam")

    def state(self) -> dict:
        return dict(params=self.p32.cpu().numpy(), lv_shift=self.lv_shift,
                    lv_scale=self.lv_scale)


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases (layout of vecchia_surrogate.h)."""
    rng = np.random.default_rng(seed)
    shapes = [(HID, IN), (HID, HID), (HID, HID), (OUT, HID)]
    parts = []
    for a, b in shapes:
        lim = math.sqrt(6.0 / (a + b))
        parts.append(rng.uniform(-lim, lim, size=a * b))
        parts.append(np.zeros(a))
    return np.concatenate(parts)


def features(ev: V.Vecchia, covparms, i0: int, i1: int, dist_lo: float, dist_hi: float,
             feat: torch.Tensor | None = None, flag: torch.Tensor | None = None):
    """Network inputs (BF16 [rows][64], rows = i1 - i0 padded to 32 with zero
    rows) and the hand-back flags of observations [i0, i1)."""
    rows = _pad32(i1 - i0)
    cp = ev.covparms(covparms) if not (isinstance(covparms, torch.Tensor) and covparms.is_cuda) \
        else covparms
    if feat is None:
        feat = torch.zeros(rows, IN, dtype=torch.bfloat16, device=ev.device)
    if flag is None:
        flag = torch.zeros(rows, dtype=torch.uint8, device=ev.device)
    _check(_lib().vec_surrogate_features(ctypes.byref(ev.pb), ev.locs.data_ptr(),
                                         ev.NN.data_ptr(), cp.data_ptr(), i0, i1,
                                         float(dist_lo), float(dist_hi), feat.data_ptr(),
                                         flag.data_ptr(), _stream()), "vec_surrogate_features")
    return feat, flag


def training_set(n_neigh: int, seed: int = 6, n_min: int = 5_000, n_max: int = 200_000,
                 rho_range=(0.02, 0.5), tau2_range=(0.01, 0.5), nus=(0.5, 1.5, 2.5),
                 draws_per_set: int = 8, workers: int | None = None, log=None):
    """About n_neigh neighbourhoods with inputs and exact targets.  Point
    sets: maxmin-ordered uniform 2-D points (observations i >= m); each set
    is used with draws_per_set covariance parameter draws (log-uniform range,
    uniform nugget ratio, smoothness from nus: the batched workload's ranges,
    the range widened towards denser geometries).  Point sets are drawn on
    host processes; weights and features come from the library's kernels.
    Returns (x BF16 [N][64], raw targets FP64 [N][31] = (b, log v / sigma2),
    range of the neighbour offset lengths)."""
    rng = np.random.default_rng(seed)
    per_set = draws_per_set * (0.5 * (n_min + n_max) - M)
    nsets = max(1, int(math.ceil(n_neigh / per_set)))
    w = S.batched_uneven(seed=int(rng.integers(1 << 30)), nsets=nsets, n_min=n_min, n_max=n_max,
                         ms=(M,), workers=workers)
    xs, ts = [], []
    lo, hi = np.inf, 0.0
    total = 0
    for b in range(nsets):
        d = S.batch_member(w, b)
        for _ in range(draws_per_set):
            rho = math.exp(rng.uniform(math.log(rho_range[0]), math.log(rho_range[1])))
            nu = float(rng.choice(nus))
            t2 = float(rng.uniform(*tau2_range))
            ev = V.Vecchia(d["locs"], d["NN"], d["y"], d["X"], V.FAMILY_ISO, nu, 0)
            cp = ev.covparms((1.0, rho, t2))
            n = ev.n
            W = ev.kriging_weights(cp, M, n)
            feat, _ = features(ev, cp, M, n, 0.0, 1e30)
            keep = n - M
            xs.append(feat[:keep])
            ts.append(W)
            f = feat[:keep, :2 * M].float()
            dist = torch.sqrt(f[:, 0::2] ** 2 + f[:, 1::2] ** 2)
            lo = min(lo, float(dist.min()))
            hi = max(hi, float(dist.max()))
            total += keep
            ev.check_status("training_set")
            if total >= n_neigh:
                break
        if log:
            log(f"training set: {b + 1} of {nsets} point sets, {total} neighbourhoods")
        if total >= n_neigh:
            break
    return torch.cat(xs), torch.cat(ts), (lo, hi)


def targets_of(raw: torch.Tensor, lv_shift: float, lv_scale: float) -> torch.Tensor:
    """FP32 training targets [N][32]: weights, (log v - shift) / scale, 0."""
    t = torch.zeros(raw.shape[0], OUT, dtype=torch.float32, device=raw.device)
    t[:, :M] = raw[:, :M].float()
    t[:, M] = ((raw[:, M] - lv_shift) / lv_scale).float()
    return t


def column_weights(lv_weight: float = 1.0, device="cuda") -> torch.Tensor:
    w = torch.ones(OUT, dtype=torch.float32, device=device)
    w[M] = lv_weight
    w[M + 1:] = 0.0
    return w


def train(mlp: MLP, x: torch.Tensor, t: torch.Tensor, epochs: int = 4, batch: int = 4096,
          lr: float = 1e-3, lr_final: float = 2e-5, lv_weight: float = 1.0, seed: int = 0,
          log=None) -> list:
    """Mini-batch Adam with a cosine learning-rate schedule; returns the mean
    loss of each epoch."""
    assert batch % 32 == 0
    N = x.shape[0]
    colw = column_weights(lv_weight, x.device)
    g = torch.Generator(device=x.device)
    g.manual_seed(seed)
    steps_per_epoch = N // batch
    total = epochs * steps_per_epoch
    hist = []
    k = 0
    for ep in range(epochs):
        perm = torch.randperm(N, device=x.device, generator=g)
        acc = torch.zeros(1, dtype=torch.float64, device=x.device)
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = x[idx].contiguous()
            tb = t[idx].contiguous()
            loss = mlp.loss_grad(xb, tb, colw, 1.0 / batch)
            acc += loss
            frac = k / max(1, total - 1)
            mlp.adam(lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac)))
            k += 1
        hist.append(float(acc) / max(1, steps_per_epoch))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    return hist


class SurrogateLoglik:
    """Profile log-likelihood of a 2-D isotropic problem (m = 30) with the
    network serving the neighbourhoods it can and the exact kernel the rest."""

    def __init__(self, ev: V.Vecchia, mlp: MLP, dist_range, chunk: int = 1 << 18,
                 lv_slack: float = 0.0, lv_floor: float = -1e30):
        assert ev.pb.m == M and ev.pb.family == V.FAMILY_ISO and ev.pb.d == 2
        self.ev, self.mlp = ev, mlp
        self.dist_lo, self.dist_hi = dist_range
        self.chunk = _pad32(chunk)
        self.lv_slack = lv_slack
        self.lv_floor = lv_floor
        dev = ev.device
        L = _lib()
        nr = 2 + ev.p * ev.p + ev.p
        self.raw_s = torch.zeros(nr, dtype=torch.float64, device=dev)
        self.raw_e = torch.zeros(nr, dtype=torch.float64, device=dev)
        self.raw_sum = torch.zeros(nr, dtype=torch.float64, device=dev)
        self.out = torch.zeros(1 + ev.p + ev.p * ev.p, dtype=torch.float64, device=dev)
        self.back = torch.zeros(ev.n, dtype=torch.int32, device=dev)
        self.nback = torch.zeros(1, dtype=torch.int32, device=dev)
        self.sws = torch.empty(L.vec_surrogate_workspace_bytes(ctypes.byref(ev.pb)),
                               dtype=torch.uint8, device=dev)
        self.feat = torch.zeros(self.chunk, IN, dtype=torch.bfloat16, device=dev)
        self.flag = torch.zeros(self.chunk, dtype=torch.uint8, device=dev)
        self.pred = torch.zeros(self.chunk, OUT, dtype=torch.float32, device=dev)

    def evaluate(self, covparms) -> dict:
        ev, L = self.ev, _lib()
        cp = ev.covparms(covparms) if not (isinstance(covparms, torch.Tensor) and
                                           covparms.is_cuda) else covparms
        self.nback.zero_()
        first = True
        # the first m observations have fewer neighbours: handed back too
        for i0 in range(0, ev.n, self.chunk):
            i1 = min(ev.n, i0 + self.chunk)
            rows = _pad32(i1 - i0)
            feat, flag = features(ev, cp, i0, i1, self.dist_lo, self.dist_hi, self.feat[:rows],
                                  self.flag[:rows])
            pred = self.mlp.forward(feat, self.pred[:rows])
            _check(L.vec_surrogate_sums(ctypes.byref(ev.pb), ev.NN.data_ptr(), ev.y.data_ptr(),
                                        ev.X.data_ptr(), cp.data_ptr(), i0, i1, pred.data_ptr(),
                                        flag.data_ptr(), self.mlp.lv_scale, self.mlp.lv_shift,
                                        self.lv_slack, self.lv_floor, self.raw_s.data_ptr(),
                                        int(not first),
                                        self.back.data_ptr(), self.nback.data_ptr(),
                                        self.sws.data_ptr(), self.sws.numel(), _stream()),
                   "vec_surrogate_sums")
            first = False
        nb = int(self.nback.item())
        ws = ev.workspace(0, max(nb, 1))
        _check(L.vec_loglik_sums_at(ctypes.byref(ev.pb), ev.locs.data_ptr(), ev.NN.data_ptr(),
                                    ev.y.data_ptr(), ev.X.data_ptr(), cp.data_ptr(),
                                    self.back.data_ptr(), nb, self.raw_e.data_ptr(),
                                    ws.data_ptr(), ws.numel() * 8, ev.status.data_ptr(),
                                    _stream()), "vec_loglik_sums_at")
        _check(L.vec_combine_loglik(ctypes.byref(ev.pb), self.raw_s.data_ptr(),
                                    self.raw_e.data_ptr(), self.raw_sum.data_ptr(),
                                    self.out.data_ptr(), ev.status.data_ptr(), _stream()),
               "vec_combine_loglik")
        ev.check_status("surrogate loglik")
        o = self.out.cpu().numpy()
        return dict(loglik=float(o[0]), betahat=o[1:1 + ev.p].copy(), handed_back=nb,
                    served=ev.n - nb)


def save(path: str, mlp: MLP, dist_range):
    st = mlp.state()
    np.savez(path, params=st["params"], lv_shift=st["lv_shift"], lv_scale=st["lv_scale"],
             dist_lo=dist_range[0], dist_hi=dist_range[1])


def load(path: str, device="cuda"):
    z = np.load(path, allow_pickle=False)
    mlp = MLP(params=z["params"].astype(np.float64), device=device, lv_shift=float(z["lv_shift"]),
              lv_scale=float(z["lv_scale"]))
    return mlp, (float(z["dist_lo"]), float(z["dist_hi"]))


def exact_loglik(ev: V.Vecchia, covparms) -> dict:
    """The exact FP64 path's profile log-likelihood (the judge of the
    surrogate's error)."""
    o = ev.loglik(covparms).cpu().numpy()
    return dict(loglik=float(o[0]), betahat=o[1:1 + ev.p].copy())



def validation_loss(mlp: MLP, x: torch.Tensor, t: torch.Tensor, lv_weight: float = 1.0,
                    batch: int = 8192) -> float:
    """Mean per-row loss of the network on held-out neighbourhoods."""
    colw = column_weights(lv_weight, x.device)
    N = x.shape[0] // batch * batch
    acc = 0.0
    for a in range(0, N, batch):
        acc += float(mlp.loss_grad(x[a:a + batch].contiguous(), t[a:a + batch].contiguous(), colw,
                                   1.0 / batch))
    return acc / max(1, N // batch)


def calibrate_floor(ev: V.Vecchia, mlp: MLP, dist_range, covparms, bound: float = 1e-6,
                    floors=None) -> dict:
    """The variance floor (log v / sigma2) that serves the most
    neighbourhoods while the surrogate's |loglik error| / n on the problem
    `ev` (a validation problem, judged by the exact path) stays within
    `bound`; returns that floor with its error and served count, and the
    whole sweep.  The last floor serves nothing, so one always qualifies."""
    exact = exact_loglik(ev, covparms)["loglik"]
    if floors is None:
        floors = [math.log(v) for v in (0.02, 0.05, 0.1, 0.2, 0.3, 0.5, 0.7, 0.9, 0.95, 0.99)]
        floors.append(1e30)  # serves nothing: the exact path
    sweep = []
    for f in floors:
        r = SurrogateLoglik(ev, mlp, dist_range, lv_floor=f).evaluate(covparms)
        err = abs(r["loglik"] - exact) / ev.n
        sweep.append(dict(floor=f, err=err, served=r["served"]))
    # among the floors within the bound, the one that serves the most
    within = [r for r in sweep if r["err"] <= bound]
    chosen = max(within, key=lambda r: r["served"]) if within else None
    return dict(chosen=chosen, sweep=sweep)
