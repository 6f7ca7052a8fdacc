"""Thin Python binding of libvecchia.so (include/vecchia.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.  If
the library has not been built this module raises on first use; there is no
CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvecchia.so")

VEC_OK, VEC_EINVAL, VEC_ENOTPD, VEC_EBADNN, VEC_ENONFINITE, VEC_EHIP, VEC_EWORKSPACE = \
    0, -1, -2, -3, -4, -5, -6
FAMILY_ISO, FAMILY_SPACETIME, FAMILY_ANISO = 0, 1, 2
ERRORS = {VEC_EINVAL: "invalid argument", VEC_ENOTPD: "covariance not positive definite",
          VEC_EBADNN: "malformed NNarray row", VEC_ENONFINITE: "non-finite value",
          VEC_EHIP: "HIP runtime error", VEC_EWORKSPACE: "workspace too small"}


class VecchiaError(RuntimeError):
    def __init__(self, code: int, where: str = "", bad_i: int | None = None):
        msg = f"{where}: {ERRORS.get(code, code)}"
        if bad_i is not None:
            msg += f" (first at observation {bad_i})"
        super().__init__(msg)
        self.code = code
        self.bad_i = bad_i


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int32), ("d", ctypes.c_int32),
                ("p", ctypes.c_int32), ("family", ctypes.c_int32), ("smoothness", ctypes.c_double),
                ("nspace", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None
_VP = ctypes.c_void_p


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2407_02740_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        pp = ctypes.POINTER(Problem)
        for name in ("vec_nparms", "vec_nraw", "vec_nout"):
            getattr(L, name).restype = ctypes.c_int
            getattr(L, name).argtypes = [pp]
        L.vec_max_m.restype = ctypes.c_int
        L.vec_max_m.argtypes = []
        L.vec_workspace_bytes.restype = ctypes.c_size_t
        L.vec_workspace_bytes.argtypes = [pp, ctypes.c_int64, ctypes.c_int64]
        L.vec_raw_sums.restype = ctypes.c_int
        L.vec_raw_sums.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int64,
                                   _VP, _VP, ctypes.c_size_t, _VP, _VP]
        L.vec_block_sums.restype = ctypes.c_int
        L.vec_block_sums.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_int64,
                                     _VP, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32), _VP, _VP]
        L.vec_combine.restype = ctypes.c_int
        L.vec_combine.argtypes = [pp, _VP, _VP, _VP, _VP]
        L.vecchia_loglik_grad_info.restype = ctypes.c_int
        L.vecchia_loglik_grad_info.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                           ctypes.c_size_t, _VP, _VP]
        L.vecchia_loglik_grad_info_noalloc.restype = ctypes.c_int
        L.vecchia_loglik_grad_info_noalloc.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                                       _VP]
        L.vec_loglik.restype = ctypes.c_int
        L.vec_loglik.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP,
                                 _VP]
        L.vec_loglik_adjoint.restype = ctypes.c_int
        L.vec_loglik_adjoint.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                         ctypes.c_size_t, _VP, _VP]
        L.vec_kriging_weights.restype = ctypes.c_int
        L.vec_kriging_weights.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64,
                                          ctypes.c_int64, _VP, _VP, _VP, ctypes.c_size_t, _VP, _VP]
        L.vec_kriging_predict_workspace_bytes.restype = ctypes.c_size_t
        L.vec_kriging_predict_workspace_bytes.argtypes = [pp, ctypes.c_int64]
        L.vec_kriging_predict.restype = ctypes.c_int
        L.vec_kriging_predict.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP,
                                          _VP, _VP, ctypes.c_size_t, _VP, _VP]
        L.vec_ordered_nn_workspace_bytes.restype = ctypes.c_size_t
        L.vec_ordered_nn_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32,
                                                     ctypes.c_int32]
        L.vec_ordered_nn.restype = ctypes.c_int
        L.vec_ordered_nn.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP,
                                     ctypes.c_size_t, _VP]
        L.vec_maxmin_order_workspace_bytes.restype = ctypes.c_size_t
        L.vec_maxmin_order_workspace_bytes.argtypes = [ctypes.c_int64, ctypes.c_int32]
        L.vec_maxmin_order.restype = ctypes.c_int
        L.vec_maxmin_order.argtypes = [ctypes.c_int64, ctypes.c_int32, _VP, _VP, _VP, _VP, _VP,
                                       ctypes.c_size_t, _VP]
        L.vec_grouped_workspace_bytes.restype = ctypes.c_size_t
        L.vec_grouped_workspace_bytes.argtypes = [pp, ctypes.c_int64]
        L.vec_grouped_raw_sums.restype = ctypes.c_int
        L.vec_grouped_raw_sums.argtypes = [pp, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP, _VP, _VP,
                                           ctypes.c_int64, ctypes.c_int32, _VP, _VP,
                                           ctypes.c_size_t, _VP, _VP]
        L.vec_grouped_fisher_fit.restype = ctypes.c_int
        L.vec_grouped_fisher_fit.argtypes = [pp, _VP, _VP, _VP, _VP, ctypes.c_int64, _VP, _VP, _VP,
                                             ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_double, _VP, _VP, _VP, ctypes.c_size_t, _VP,
                                             ctypes.c_int32, _VP]
        L.vec_fisher_update.restype = ctypes.c_int
        L.vec_fisher_update.argtypes = [pp, _VP, _VP, _VP, ctypes.c_double, _VP]
        L.vec_fisher_fit.restype = ctypes.c_int
        L.vec_fisher_fit.argtypes = [pp, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_double,
                                     _VP, _VP, _VP, ctypes.c_size_t, _VP, ctypes.c_int32, _VP]
        L.vec_status_clear.restype = ctypes.c_int
        L.vec_status_clear.argtypes = [_VP, _VP]
        L.vec_status_code.restype = ctypes.c_int
        L.vec_status_code.argtypes = [ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != VEC_OK:
        raise VecchiaError(rc, where)


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def nparms(family: int, d: int | None = None) -> int:
    if family == FAMILY_ANISO:
        if d is None:
            raise ValueError("the anisotropic family needs the dimension d")
        return d + 2
    return {FAMILY_ISO: 3, FAMILY_SPACETIME: 4}[family]


def nraw(p: int, P: int) -> int:
    return 2 + p * p + p + P * (2 + p * p + p) + P * P


def unpack_out(out, p: int, P: int) -> dict:
    """Split out[nout] = [loglik, grad[P], info[P][P], betahat[p], betainfo[p][p]]."""
    o = out.detach().double().cpu().numpy() if isinstance(out, torch.Tensor) else out
    return dict(loglik=float(o[0]), grad=o[1:1 + P].copy(),
                info=o[1 + P:1 + P + P * P].reshape(P, P).copy(),
                betahat=o[1 + P + P * P:1 + P + P * P + p].copy(),
                betainfo=o[1 + P + P * P + p:].reshape(p, p).copy())


class Vecchia:
    """Device-resident problem: inputs copied to the GPU once, then evaluated
    by the library entry points on the current torch stream."""

    def __init__(self, locs, NN, y, X, family: int = FAMILY_ISO, smoothness: float = 0.5,
                 nspace: int = 0, device: str = "cuda", _check_rows: bool = True):
        def f64(a):
            return torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)

        self.locs = f64(locs)
        if self.locs.dim() == 1:
            self.locs = self.locs[:, None].contiguous()
        self.NN = torch.as_tensor(NN, dtype=torch.int32).contiguous().to(device)
        self.y = f64(y)
        self.X = f64(X)
        if self.X.dim() == 1:
            self.X = self.X[:, None].contiguous()
        n, d = self.locs.shape
        # shapes are checked here: the kernels read NN, y and X by these sizes
        if self.NN.dim() != 2 or self.NN.shape[1] < 1 or (_check_rows and self.NN.shape[0] != n):
            raise ValueError(f"NN must be [n = {n}][m + 1], got {tuple(self.NN.shape)}")
        if self.y.shape != (n,):
            raise ValueError(f"y must be [n = {n}], got {tuple(self.y.shape)}")
        if self.X.dim() != 2 or self.X.shape[0] != n:
            raise ValueError(f"X must be [n = {n}][p], got {tuple(self.X.shape)}")
        self.pb = Problem(n=n, m=self.NN.shape[1] - 1, d=d, p=self.X.shape[1], family=family,
                          smoothness=float(smoothness), nspace=int(nspace), reserved=0)
        L = lib()
        self.P = L.vec_nparms(ctypes.byref(self.pb))
        if self.P < 0:
            raise VecchiaError(VEC_EINVAL, "problem description")
        self.p = self.pb.p
        self.n = n
        self.nraw = L.vec_nraw(ctypes.byref(self.pb))
        self.nout = L.vec_nout(ctypes.byref(self.pb))
        self.device = self.y.device
        self.status = torch.zeros(2, dtype=torch.int32, device=self.device)
        self.raw = torch.zeros(self.nraw, dtype=torch.float64, device=self.device)
        self.out = torch.zeros(self.nout, dtype=torch.float64, device=self.device)
        self._ws = None
        self.clear_status()

    # -- helpers ------------------------------------------------------------
    def workspace(self, i0: int = 0, i1: int | None = None) -> torch.Tensor:
        i1 = self.n if i1 is None else i1
        nb = lib().vec_workspace_bytes(ctypes.byref(self.pb), i0, i1)
        if nb == 0:
            raise VecchiaError(VEC_EINVAL, "vec_workspace_bytes")
        if self._ws is None or self._ws.numel() * 8 < nb:
            self._ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        return self._ws

    def covparms(self, covparms) -> torch.Tensor:
        """covparms as a contiguous FP64 device tensor of P entries: a device
        tensor that already is one is passed through (no copy), anything else
        is copied to the device."""
        if isinstance(covparms, torch.Tensor) and covparms.is_cuda:
            if covparms.numel() != self.P:
                raise ValueError(f"covparms needs {self.P} entries, got {covparms.numel()}")
            _dev(covparms, torch.float64, "covparms")
            return covparms
        t = torch.as_tensor(covparms, dtype=torch.float64).to(self.device).contiguous()
        if t.numel() != self.P:
            raise ValueError(f"covparms needs {self.P} entries")
        return t

    def _inplace_cp(self, covparms) -> torch.Tensor:
        # parameters updated in place on the device: must already be a
        # device tensor of P entries
        if not (isinstance(covparms, torch.Tensor) and covparms.is_cuda):
            raise TypeError("covparms must be a device tensor (updated in place)")
        return self.covparms(covparms)

    def clear_status(self):
        _check(lib().vec_status_clear(_dev(self.status, torch.int32, "status"), _stream()),
               "vec_status_clear")

    def check_status(self, where: str = "device"):
        host = self.status.cpu()
        arr = (ctypes.c_int32 * 2)(int(host[0]), int(host[1]))
        rc = lib().vec_status_code(arr)
        if rc != VEC_OK:
            raise VecchiaError(rc, where, int(host[1]))

    # -- entry points ---------------------------------------------------------
    def raw_sums(self, covparms, i0: int = 0, i1: int | None = None, check: bool = True):
        i1 = self.n if i1 is None else i1
        cp = self.covparms(covparms)
        ws = self.workspace(i0, i1)
        _check(lib().vec_raw_sums(ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(),
                                  self.y.data_ptr(), self.X.data_ptr(),
                                  _dev(cp, torch.float64, "covparms"), i0, i1,
                                  self.raw.data_ptr(), ws.data_ptr(), ws.numel() * 8,
                                  self.status.data_ptr(), _stream()), "vec_raw_sums")
        if check:
            self.check_status("vec_raw_sums")
        return self.raw

    def block_sums(self, covparms: torch.Tensor, i0: int = 0, i1: int | None = None) -> int:
        """Launch the fused kernel alone; returns the number of partial rows
        written to the workspace (no status check, no synchronisation)."""
        i1 = self.n if i1 is None else i1
        ws = self.workspace(i0, i1)
        nb = ctypes.c_int32(0)
        _check(lib().vec_block_sums(ctypes.byref(self.pb), self.locs.data_ptr(),
                                    self.NN.data_ptr(), self.y.data_ptr(), self.X.data_ptr(),
                                    _dev(covparms, torch.float64, "covparms"), i0, i1,
                                    ws.data_ptr(), ws.numel() * 8, ctypes.byref(nb),
                                    self.status.data_ptr(), _stream()), "vec_block_sums")
        return nb.value

    def loglik_grad_info(self, covparms, check: bool = True):
        cp = self.covparms(covparms)
        ws = self.workspace()
        _check(lib().vecchia_loglik_grad_info(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(cp, torch.float64, "covparms"), self.raw.data_ptr(),
            self.out.data_ptr(), ws.data_ptr(), ws.numel() * 8, self.status.data_ptr(), _stream()),
            "vecchia_loglik_grad_info")
        if check:
            self.check_status("vecchia_loglik_grad_info")
        return self.out

    def loglik_grad_info_noalloc(self, covparms, check: bool = True):
        """loglik_grad_info through the entry point that allocates nothing:
        the library's own per-device scratch array replaces the workspace."""
        cp = self.covparms(covparms)
        _check(lib().vecchia_loglik_grad_info_noalloc(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(cp, torch.float64, "covparms"), self.raw.data_ptr(),
            self.out.data_ptr(), self.status.data_ptr(), _stream()),
            "vecchia_loglik_grad_info_noalloc")
        if check:
            self.check_status("vecchia_loglik_grad_info_noalloc")
        return self.out

    def loglik(self, covparms, check: bool = True) -> torch.Tensor:
        """Profile log-likelihood alone (the sums of Algorithm 1 and the
        combine step): a new tensor [loglik, betahat[p], betainfo[p][p]]."""
        cp = self.covparms(covparms)
        ws = self.workspace()
        out = torch.empty(1 + self.p + self.p * self.p, dtype=torch.float64, device=self.device)
        _check(lib().vec_loglik(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(cp, torch.float64, "covparms"), self.raw.data_ptr(),
            out.data_ptr(), ws.data_ptr(), ws.numel() * 8, self.status.data_ptr(), _stream()),
            "vec_loglik")
        if check:
            self.check_status("vec_loglik")
        return out

    def loglik_adjoint(self, covparms, betahat, grad_out: torch.Tensor | None = None,
                       check: bool = True):
        """Reverse-mode gradient of the log-likelihood at the mean vector
        betahat, each neighbourhood's factor recomputed: returns new tensors
        (loglik at betahat, grad_out * d loglik / d covparms)."""
        cp = self.covparms(covparms)
        beta = torch.as_tensor(betahat, dtype=torch.float64).to(self.device).contiguous()
        if beta.numel() != self.p:
            raise ValueError(f"betahat needs {self.p} entries")
        go = 0
        if grad_out is not None:
            grad_out = grad_out.to(device=self.device, dtype=torch.float64).contiguous()
            go = _dev(grad_out, torch.float64, "grad_out")
        ws = self.workspace()
        ll = torch.empty(1, dtype=torch.float64, device=self.device)
        dcp = torch.empty(self.P, dtype=torch.float64, device=self.device)
        _check(lib().vec_loglik_adjoint(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(cp, torch.float64, "covparms"), beta.data_ptr(), go,
            ll.data_ptr(), dcp.data_ptr(), ws.data_ptr(), ws.numel() * 8,
            self.status.data_ptr(), _stream()), "vec_loglik_adjoint")
        if check:
            self.check_status("vec_loglik_adjoint")
        return ll, dcp

    def kriging_weights(self, covparms, i0: int = 0, i1: int | None = None,
                        out: torch.Tensor | None = None, check: bool = True) -> torch.Tensor:
        """Per observation of [i0, i1): kriging weights of its neighbours
        (NNarray column order) and log conditional variance in correlation
        units, [i1 - i0][m + 1] FP64; self.raw receives the loglik sums."""
        i1 = self.n if i1 is None else i1
        cp = self.covparms(covparms)
        m1 = self.pb.m + 1
        if out is None:
            out = torch.empty(max(i1 - i0, 0), m1, dtype=torch.float64, device=self.device)
        if out.shape != (i1 - i0, m1) or out.dtype != torch.float64 or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 [i1 - i0][m + 1] tensor")
        ws = self.workspace(i0, i1)
        _check(lib().vec_kriging_weights(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(cp, torch.float64, "covparms"), i0, i1, out.data_ptr(),
            self.raw.data_ptr(), ws.data_ptr(), ws.numel() * 8, self.status.data_ptr(),
            _stream()), "vec_kriging_weights")
        if check:
            self.check_status("vec_kriging_weights")
        return out

    def fisher_update(self, covparms: torch.Tensor, max_step: float = 1.0):
        covparms = self._inplace_cp(covparms)
        _check(lib().vec_fisher_update(ctypes.byref(self.pb), self.out.data_ptr(),
                                       _dev(covparms, torch.float64, "covparms"),
                                       self.status.data_ptr(), float(max_step), _stream()),
               "vec_fisher_update")
        return covparms

    def fisher_fit(self, covparms: torch.Tensor, iters: int, use_graph: bool = True,
                   max_step: float = 1.0, check: bool = True):
        covparms = self._inplace_cp(covparms)
        ws = self.workspace()
        _check(lib().vec_fisher_fit(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(covparms, torch.float64, "covparms"), int(iters),
            float(max_step), self.raw.data_ptr(), self.out.data_ptr(), ws.data_ptr(),
            ws.numel() * 8, self.status.data_ptr(), int(bool(use_graph)), _stream()),
            "vec_fisher_fit")
        if check:
            self.check_status("vec_fisher_fit")
        return covparms


def ordered_nn(locs, m: int, device: str = "cuda") -> torch.Tensor:
    """NNarray [n][m + 1] (int32, on the device) of the ordered points locs
    ([n][d], d <= 32; a grid search up to d = 4, exhaustive above) by the
    library's neighbour search (vec_ordered_nn)."""
    x = torch.as_tensor(locs, dtype=torch.float64).to(device).contiguous()
    if x.dim() == 1:
        x = x[:, None].contiguous()
    n, d = x.shape
    nb = lib().vec_ordered_nn_workspace_bytes(n, d, m)
    if nb == 0:
        raise VecchiaError(VEC_EINVAL, "vec_ordered_nn_workspace_bytes")
    ws = torch.empty(nb, dtype=torch.uint8, device=x.device)
    NN = torch.empty(n, m + 1, dtype=torch.int32, device=x.device)
    _check(lib().vec_ordered_nn(n, d, m, x.data_ptr(), NN.data_ptr(), ws.data_ptr(), nb,
                                _stream()), "vec_ordered_nn")
    return NN


def maxmin_order(locs, tie, device: str = "cuda"):
    """(order, reordered locs) of the points locs ([n][d], d <= 4) by the
    library's coarse-to-fine ordering (vec_maxmin_order); tie [n] breaks the
    order within a grid cell.  order is int64 on the device."""
    x = torch.as_tensor(locs, dtype=torch.float64).to(device).contiguous()
    if x.dim() == 1:
        x = x[:, None].contiguous()
    n, d = x.shape
    t = torch.as_tensor(tie, dtype=torch.float64).to(x.device).contiguous()
    if t.shape != (n,):
        raise ValueError("tie must hold one value per point")
    nb = lib().vec_maxmin_order_workspace_bytes(n, d)
    if nb == 0:
        raise VecchiaError(VEC_EINVAL, "vec_maxmin_order_workspace_bytes")
    ws = torch.empty(nb, dtype=torch.uint8, device=x.device)
    order = torch.empty(n, dtype=torch.int64, device=x.device)
    out = torch.empty_like(x)
    _check(lib().vec_maxmin_order(n, d, x.data_ptr(), t.data_ptr(), order.data_ptr(),
                                  out.data_ptr(), ws.data_ptr(), nb, _stream()),
           "vec_maxmin_order")
    return order, out


class GroupedVecchia(Vecchia):
    """Grouped Vecchia (vec_grouped_*): consecutive blocks of observations
    [block_start[b], block_start[b + 1]) with conditioning sets
    cond[cond_start[b]:cond_start[b + 1]] of earlier observations."""

    def __init__(self, locs, y, X, block_start, cond_start, cond, family: int = FAMILY_ISO,
                 smoothness: float = 0.5, nspace: int = 0, device: str = "cuda"):
        bs = np.asarray(block_start, dtype=np.int64)
        cs = np.asarray(cond_start, dtype=np.int64)
        m = int(np.diff(cs).max()) if len(cs) > 1 else 0
        self.max_block = int(np.diff(bs).max()) if len(bs) > 1 else 1
        self.nblocks = len(bs) - 1
        n = len(np.asarray(y))
        dummy_nn = np.zeros((1, m + 1), dtype=np.int32)
        super().__init__(locs, dummy_nn, y, X, family, smoothness, nspace, device,
                         _check_rows=False)
        self.pb.n = n
        self.n = n
        self.block_start = torch.as_tensor(bs, device=self.device)
        self.cond_start = torch.as_tensor(cs, device=self.device)
        c = np.asarray(cond, dtype=np.int32)
        self.cond = torch.as_tensor(c if c.size else np.zeros(1, np.int32), device=self.device)
        self.ncond = int(c.size)

    def workspace(self, i0: int = 0, i1: int | None = None) -> torch.Tensor:
        nb = lib().vec_grouped_workspace_bytes(ctypes.byref(self.pb), self.nblocks)
        if nb == 0:
            raise VecchiaError(VEC_EINVAL, "vec_grouped_workspace_bytes")
        if self._ws is None or self._ws.numel() * 8 < nb:
            self._ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        return self._ws

    def _blocks(self):
        return (self.nblocks, self.block_start.data_ptr(), self.cond_start.data_ptr(),
                self.cond.data_ptr(), self.ncond, self.max_block)

    def raw_sums(self, covparms, i0: int = 0, i1: int | None = None, check: bool = True):
        cp = self.covparms(covparms)
        ws = self.workspace()
        _check(lib().vec_grouped_raw_sums(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.y.data_ptr(), self.X.data_ptr(),
            _dev(cp, torch.float64, "covparms"), *self._blocks(), self.raw.data_ptr(),
            ws.data_ptr(), ws.numel() * 8, self.status.data_ptr(), _stream()),
            "vec_grouped_raw_sums")
        if check:
            self.check_status("vec_grouped_raw_sums")
        return self.raw

    def loglik_grad_info(self, covparms, check: bool = True):
        self.raw_sums(covparms, check=False)
        _check(lib().vec_combine(ctypes.byref(self.pb), self.raw.data_ptr(), self.out.data_ptr(),
                                 self.status.data_ptr(), _stream()), "vec_combine")
        if check:
            self.check_status("grouped loglik_grad_info")
        return self.out

    def fisher_fit(self, covparms: torch.Tensor, iters: int, use_graph: bool = True,
                   max_step: float = 1.0, check: bool = True):
        ws = self.workspace()
        covparms = self._inplace_cp(covparms)
        _check(lib().vec_grouped_fisher_fit(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.y.data_ptr(), self.X.data_ptr(),
            _dev(covparms, torch.float64, "covparms"), *self._blocks(), int(iters),
            float(max_step), self.raw.data_ptr(), self.out.data_ptr(), ws.data_ptr(),
            ws.numel() * 8, self.status.data_ptr(), int(bool(use_graph)), _stream()),
            "vec_grouped_fisher_fit")
        if check:
            self.check_status("vec_grouped_fisher_fit")
        return covparms

    def block_sums(self, *args, **kwargs):
        raise NotImplementedError("grouped problems reduce on the device (raw_sums)")


class Predictor:
    """Kriging prediction at new points from their m_pred nearest observed
    neighbours (vec_kriging_predict): the prediction points are appended to
    a copy of the observation arrays on the device.  m_pred is the width of
    NN_pred minus one and need not equal the m of the fitted model."""

    def __init__(self, ev: Vecchia, locs_pred, X_pred, NN_pred):
        dev = ev.device
        lp = torch.as_tensor(locs_pred, dtype=torch.float64).reshape(-1, ev.locs.shape[1]).to(dev)
        xp = torch.as_tensor(X_pred, dtype=torch.float64).reshape(-1, ev.p).to(dev)
        self.n_obs, self.n_pred = ev.n, lp.shape[0]
        self.locs = torch.cat([ev.locs, lp]).contiguous()
        self.y = torch.cat([ev.y, torch.zeros(self.n_pred, dtype=torch.float64, device=dev)])
        self.X = torch.cat([ev.X, xp]).contiguous()
        self.NN = torch.as_tensor(NN_pred, dtype=torch.int32).to(dev).contiguous()
        if self.NN.dim() != 2 or self.NN.shape[0] != self.n_pred or self.NN.shape[1] < 1:
            raise ValueError("NN_pred must be [n_pred][m_pred + 1]")
        self.pb = Problem(n=self.n_obs + self.n_pred, m=self.NN.shape[1] - 1, d=ev.pb.d, p=ev.p,
                          family=ev.pb.family, smoothness=ev.pb.smoothness,
                          nspace=ev.pb.nspace, reserved=0)
        self.ev = ev
        nb = lib().vec_kriging_predict_workspace_bytes(ctypes.byref(self.pb), self.n_obs)
        if nb == 0:
            raise VecchiaError(VEC_EINVAL, "vec_kriging_predict_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)

    def predict(self, covparms, betahat, check: bool = True):
        ev = self.ev
        cp = ev.covparms(covparms)
        beta = torch.as_tensor(betahat, dtype=torch.float64).to(ev.device).contiguous()
        mean = torch.empty(self.n_pred, dtype=torch.float64, device=ev.device)
        var = torch.empty_like(mean)
        _check(lib().vec_kriging_predict(
            ctypes.byref(self.pb), self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(),
            self.X.data_ptr(), _dev(cp, torch.float64, "covparms"), beta.data_ptr(), self.n_obs,
            mean.data_ptr(), var.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
            ev.status.data_ptr(), _stream()), "vec_kriging_predict")
        if check:
            ev.check_status("vec_kriging_predict")
        return mean, var


class VecchiaLoglik(torch.autograd.Function):
    """Profile log-likelihood as a differentiable function of covparms.

    forward:  the loglik-only pass (betahat comes with it).
    backward: the adjoint pass at that betahat, scaled by grad_output on the
              device.  Because betahat maximises the likelihood over the mean
              parameters, the derivative at fixed betahat is the derivative of
              the profile likelihood.
    Only covparms receives a gradient.
    """

    @staticmethod
    def forward(ctx, covparms: torch.Tensor, ev: "Vecchia", check: bool = True):
        cp = covparms.detach().to(device=ev.device, dtype=torch.float64).contiguous()
        out = ev.loglik(cp, check=check)
        ctx.ev = ev
        ctx.check = check
        ctx.save_for_backward(cp, out[1:1 + ev.p].clone())
        return out[0].clone()

    @staticmethod
    def backward(ctx, grad_output):
        cp, beta = ctx.saved_tensors
        _, dcp = ctx.ev.loglik_adjoint(cp, beta, grad_output.reshape(1), check=ctx.check)
        return dcp, None, None


def vecchia_loglik(ev: Vecchia, covparms: torch.Tensor, check: bool = True) -> torch.Tensor:
    """Differentiable profile log-likelihood (see VecchiaLoglik)."""
    return VecchiaLoglik.apply(covparms, ev, check)


# ---------------------------------------------------------------------------
# batches of independent datasets
# ---------------------------------------------------------------------------
NUM_CLASSES = 4
CLASS_K = (11, 21, 31, 41)


class Batch(ctypes.Structure):
    _fields_ = [("nsets", ctypes.c_int32), ("d", ctypes.c_int32), ("p", ctypes.c_int32),
                ("family", ctypes.c_int32), ("nspace", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_total", ctypes.c_int64),
                ("nn_total", ctypes.c_int64)]


class Dataset(ctypes.Structure):
    _fields_ = [("obs_offset", ctypes.c_int64), ("nn_offset", ctypes.c_int64),
                ("n", ctypes.c_int64), ("m", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("smoothness", ctypes.c_double)]


class Schedule(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32 * NUM_CLASSES),
                ("blocks_per_cu", ctypes.c_int32 * NUM_CLASSES)]


class Plan(ctypes.Structure):
    _fields_ = [("nsets", ctypes.c_int32), ("count", ctypes.c_int32 * NUM_CLASSES),
                ("grid", ctypes.c_int32 * NUM_CLASSES), ("reserved", ctypes.c_int32),
                ("ntiles", ctypes.c_int64 * NUM_CLASSES), ("rows", ctypes.c_int64),
                ("plan_bytes", ctypes.c_int64), ("sched", Schedule)]


def _batch_lib():
    L = lib()
    if not getattr(L, "_batch_ready", False):
        bp, pl, sc = ctypes.POINTER(Batch), ctypes.POINTER(Plan), ctypes.POINTER(Schedule)
        L.vec_batch_plan_bytes.restype = ctypes.c_size_t
        L.vec_batch_plan_bytes.argtypes = [ctypes.c_int32]
        L.vec_batch_make_plan.restype = ctypes.c_int
        L.vec_batch_make_plan.argtypes = [bp, ctypes.POINTER(Dataset), sc, pl, _VP,
                                          ctypes.c_size_t, _VP]
        L.vec_batch_workspace_bytes.restype = ctypes.c_size_t
        L.vec_batch_workspace_bytes.argtypes = [bp, pl]
        L.vec_batch_raw_sums.restype = ctypes.c_int
        L.vec_batch_raw_sums.argtypes = [bp, pl, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                         ctypes.c_size_t, _VP, _VP]
        L.vec_batch_loglik_grad_info.restype = ctypes.c_int
        L.vec_batch_loglik_grad_info.argtypes = [bp, pl, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP,
                                                 _VP, ctypes.c_size_t, _VP, _VP]
        L.vec_batch_fisher_fit.restype = ctypes.c_int
        L.vec_batch_fisher_fit.argtypes = [bp, pl, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32,
                                           ctypes.c_double, _VP, _VP, _VP, ctypes.c_size_t, _VP,
                                           ctypes.c_int32, _VP]
        L.vec_batch_status_clear.restype = ctypes.c_int
        L.vec_batch_status_clear.argtypes = [_VP, ctypes.c_int32, _VP]
        L._batch_ready = True
    return L


def schedule(tile=None, blocks_per_cu=None) -> Schedule:
    """A schedule from per-class lists (or one value for every class); 0 =
    the library default."""
    def four(v):
        if v is None:
            return [0] * NUM_CLASSES
        if isinstance(v, int):
            return [v] * NUM_CLASSES
        return list(v)
    s = Schedule()
    for c, (t, b) in enumerate(zip(four(tile), four(blocks_per_cu))):
        s.tile[c] = int(t)
        s.blocks_per_cu[c] = int(b)
    return s


class VecchiaBatch:
    """Many independent datasets resident on the device, evaluated together.

    locs, y, X are the concatenation of the datasets' arrays; NN_blocks is a
    list of per-dataset NNarray blocks (local indices) or their flat
    concatenation with the offsets in ``nn_offset``."""

    def __init__(self, locs, NN, y, X, obs_offset, nn_offset, n, m, smoothness,
                 family: int = FAMILY_ISO, nspace: int = 0, device: str = "cuda",
                 sched: Schedule | None = None):
        def f64(a):
            return torch.as_tensor(a, dtype=torch.float64).contiguous().to(device)

        self.locs = f64(locs)
        if self.locs.dim() == 1:
            self.locs = self.locs[:, None].contiguous()
        self.NN = torch.as_tensor(NN, dtype=torch.int32).reshape(-1).contiguous().to(device)
        self.y = f64(y)
        self.X = f64(X)
        if self.X.dim() == 1:
            self.X = self.X[:, None].contiguous()
        nsets = len(n)
        if self.y.dim() != 1 or self.X.shape[0] != self.locs.shape[0] or \
                self.y.shape[0] != self.locs.shape[0]:
            raise ValueError("locs, y and X must have the same number of rows")
        self.nsets = nsets
        self.sets = (Dataset * nsets)()
        for b in range(nsets):
            self.sets[b] = Dataset(obs_offset=int(obs_offset[b]), nn_offset=int(nn_offset[b]),
                                   n=int(n[b]), m=int(m[b]), reserved=0,
                                   smoothness=float(smoothness[b]))
        self.n = [int(v) for v in n]
        self.bt = Batch(nsets=nsets, d=self.locs.shape[1], p=self.X.shape[1], family=family,
                        nspace=int(nspace), reserved=0, n_total=self.locs.shape[0],
                        nn_total=self.NN.numel())
        self.p = self.bt.p
        pb = Problem(n=1, m=0, d=self.bt.d, p=self.p, family=family, smoothness=0.5,
                     nspace=int(nspace), reserved=0)
        L = _batch_lib()
        self.P = L.vec_nparms(ctypes.byref(pb))
        if self.P < 0:
            raise VecchiaError(VEC_EINVAL, "batch description")
        self.nraw = L.vec_nraw(ctypes.byref(pb))
        self.nout = L.vec_nout(ctypes.byref(pb))
        self.device = self.y.device
        nb = L.vec_batch_plan_bytes(nsets)
        if nb == 0:
            raise VecchiaError(VEC_EINVAL, "vec_batch_plan_bytes")
        self.plan_dev = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        self.status = torch.zeros(nsets, 2, dtype=torch.int32, device=self.device)
        self.raw = torch.zeros(nsets, self.nraw, dtype=torch.float64, device=self.device)
        self.out = torch.zeros(nsets, self.nout, dtype=torch.float64, device=self.device)
        self._ws = None
        self.make_plan(sched)
        self.clear_status()

    def make_plan(self, sched: Schedule | None = None):
        L = _batch_lib()
        self.plan = Plan()
        _check(L.vec_batch_make_plan(ctypes.byref(self.bt), self.sets,
                                     ctypes.byref(sched) if sched is not None else None,
                                     ctypes.byref(self.plan), self.plan_dev.data_ptr(),
                                     self.plan_dev.numel() * 8, _stream()), "vec_batch_make_plan")
        nb = L.vec_batch_workspace_bytes(ctypes.byref(self.bt), ctypes.byref(self.plan))
        if self._ws is None or self._ws.numel() * 8 < nb:
            self._ws = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        return self.plan

    def covparms(self, covparms) -> torch.Tensor:
        if isinstance(covparms, torch.Tensor) and covparms.is_cuda:
            if covparms.numel() != self.nsets * self.P:
                raise ValueError(f"covparms must be [{self.nsets}][{self.P}]")
            _dev(covparms, torch.float64, "covparms")
            return covparms
        t = torch.as_tensor(covparms, dtype=torch.float64).to(self.device).contiguous()
        if t.shape != (self.nsets, self.P):
            raise ValueError(f"covparms must be [{self.nsets}][{self.P}]")
        return t

    def clear_status(self):
        _check(_batch_lib().vec_batch_status_clear(self.status.data_ptr(), self.nsets, _stream()),
               "vec_batch_status_clear")

    def status_codes(self) -> list:
        host = self.status.cpu().numpy()
        L = lib()
        return [L.vec_status_code((ctypes.c_int32 * 2)(int(a), int(b))) for a, b in host]

    def check_status(self, where: str = "device"):
        host = self.status.cpu().numpy()
        for b, code in enumerate(self.status_codes()):
            if code != VEC_OK:
                raise VecchiaError(code, f"{where}, dataset {b}", int(host[b, 1]))

    def _args(self, cp):
        return (ctypes.byref(self.bt), ctypes.byref(self.plan), self.plan_dev.data_ptr(),
                self.locs.data_ptr(), self.NN.data_ptr(), self.y.data_ptr(), self.X.data_ptr(),
                _dev(cp, torch.float64, "covparms"))

    def raw_sums(self, covparms, check: bool = True):
        cp = self.covparms(covparms)
        _check(_batch_lib().vec_batch_raw_sums(*self._args(cp), self.raw.data_ptr(),
                                               self._ws.data_ptr(), self._ws.numel() * 8,
                                               self.status.data_ptr(), _stream()),
               "vec_batch_raw_sums")
        if check:
            self.check_status("vec_batch_raw_sums")
        return self.raw

    def loglik_grad_info(self, covparms, check: bool = True):
        cp = self.covparms(covparms)
        _check(_batch_lib().vec_batch_loglik_grad_info(
            *self._args(cp), self.raw.data_ptr(), self.out.data_ptr(), self._ws.data_ptr(),
            self._ws.numel() * 8, self.status.data_ptr(), _stream()),
            "vec_batch_loglik_grad_info")
        if check:
            self.check_status("vec_batch_loglik_grad_info")
        return self.out

    def fisher_fit(self, covparms: torch.Tensor, iters: int, use_graph: bool = True,
                   max_step: float = 1.0, check: bool = True):
        if not (isinstance(covparms, torch.Tensor) and covparms.is_cuda):
            raise TypeError("covparms must be a device tensor (updated in place)")
        covparms = self.covparms(covparms)
        _check(_batch_lib().vec_batch_fisher_fit(
            *self._args(covparms), int(iters), float(max_step), self.raw.data_ptr(),
            self.out.data_ptr(), self._ws.data_ptr(), self._ws.numel() * 8,
            self.status.data_ptr(), int(bool(use_graph)), _stream()), "vec_batch_fisher_fit")
        if check:
            self.check_status("vec_batch_fisher_fit")
        return covparms
