"""Python binding of the DPMM HIP library (argument marshalling only).

`Sampler` wraps one dpmm_ctx.  Data and labels are torch tensors in device
memory; parameters and statistics cross as float64 / int64 numpy arrays in
the layouts include/dpmm.h documents.  Every computation runs in the HIP
kernels of libdpmm.so; nothing here computes any part of the sampler.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import DpmmError


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class SparseCounts:
    """Count rows in compressed sparse rows on the device: row_ptr int64
    [n + 1], col int32 [nnz] (words in [0, V)), val int32 [nnz] (counts).
    The data argument of a Sampler created with sparse=True."""

    def __init__(self, row_ptr, col, val, V):
        import torch
        self.row_ptr = row_ptr.to(device="cuda", dtype=torch.int64).contiguous()
        self.col = col.to(device="cuda", dtype=torch.int32).contiguous()
        self.val = val.to(device="cuda", dtype=torch.int32).contiguous()
        self.shape = (self.row_ptr.shape[0] - 1, int(V))
        self.device = self.row_ptr.device
        self._desc = _lib.CSR(self.row_ptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr(),
                              self.col.shape[0])

    @classmethod
    def from_numpy(cls, indptr, indices, data, V):
        import torch
        return cls(torch.from_numpy(np.ascontiguousarray(indptr, dtype=np.int64)),
                   torch.from_numpy(np.ascontiguousarray(indices, dtype=np.int32)),
                   torch.from_numpy(np.ascontiguousarray(data, dtype=np.int32)), V)

    def ptr(self):
        return ctypes.cast(ctypes.pointer(self._desc), ctypes.c_void_p)


def _xptr(x):
    """The data argument: a device tensor's address or a dpmm_csr descriptor."""
    return x.ptr() if isinstance(x, SparseCounts) else _tptr(x)


class Sampler:
    """One sampler context on the current HIP device and torch stream."""

    def __init__(self, family, d, k_max, alpha, seed, kappa=1.0, nu=None, m=None, psi=None,
                 beta=None, burn_out=15, merge_form="paper", precision="fp32", learned=0, stream=None,
                 gamma_shape=None, gamma_rate=None, sparse=False):
        import torch
        self.torch = torch
        L = _lib.lib()
        self.family = family
        self.d = int(d)
        cfg = _lib.Config()
        cfg.family = {"gaussian": _lib.GAUSSIAN, "multinomial": _lib.MULTINOMIAL, "poisson": _lib.POISSON}[family]
        cfg.d = self.d
        cfg.k_max = int(k_max)
        cfg.burn_out = int(burn_out)
        cfg.alpha = float(alpha)
        cfg.kappa = float(kappa)
        cfg.nu = float(nu if nu is not None else self.d + 3)
        self._keep = []
        if family == "gaussian":
            m = np.ascontiguousarray(np.zeros(self.d) if m is None else m, dtype=np.float64)
            psi = np.ascontiguousarray(np.eye(self.d) if psi is None else psi, dtype=np.float64)
            self._keep += [m, psi]
            cfg.m, cfg.psi = _dptr(m), _dptr(psi)
        elif family == "poisson":
            a = np.ascontiguousarray(np.ones(self.d) if gamma_shape is None else gamma_shape, dtype=np.float64)
            b = np.ascontiguousarray(np.ones(self.d) if gamma_rate is None else gamma_rate, dtype=np.float64)
            self._keep += [a, b]
            cfg.gamma_shape, cfg.gamma_rate = _dptr(a), _dptr(b)
        else:
            beta = np.ascontiguousarray(np.ones(self.d) if beta is None else beta, dtype=np.float64)
            self._keep.append(beta)
            cfg.beta = _dptr(beta)
        cfg.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        cfg.precision = {"fp32": _lib.FP32, "bf16": _lib.BF16, "bf16x3": _lib.BF16X3}[precision]
        cfg.merge_form = {"paper": _lib.MERGE_PAPER, "inverse_split": _lib.MERGE_INVERSE_SPLIT}[merge_form]
        cfg.learned = int(learned)
        cfg.sparse = 1 if sparse else 0
        self.learned = int(learned)
        self._L = L
        self._ctx = ctypes.c_void_p()
        st = stream if stream is not None else _stream(torch)
        s = L.dpmm_create(ctypes.byref(cfg), st, ctypes.byref(self._ctx))
        if s != _lib.DPMM_OK:
            raise DpmmError(s, L.dpmm_last_error(None).decode())
        self.k_max = int(k_max)

    # ------------------------------------------------------------------ utils
    def _check(self, s):
        if s != _lib.DPMM_OK:
            raise DpmmError(s, self._L.dpmm_last_error(self._ctx).decode())

    def close(self):
        if self._ctx:
            self._L.dpmm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _param_width(self):
        return self.d + self.d * self.d if self.family == "gaussian" else self.d

    def _stat_width(self):
        return 1 + self.d + self.d * self.d if self.family == "gaussian" else 1 + self.d

    @staticmethod
    def _check_rows(x, n):
        if x.shape[0] != n:
            raise ValueError("row count mismatch")

    # ------------------------------------------------------------------ state
    @property
    def K(self):
        k = ctypes.c_int32()
        self._check(self._L.dpmm_get_state(self._ctx, ctypes.byref(k), None))
        return int(k.value)

    def ages(self):
        K = self.K
        a = np.zeros(K, dtype=np.int32)
        k = ctypes.c_int32()
        self._check(self._L.dpmm_get_state(self._ctx, ctypes.byref(k), a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return a

    def set_state(self, K, ages=None):
        a = None
        if ages is not None:
            a = np.ascontiguousarray(ages, dtype=np.int32)
        self._check(self._L.dpmm_set_state(self._ctx, int(K), None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))

    def init_labels(self, n):
        z = self.torch.empty(n, dtype=self.torch.int32, device="cuda")
        zs = self.torch.empty(n, dtype=self.torch.uint8, device="cuda")
        self._check(self._L.dpmm_init_labels(self._ctx, int(n), _tptr(z), _tptr(zs)))
        return z, zs

    def set_params(self, log_pi, log_pisub, comp):
        log_pi = np.ascontiguousarray(log_pi, dtype=np.float64)
        K = log_pi.shape[0]
        log_pisub = np.ascontiguousarray(log_pisub, dtype=np.float64).reshape(K, 2)
        comp = np.ascontiguousarray(comp, dtype=np.float64).reshape(K, 3, self._param_width())
        self._check(self._L.dpmm_set_params(self._ctx, K, _dptr(log_pi), _dptr(log_pisub), _dptr(comp)))

    def get_params(self):
        K = self.K
        lp = np.zeros(K)
        lps = np.zeros((K, 2))
        comp = np.zeros((K, 3, self._param_width()))
        self._check(self._L.dpmm_get_params(self._ctx, _dptr(lp), _dptr(lps), _dptr(comp)))
        return lp, lps, comp

    def set_stats(self, stats):
        K = stats.shape[0]
        if self.family == "gaussian":
            a = np.ascontiguousarray(stats, dtype=np.float64).reshape(K, 2, self._stat_width())
        else:
            a = np.ascontiguousarray(stats, dtype=np.int64).reshape(K, 2, self._stat_width())
        self._check(self._L.dpmm_set_stats(self._ctx, K, ctypes.c_void_p(a.ctypes.data)))

    def get_stats(self):
        K = self.K
        dt = np.float64 if self.family == "gaussian" else np.int64
        a = np.zeros((K, 2, self._stat_width()), dtype=dt)
        self._check(self._L.dpmm_get_stats(self._ctx, ctypes.c_void_p(a.ctypes.data)))
        return a

    # ------------------------------------------------------------------ hot path
    def loglik(self, x):
        n = x.shape[0]
        out = self.torch.empty((n, 3 * self.K), dtype=self.torch.float32, device=x.device)
        self._check(self._L.dpmm_loglik(self._ctx, _xptr(x), n, _tptr(out)))
        return out

    def sample_labels(self, x, t, z=None, zsub=None):
        n = x.shape[0]
        if z is None:
            z = self.torch.empty(n, dtype=self.torch.int32, device=x.device)
        if zsub is None:
            zsub = self.torch.empty(n, dtype=self.torch.uint8, device=x.device)
        self._check(self._L.dpmm_sample_labels(self._ctx, _xptr(x), n, int(t), _tptr(z), _tptr(zsub)))
        return z, zsub

    def suffstats(self, x, z, zsub):
        self._check(self._L.dpmm_suffstats(self._ctx, _xptr(x), x.shape[0], _tptr(z), _tptr(zsub)))

    def sample_params(self, t):
        self._check(self._L.dpmm_sample_params(self._ctx, int(t)))

    def split_merge(self, x, t, z, zsub):
        info = _lib.IterInfo()
        self._check(self._L.dpmm_split_merge(self._ctx, _xptr(x), x.shape[0], int(t), _tptr(z), _tptr(zsub),
                                             ctypes.byref(info)))
        return info.as_dict()

    def step(self, x, t, z, zsub):
        info = _lib.IterInfo()
        self._check(self._L.dpmm_step(self._ctx, _xptr(x), x.shape[0], int(t), _tptr(z), _tptr(zsub),
                                      ctypes.byref(info)))
        return info.as_dict()

    def fit(self, x, t0, iters, z, zsub, train_every=0, train_until=0, train_steps=20, train_batch=4096,
            train_lr=1e-3):
        """Iterations t0 ... t0 + iters - 1 (dpmm_fit): per-iteration info
        dicts and wall-clock seconds."""
        opt = _lib.FitOptions(int(t0), int(iters), int(train_every), int(train_until), int(train_steps),
                              int(train_batch), float(train_lr), 0)
        trace = (_lib.IterInfo * max(int(iters), 1))()
        secs = np.zeros(max(int(iters), 1))
        self._check(self._L.dpmm_fit(self._ctx, _xptr(x), x.shape[0], ctypes.byref(opt), _tptr(z), _tptr(zsub),
                                     trace, _dptr(secs)))
        return [trace[j].as_dict() for j in range(int(iters))], secs[:int(iters)]

    def save_checkpoint(self, path, t, z, zsub):
        self._check(self._L.dpmm_save_checkpoint(self._ctx, str(path).encode(), z.shape[0], int(t), _tptr(z),
                                                 _tptr(zsub)))

    def load_checkpoint(self, path, z, zsub):
        """Labels into z / zsub, K and ages into the context; returns the
        checkpoint's iteration t."""
        t = ctypes.c_uint32()
        self._check(self._L.dpmm_load_checkpoint(self._ctx, str(path).encode(), z.shape[0], ctypes.byref(t),
                                                 _tptr(z), _tptr(zsub)))
        return int(t.value)

    # ------------------------------------------------------------------ learned proposal
    @property
    def n_mlp_params(self):
        return int(self._L.dpmm_mlp_n_params(self._ctx))

    def mlp_set_weights(self, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        if p.shape != (self.n_mlp_params,):
            raise ValueError("parameter vector length mismatch")
        self._check(self._L.dpmm_mlp_set_weights(self._ctx, _dptr(p)))

    def mlp_get_weights(self):
        p = np.zeros(self.n_mlp_params)
        self._check(self._L.dpmm_mlp_get_weights(self._ctx, _dptr(p)))
        return p

    def mlp_forward(self, X):
        out = self.torch.empty(X.shape[0], dtype=self.torch.float32, device=X.device)
        self._check(self._L.dpmm_mlp_forward(self._ctx, _tptr(X), X.shape[0], _tptr(out)))
        return out

    def mlp_grad(self, X, y):
        g = np.zeros(self.n_mlp_params)
        loss = ctypes.c_double()
        self._check(self._L.dpmm_mlp_grad(self._ctx, _tptr(X), _tptr(y), X.shape[0], _dptr(g), ctypes.byref(loss)))
        return g, loss.value

    def mlp_adam_step(self, X, y, lr):
        loss = ctypes.c_double()
        self._check(self._L.dpmm_mlp_adam_step(self._ctx, _tptr(X), _tptr(y), X.shape[0], float(lr),
                                               ctypes.byref(loss)))
        return loss.value

    def set_features(self, x, z, k1, k2=-1):
        """(features float32 [n_set][F], point indices int32 [n_set]) of the set."""
        n_set = ctypes.c_int64()
        self._check(self._L.dpmm_set_features(self._ctx, _tptr(x), x.shape[0], _tptr(z), int(k1), int(k2), None,
                                              None, 0, ctypes.byref(n_set)))
        F = 2 * self.learned
        feats = self.torch.empty((n_set.value, F), dtype=self.torch.float32, device=x.device)
        idx = self.torch.empty(n_set.value, dtype=self.torch.int32, device=x.device)
        self._check(self._L.dpmm_set_features(self._ctx, _tptr(x), x.shape[0], _tptr(z), int(k1), int(k2),
                                              _tptr(feats), _tptr(idx), n_set.value, ctypes.byref(n_set)))
        return feats, idx

    def learned_move(self, x, t, z, zsub, side=None):
        info = _lib.LearnedInfo()
        self._check(self._L.dpmm_learned_move(self._ctx, _tptr(x), x.shape[0], int(t), _tptr(z), _tptr(zsub),
                                              _tptr(side), ctypes.byref(info)))
        return info.as_dict()

    def mlp_train(self, x, z, zsub, steps, batch, lr):
        loss = ctypes.c_double()
        self._check(self._L.dpmm_mlp_train(self._ctx, _tptr(x), x.shape[0], _tptr(z), _tptr(zsub), int(steps),
                                           int(batch), float(lr), ctypes.byref(loss)))
        return loss.value

    def mlp_training_set(self, x, z, zsub):
        """(features float32 [rows][F], targets float32 [rows], point indices
        int32 [rows]) of the rows mlp_train draws its batches from."""
        n_rows = ctypes.c_int64()
        self._check(self._L.dpmm_mlp_training_set(self._ctx, _tptr(x), x.shape[0], _tptr(z), _tptr(zsub), None, None,
                                                  None, 0, ctypes.byref(n_rows)))
        r = n_rows.value
        F = 2 * self.learned
        feats = self.torch.empty((r, F), dtype=self.torch.float32, device=x.device)
        y = self.torch.empty(r, dtype=self.torch.float32, device=x.device)
        idx = self.torch.empty(r, dtype=self.torch.int32, device=x.device)
        if r:
            self._check(self._L.dpmm_mlp_training_set(self._ctx, _tptr(x), x.shape[0], _tptr(z), _tptr(zsub),
                                                      _tptr(feats), _tptr(y), _tptr(idx), r, ctypes.byref(n_rows)))
        return feats, y, idx
