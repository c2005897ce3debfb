"""Thin ctypes binding of the hcov C ABI (include/hcov.h).

Argument marshalling only: every step of the likelihood runs in the HIP
library ``libhcov.so``.  Loading fails loudly when the library is missing;
there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhcov.so")

OK, EINVAL, ENOTSPD, ENOMEM, ESTATE, EDEVICE, ERANK = 0, -1, -2, -3, -4, -5, -6
HOST, DEVICE = 0, 1
FP64, MIXED = 0, 1
SAT_RETRY, SAT_ERROR = 0, 1
QUAD_DIRECT, QUAD_PCG = 0, 1
ADM_MIN, ADM_MAX, ADM_WEAK = 0, 1, 2


class Theta(C.Structure):
    _fields_ = [("sigma2", C.c_double), ("ell", C.c_double), ("nu", C.c_double), ("nugget", C.c_double)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
OBJ_FN = C.CFUNCTYPE(C.c_double, C.POINTER(C.c_double), C.c_int, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Request(C.Structure):
    _fields_ = [("locs", C.c_void_p), ("n", C.c_int64), ("z", C.c_void_p), ("theta", Theta), ("eps", C.c_double),
                ("leaf", C.c_int), ("eta", C.c_double), ("dataset", C.c_int)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int), ("loglik", C.c_double), ("logdet", C.c_double), ("quad", C.c_double),
                ("queue_ms", C.c_double), ("service_ms", C.c_double), ("latency_ms", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("max_rank", C.c_int), ("aca_eps_factor", C.c_double),
                ("fuse_solve", C.c_int), ("mem_cap_bytes", C.c_size_t), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_user", C.c_void_p), ("use_graphs", C.c_int),
                ("oversample", C.c_int), ("on_saturation", C.c_int), ("keep_matrix", C.c_int),
                ("quad_mode", C.c_int), ("pcg_tol", C.c_double), ("pcg_max_iter", C.c_int), ("fixed_rank", C.c_int),
                ("adm_rule", C.c_int), ("autotune", C.c_int), ("seed", C.c_uint64),
                ("initial_rank_cap", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("leaf", C.c_int), ("depth", C.c_int), ("n_dense_blocks", C.c_int64),
                ("n_lr_blocks", C.c_int64), ("dense_entries", C.c_int64), ("lr_rows", C.c_int64),
                ("max_rank_seen", C.c_int), ("mean_rank", C.c_double), ("bytes_device", C.c_int64),
                ("bytes_factor", C.c_int64), ("ms_tree", C.c_double), ("ms_assemble", C.c_double),
                ("ms_factor", C.c_double), ("ms_solve", C.c_double), ("n_steps", C.c_int64),
                ("n_launches_factor", C.c_int64), ("n_graph_replays", C.c_int64),
                ("n_sketch_retries", C.c_int64), ("sketch_saturated", C.c_int), ("mean_sketch_width", C.c_double),
                ("pcg_iters", C.c_int), ("pcg_relres", C.c_double), ("n_gemm_grouped", C.c_int64),
                ("n_autotune_switched", C.c_int64), ("gemm_flops_factor", C.c_double),
                ("gemm_bytes_factor", C.c_double), ("n_replans", C.c_int64), ("bytes_lowrank", C.c_int64)]


_lib = None


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"hcov HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.hcov_opts_default.argtypes = [C.POINTER(Opts)]
        L.hcov_build.argtypes = [dp, C.c_int64, Theta, C.c_double, C.c_int, C.c_double, C.POINTER(Opts),
                                 C.c_void_p, C.POINTER(C.c_void_p)]
        L.hcov_set_theta.argtypes = [C.c_void_p, Theta]
        L.hcov_cholesky.argtypes = [C.c_void_p]
        L.hcov_logdet.argtypes = [C.c_void_p, dp]
        L.hcov_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.hcov_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, dp, C.c_int]
        L.hcov_sample.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.hcov_matvec.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.hcov_factor_matvec.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.hcov_error_norms.argtypes = [C.c_void_p, C.c_int, C.c_uint64, dp, dp, dp]
        L.hcov_exact_matvec.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.hcov_exact_norms.argtypes = [C.c_void_p, C.c_int, C.c_uint64, dp, dp]
        L.hcov_loglik.argtypes = [C.c_void_p, C.c_void_p, C.c_int, dp, dp, dp]
        L.hcov_stats.argtypes = [C.c_void_p, C.POINTER(Stats)]
        L.hcov_estimate_bytes.argtypes = [dp, C.c_int64, C.c_double, C.c_int, C.c_double, C.POINTER(Opts),
                                          C.POINTER(C.c_size_t)]
        L.hcov_perm.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.hcov_destroy.argtypes = [C.c_void_p]
        L.hcov_destroy.restype = None
        L.hcov_strerror.argtypes = [C.c_int]
        L.hcov_strerror.restype = C.c_char_p
        L.hcov_last_error.argtypes = [C.c_void_p]
        L.hcov_last_error.restype = C.c_char_p
        L.hcov_tree_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int64)]
        L.hcov_tree_dump.argtypes = [C.c_void_p, dp, C.POINTER(C.c_int64)]
        L.hcov_matern_eval.argtypes = [Theta, dp, dp, C.c_int64]
        L.hcov_nm_minimize.argtypes = [OBJ_FN, C.c_void_p, dp, dp, C.c_int, C.c_int, C.c_double, dp, dp,
                                       C.POINTER(C.c_int), dp, dp]
        L.hcov_fit.argtypes = [C.c_void_p, C.c_void_p, C.c_int, dp, dp, C.c_double, C.c_int, C.c_double, dp, dp,
                               C.POINTER(C.c_int), dp, dp]
        L.hcov_server_create.argtypes = [C.c_int, C.c_size_t, C.POINTER(Opts), C.POINTER(C.c_void_p)]
        L.hcov_server_dataset.argtypes = [C.c_void_p, dp, C.c_int64, Theta, C.c_double, C.c_int, C.c_double,
                                          C.POINTER(C.c_int)]
        L.hcov_server_release.argtypes = [C.c_void_p, C.c_int]
        L.hcov_server_submit.argtypes = [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]
        L.hcov_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Result)]
        L.hcov_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(Result)]
        L.hcov_server_destroy.argtypes = [C.c_void_p]
        L.hcov_server_destroy.restype = None
        L.hcov_profile_begin.argtypes = [C.c_void_p, C.c_int]
        L.hcov_profile_end.argtypes = [C.c_void_p, C.POINTER(C.c_int64), dp, dp, dp]
        L.hcov_profile_times.argtypes = [C.c_void_p, dp, C.c_int64, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


EXPORTS = ["hcov_opts_default", "hcov_build", "hcov_set_theta", "hcov_cholesky", "hcov_logdet", "hcov_solve",
           "hcov_forward", "hcov_sample", "hcov_matvec", "hcov_loglik", "hcov_stats", "hcov_estimate_bytes",
           "hcov_perm", "hcov_destroy", "hcov_strerror", "hcov_last_error", "hcov_tree_sizes", "hcov_tree_dump",
           "hcov_matern_eval", "hcov_profile_begin", "hcov_profile_end", "hcov_nm_minimize", "hcov_fit",
           "hcov_server_create", "hcov_server_dataset", "hcov_server_release", "hcov_server_submit",
           "hcov_server_poll", "hcov_server_wait", "hcov_server_destroy"]

EAGAIN = -7

STAGE_KINDS = {"gemm": 0, "tsqr_seg": 1, "tsqr_red": 2, "small": 3, "leaf": 4, "trsm": 5, "trmm": 9}


class HcovError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hcov error {code}: {msg}")
        self.code = code


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _theta(t):
    if isinstance(t, Theta):
        return t
    if isinstance(t, dict):
        return Theta(t["sigma2"], t["ell"], t["nu"], t.get("nugget", 0.0))
    s2, ell, nu, nug = t
    return Theta(float(s2), float(ell), float(nu), float(nug))


def default_opts(**kw):
    o = Opts()
    lib().hcov_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def torch_allocator():
    """(alloc, free) callbacks backed by the PyTorch caching allocator on the
    current device, for Opts.alloc / Opts.free."""
    import torch

    def _alloc(nbytes, user):
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    def _free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    return ALLOC_FN(_alloc), FREE_FN(_free)


def matern_eval(theta, h):
    """Eq. (3) evaluated by the device Matérn/K_nu code for distances h."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.empty_like(h)
    rc = lib().hcov_matern_eval(_theta(theta), _dp(h), _dp(out), h.size)
    if rc:
        raise HcovError(rc, lib().hcov_strerror(rc).decode())
    return out


def nm_minimize(f, x0, steps, max_evals=200, size_tol=1e-5):
    """Library Nelder-Mead on a Python objective f(x) -> float.  Returns
    (x, f(x), n_evals, history list of (x, f))."""
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    st = np.ascontiguousarray(steps, dtype=np.float64)
    d = x0.size
    cb = OBJ_FN(lambda xp, dim, user: float(f(np.array([xp[i] for i in range(dim)]))))
    ox = np.empty(d)
    of = C.c_double()
    ne = C.c_int()
    hx = np.empty(max_evals * d)
    hf = np.empty(max_evals)
    rc = lib().hcov_nm_minimize(cb, None, _dp(x0), _dp(st), d, int(max_evals), float(size_tol), _dp(ox),
                                C.byref(of), C.byref(ne), _dp(hx), _dp(hf))
    if rc:
        raise HcovError(rc, lib().hcov_strerror(rc).decode())
    n = ne.value
    hist = [(hx[i * d:(i + 1) * d].copy(), hf[i]) for i in range(n)]
    return ox, of.value, n, hist


def estimate_bytes(locs, eps, leaf, eta, opts=None):
    locs = np.ascontiguousarray(locs, dtype=np.float64)
    out = C.c_size_t(0)
    rc = lib().hcov_estimate_bytes(_dp(locs), locs.shape[0], eps, leaf, eta,
                                   C.byref(opts) if opts is not None else None, C.byref(out))
    if rc:
        raise HcovError(rc, lib().hcov_strerror(rc).decode())
    return int(out.value)


class HCov:
    """One H-matrix context: trees, plan, assembled matrix and factor."""

    def __init__(self, locs, theta, eps=1e-8, leaf=64, eta=2.0, opts=None, stream=None, torch_alloc=False):
        L = lib()
        self._ctx = C.c_void_p(None)
        locs = np.ascontiguousarray(locs, dtype=np.float64)
        if locs.ndim != 2 or locs.shape[1] != 2:
            raise ValueError("locs must be n x 2")
        self.n = locs.shape[0]
        if opts is None:
            opts = default_opts()
        elif isinstance(opts, dict):
            opts = default_opts(**opts)
        self._cb = None
        if torch_alloc:
            self._cb = torch_allocator()
            opts.alloc, opts.free = self._cb
        self.opts = opts
        st = C.c_void_p(stream) if stream is not None else None
        rc = L.hcov_build(_dp(locs), self.n, _theta(theta), float(eps), int(leaf), float(eta), C.byref(opts), st,
                          C.byref(self._ctx))
        if rc:
            raise HcovError(rc, L.hcov_strerror(rc).decode())

    def _chk(self, rc):
        if rc:
            msg = lib().hcov_last_error(self._ctx).decode() if self._ctx else ""
            raise HcovError(rc, f"{lib().hcov_strerror(rc).decode()}: {msg}")

    def close(self):
        if self._ctx:
            lib().hcov_destroy(self._ctx)
            self._ctx = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_theta(self, theta):
        self._chk(lib().hcov_set_theta(self._ctx, _theta(theta)))

    def cholesky(self):
        self._chk(lib().hcov_cholesky(self._ctx))

    def logdet(self):
        out = C.c_double(0)
        self._chk(lib().hcov_logdet(self._ctx, C.byref(out)))
        return out.value

    def _vec(self, v):
        """(pointer, where, keepalive) for a numpy array or a torch tensor."""
        try:
            import torch
            if isinstance(v, torch.Tensor):
                if v.dtype != torch.float64 or not v.is_contiguous() or v.numel() != self.n:
                    raise ValueError("expected a contiguous float64 tensor of n elements")
                return C.c_void_p(v.data_ptr()), (DEVICE if v.is_cuda else HOST), v
        except ImportError:
            pass
        a = np.ascontiguousarray(v, dtype=np.float64)
        if a.size != self.n:
            raise ValueError("vector length must be n")
        return C.c_void_p(a.ctypes.data), HOST, a

    def loglik(self, z):
        """(L, log|C~|, z^T C~^{-1} z) with L of Eq. (2) (paper's sign)."""
        p, w, keep = self._vec(z)
        ll, ld, q = C.c_double(), C.c_double(), C.c_double()
        self._chk(lib().hcov_loglik(self._ctx, p, w, C.byref(ll), C.byref(ld), C.byref(q)))
        return ll.value, ld.value, q.value

    def solve(self, z):
        p, w, keep = self._vec(z)
        if w == HOST:
            x = np.empty(self.n)
            self._chk(lib().hcov_solve(self._ctx, p, C.c_void_p(x.ctypes.data), HOST))
            return x
        import torch
        x = torch.empty_like(keep)
        self._chk(lib().hcov_solve(self._ctx, p, C.c_void_p(x.data_ptr()), DEVICE))
        return x

    def forward(self, z):
        p, w, keep = self._vec(z)
        q = C.c_double()
        v = np.empty(self.n)
        if w != HOST:
            raise ValueError("forward() returns host arrays; pass host input")
        self._chk(lib().hcov_forward(self._ctx, p, C.c_void_p(v.ctypes.data), C.byref(q), HOST))
        return v, q.value

    def sample(self, xi_cluster):
        xi = np.ascontiguousarray(xi_cluster, dtype=np.float64)
        y = np.empty(self.n)
        self._chk(lib().hcov_sample(self._ctx, C.c_void_p(xi.ctypes.data), C.c_void_p(y.ctypes.data), HOST))
        return y

    def matvec(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        self._chk(lib().hcov_matvec(self._ctx, C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data), HOST))
        return y

    def factor_matvec(self, x):
        """L~ L~^T x (needs opts keep_matrix)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        self._chk(lib().hcov_factor_matvec(self._ctx, C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data), HOST))
        return y

    def error_norms(self, iters=30, seed=1):
        """(||C~||_2, ||C~ - L~L~^T||_2, ||I - (L~L~^T)^{-1} C~||_2) by power iteration."""
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self._chk(lib().hcov_error_norms(self._ctx, int(iters), C.c_uint64(seed), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def exact_matvec(self, x):
        """C x with the exact Matérn entries (device, on the fly)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty(self.n)
        self._chk(lib().hcov_exact_matvec(self._ctx, C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data), HOST))
        return y

    def exact_norms(self, iters=30, seed=1):
        """(||C - C~||_2, ||C (L~L~^T)^{-1} - I||_2) by power iteration."""
        a, b = C.c_double(), C.c_double()
        self._chk(lib().hcov_exact_norms(self._ctx, int(iters), C.c_uint64(seed), C.byref(a), C.byref(b)))
        return a.value, b.value

    def stats(self):
        s = Stats()
        self._chk(lib().hcov_stats(self._ctx, C.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def fit(self, z, theta0, nugget, max_evals=30, size_tol=1e-5, steps=None):
        """Maximum-likelihood theta = (sigma2, ell, nu) by the library's
        Nelder-Mead on the H-likelihood.  Returns (theta, loglik, n_evals,
        history of (theta, -loglik))."""
        p, w, keep = self._vec(z)
        t0 = np.ascontiguousarray(theta0, dtype=np.float64)
        st = None if steps is None else np.ascontiguousarray(steps, dtype=np.float64)
        out = np.empty(3)
        ll = C.c_double()
        ne = C.c_int()
        ht = np.empty(max_evals * 3)
        hf = np.empty(max_evals)
        self._chk(lib().hcov_fit(self._ctx, p, w, _dp(t0), _dp(st) if st is not None else None, float(nugget),
                                 int(max_evals), float(size_tol), _dp(out), C.byref(ll), C.byref(ne), _dp(ht),
                                 _dp(hf)))
        n = ne.value
        return out, ll.value, n, [(ht[3 * i:3 * i + 3].copy(), hf[i]) for i in range(n)]

    def profile_begin(self, kind):
        self._chk(lib().hcov_profile_begin(self._ctx, STAGE_KINDS[kind] if isinstance(kind, str) else int(kind)))

    def profile_end(self):
        """(launches, summed kernel ms, algorithmic flops, algorithmic bytes)."""
        n = C.c_int64()
        ms = C.c_double()
        fl = C.c_double()
        by = C.c_double()
        self._chk(lib().hcov_profile_end(self._ctx, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)))
        return n.value, ms.value, fl.value, by.value

    def profile_times(self):
        """Per-launch durations (ms) of the last profiling session."""
        n = C.c_int64()
        self._chk(lib().hcov_profile_times(self._ctx, None, 0, C.byref(n)))
        t = np.empty(n.value)
        self._chk(lib().hcov_profile_times(self._ctx, _dp(t), n.value, C.byref(n)))
        return t

    def perm(self):
        p = np.empty(self.n, dtype=np.int64)
        self._chk(lib().hcov_perm(self._ctx, p.ctypes.data_as(C.POINTER(C.c_int64))))
        return p

    def tree(self):
        d = C.c_int()
        nb = C.c_int64()
        self._chk(lib().hcov_tree_sizes(self._ctx, C.byref(d), C.byref(nb)))
        bbox = np.empty(((2 << d.value) - 1) * 4)
        blocks = np.empty(nb.value * 4, dtype=np.int64)
        self._chk(lib().hcov_tree_dump(self._ctx, _dp(bbox), blocks.ctypes.data_as(C.POINTER(C.c_int64))))
        return d.value, bbox.reshape(-1, 4), blocks.reshape(-1, 4)


class Server:
    """Request loop of the library (worker threads with one HIP stream each,
    admission by device-memory estimate, resident data sets)."""

    def __init__(self, slots=4, mem_budget=0, opts=None):
        o = default_opts(**(opts or {}))
        h = C.c_void_p()
        rc = lib().hcov_server_create(int(slots), C.c_size_t(int(mem_budget)), C.byref(o), C.byref(h))
        if rc:
            raise HcovError(rc, lib().hcov_strerror(rc).decode())
        self._h = h

    def _chk(self, rc):
        if rc:
            raise HcovError(rc, lib().hcov_strerror(rc).decode())

    def dataset(self, locs, theta, eps=1e-8, leaf=64, eta=2.0):
        """Registers resident locations; returns the data-set id."""
        locs = np.ascontiguousarray(locs, dtype=np.float64)
        i = C.c_int()
        self._chk(lib().hcov_server_dataset(self._h, _dp(locs), locs.shape[0], _theta(theta), float(eps), int(leaf),
                                            float(eta), C.byref(i)))
        return i.value

    def release(self, ds):
        self._chk(lib().hcov_server_release(self._h, int(ds)))

    def submit(self, z, theta, locs=None, eps=1e-8, leaf=64, eta=2.0, dataset=0):
        """Queues one evaluation; returns its ticket."""
        z = np.ascontiguousarray(z, dtype=np.float64)
        r = Request()
        keep = [z]
        if locs is not None:
            locs = np.ascontiguousarray(locs, dtype=np.float64)
            keep.append(locs)
            r.locs = locs.ctypes.data
        r.n = z.shape[0]
        r.z = z.ctypes.data
        r.theta = _theta(theta)
        r.eps, r.leaf, r.eta, r.dataset = float(eps), int(leaf), float(eta), int(dataset)
        t = C.c_uint64()
        self._chk(lib().hcov_server_submit(self._h, C.byref(r), C.byref(t)))
        return t.value

    @staticmethod
    def _res(r):
        return {f: getattr(r, f) for f, _ in Result._fields_}

    def poll(self, ticket):
        """Result dict when done, None while pending."""
        r = Result()
        rc = lib().hcov_server_poll(self._h, C.c_uint64(ticket), C.byref(r))
        if rc == EAGAIN:
            return None
        self._chk(rc)
        return self._res(r)

    def wait(self, ticket):
        r = Result()
        self._chk(lib().hcov_server_wait(self._h, C.c_uint64(ticket), C.byref(r)))
        return self._res(r)

    def close(self):
        if getattr(self, "_h", None):
            lib().hcov_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
