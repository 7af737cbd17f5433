"""ctypes binding of libvsr.so (C ABI in include/vsr.h): argument marshalling only.

Vectors are torch float64 tensors on the GPU (contiguous); their device pointers
are handed to the library, which does all of the computation.  The library is
loaded from this package's directory; importing fails loudly if it is missing.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvsr.so")

VSR_OK, VSR_EINVAL, VSR_EMESH, VSR_ENOTSPD, VSR_ENOCONV, VSR_EDEVICE, VSR_ENOMEM = range(7)
STATUS_NAMES = {0: "VSR_OK", 1: "VSR_EINVAL", 2: "VSR_EMESH", 3: "VSR_ENOTSPD", 4: "VSR_ENOCONV",
                5: "VSR_EDEVICE", 6: "VSR_ENOMEM"}


class VsrError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("vertices", ctypes.POINTER(ctypes.c_double))]


class Coefficients(ctypes.Structure):
    _fields_ = [("kappa", ctypes.POINTER(ctypes.c_double)), ("mu_override", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("relax_fp32", ctypes.c_int32), ("cycle", ctypes.c_int32), ("quad_points", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("max_iterations", ctypes.c_int32),
                ("interior_patches_only", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("omega", ctypes.c_double), ("stream", ctypes.c_void_p), ("autotune", ctypes.c_int32),
                ("batch_streams", ctypes.c_int32), ("batch_eager", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
                ("share_factors", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("coarse_solver", ctypes.c_int32), ("stagnation_window", ctypes.c_int32),
                ("stagnation_factor", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("true_rel_residual", ctypes.c_double),
                ("omega", ctypes.c_double), ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("solve_seconds", ctypes.c_double),
                ("ritz_min", ctypes.c_double), ("ritz_max", ctypes.c_double), ("kappa_estimate", ctypes.c_double),
                ("fp64_iterations", ctypes.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    """Load libvsr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with python -m paper_2107_14758_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    dp = ctypes.c_void_p
    L.vsr_default_options.argtypes = [ctypes.POINTER(Options)]
    L.vsr_default_options.restype = None
    L.vsr_setup.argtypes = [ctypes.POINTER(Mesh), ctypes.c_int32, ctypes.POINTER(Coefficients),
                            ctypes.POINTER(Options), ctypes.POINTER(P)]
    L.vsr_num_dofs.argtypes = [P]
    L.vsr_num_dofs.restype = ctypes.c_int64
    L.vsr_load_vector.argtypes = [P, dp, dp]
    L.vsr_apply_operator.argtypes = [P, dp, dp]
    L.vsr_apply_operator_noalloc.argtypes = [P, dp, dp]
    L.vsr_apply_relaxation.argtypes = [P, dp, dp, ctypes.c_int32]
    L.vsr_pcg_solve.argtypes = [P, dp, dp, ctypes.c_double, ctypes.POINTER(SolveInfo)]
    L.vsr_get_damping.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
    L.vsr_set_profiling.argtypes = [P, ctypes.c_int32]
    L.vsr_kernel_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    L.vsr_factor_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    L.vsr_destroy.argtypes = [P]
    L.vsr_destroy.restype = None
    L.vsr_get_tuning.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    L.vsr_set_tuning.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    L.vsr_setup_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(Mesh), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(Coefficients), ctypes.POINTER(Options), ctypes.POINTER(P)]
    L.vsr_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(Options),
                                   ctypes.POINTER(P)]
    L.vsr_batch_size.argtypes = [P]
    L.vsr_batch_size.restype = ctypes.c_int32
    L.vsr_batch_member.argtypes = [P, ctypes.c_int32]
    L.vsr_batch_member.restype = P
    L.vsr_pcg_solve_batch.argtypes = [P, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                      ctypes.c_double, ctypes.POINTER(SolveInfo)]
    L.vsr_destroy_batch.argtypes = [P]
    L.vsr_destroy_batch.restype = None
    L.vsr_last_error.argtypes = []
    L.vsr_last_error.restype = ctypes.c_char_p
    L.vsr_elasticity_setup.argtypes = [ctypes.POINTER(Mesh), ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(Options), ctypes.POINTER(P)]
    L.vsr_elasticity_num_dofs.argtypes = [P]
    L.vsr_elasticity_num_dofs.restype = ctypes.c_int64
    L.vsr_elasticity_load_vector.argtypes = [P, dp, dp]
    L.vsr_elasticity_apply_operator.argtypes = [P, dp, dp]
    L.vsr_elasticity_apply_relaxation.argtypes = [P, dp, dp, ctypes.c_int32]
    L.vsr_elasticity_damping.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
    L.vsr_elasticity_pcg_solve.argtypes = [P, dp, dp, ctypes.c_double, ctypes.POINTER(SolveInfo)]
    L.vsr_elasticity_destroy.argtypes = [P]
    L.vsr_elasticity_destroy.restype = None
    for name in ("vsr_setup", "vsr_load_vector", "vsr_apply_operator", "vsr_apply_operator_noalloc", "vsr_apply_relaxation", "vsr_pcg_solve",
                 "vsr_get_damping", "vsr_set_profiling", "vsr_kernel_stats", "vsr_factor_info", "vsr_get_tuning", "vsr_set_tuning",
                 "vsr_setup_batch", "vsr_batch_create", "vsr_pcg_solve_batch", "vsr_elasticity_setup",
                 "vsr_elasticity_load_vector", "vsr_elasticity_apply_operator", "vsr_elasticity_apply_relaxation",
                 "vsr_elasticity_damping", "vsr_elasticity_pcg_solve"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != VSR_OK:
        raise VsrError(status, lib().vsr_last_error().decode())


def _ptr(t, numel=None):
    """Device pointer of a contiguous float64 CUDA tensor holding exactly `numel` values.

    The kernels read or write exactly that many entries through the pointer, so a
    shorter tensor is rejected here instead of being overrun on the device."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("vectors must be contiguous float64 CUDA tensors")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"vector has {t.numel()} entries, expected {numel}")
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("vectors must be contiguous float64 CUDA tensors")
    return ctypes.c_void_p(t.data_ptr())


class _Inputs:
    """Host arrays of one problem kept alive while the library reads them."""

    def __init__(self, vertices, kappa=None, mu_override=None):
        self.V = np.ascontiguousarray(vertices, dtype=np.float64)
        if self.V.ndim != 4 or self.V.shape[3] != 3 or min(self.V.shape[:3]) < 2:
            raise ValueError(f"vertices must have shape (nz+1, ny+1, nx+1, 3), got {self.V.shape}")
        nz, ny, nx = self.V.shape[0] - 1, self.V.shape[1] - 1, self.V.shape[2] - 1
        ncell = nx * ny * nz
        self.shape = (nx, ny, nz)
        self.mesh = Mesh(nx, ny, nz, self.V.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self.kappa = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
        self.mu = None if mu_override is None else np.ascontiguousarray(mu_override, dtype=np.float64).reshape(-1)
        if self.kappa is not None and self.kappa.size != ncell:
            raise ValueError(f"kappa has {self.kappa.size} values, expected one per cell ({ncell})")
        if self.mu is not None and self.mu.size != 3 * ncell:
            raise ValueError(f"mu_override has {self.mu.size} values, expected 3 per cell ({3 * ncell})")
        self.coef = Coefficients(
            None if self.kappa is None else self.kappa.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            None if self.mu is None else self.mu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def make_options(relax_fp32=False, cycle=0, lanczos_steps=20, max_iterations=1000, interior_patches_only=False, seed=0,
                 omega=0.0, stream=None, autotune=False, batch_streams=0, batch_eager=False, tune_cache=None,
                 share_factors=False, deterministic=False, coarse_solver="auto", stagnation_window=0,
                 stagnation_factor=0.0):
    opt = Options()
    lib().vsr_default_options(ctypes.byref(opt))
    opt.relax_fp32 = int(bool(relax_fp32))
    opt.cycle = int(cycle)
    opt.lanczos_steps = int(lanczos_steps)
    opt.max_iterations = int(max_iterations)
    opt.interior_patches_only = int(bool(interior_patches_only))
    opt.seed = int(seed)
    opt.omega = float(omega)
    opt.stream = None if stream is None else ctypes.c_void_p(stream)
    opt.autotune = int(bool(autotune))
    opt.batch_streams = int(batch_streams)
    opt.batch_eager = int(bool(batch_eager))
    opt.tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
    opt.share_factors = int(bool(share_factors))
    opt.deterministic = int(bool(deterministic))
    codes = {"auto": 0, "dense": 1, "gmg": 2}
    if coarse_solver not in codes:
        raise ValueError("coarse_solver must be 'auto', 'dense' or 'gmg'")
    opt.coarse_solver = codes[coarse_solver]
    opt.stagnation_window = int(stagnation_window)
    opt.stagnation_factor = float(stagnation_factor)
    return opt


class Problem:
    """One discretized Poisson problem and its preconditioner, resident on the GPU."""

    def __init__(self, vertices, p, kappa=None, mu_override=None, _handle=None, **options):
        L = lib()
        self._owned = _handle is None
        if _handle is None:
            self._in = _Inputs(vertices, kappa, mu_override)
            opt = make_options(**options)
            h = ctypes.c_void_p()
            _check(L.vsr_setup(ctypes.byref(self._in.mesh), int(p), ctypes.byref(self._in.coef), ctypes.byref(opt),
                               ctypes.byref(h)))
            self.shape = self._in.shape
        else:
            h = _handle
            self.shape = None
        self._h = h
        self.p = p
        self.n = int(L.vsr_num_dofs(h))
        self.q = (3 * (p + 1) + 1) // 2
        self.ncell = None if self.shape is None else self.shape[0] * self.shape[1] * self.shape[2]

    def tuning(self):
        """Launch shapes in use: (Cartesian-operator cells/workgroup FP64, FP32, panel unroll,
        general-operator workgroups/cell FP64, FP32, threads per patch workgroup)."""
        a = (ctypes.c_int32 * 6)()
        _check(lib().vsr_get_tuning(self._h, a))
        return tuple(a)

    def set_tuning(self, shapes):
        a = (ctypes.c_int32 * 6)(*[int(v) for v in shapes])
        _check(lib().vsr_set_tuning(self._h, a))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value and getattr(self, "_owned", True):
            lib().vsr_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_vector(self, f, b):
        _check(lib().vsr_load_vector(self._h, _ptr(f, None if self.ncell is None else self.ncell * self.q ** 3), _ptr(b, self.n)))

    def apply_operator(self, x, y):
        _check(lib().vsr_apply_operator(self._h, _ptr(x, self.n), _ptr(y, self.n)))

    def apply_operator_noalloc(self, x, y):
        """y = A x through the allocation-free entry point (static device workspace)."""
        _check(lib().vsr_apply_operator_noalloc(self._h, _ptr(x, self.n), _ptr(y, self.n)))

    def apply_relaxation(self, r, z, mode=0):
        _check(lib().vsr_apply_relaxation(self._h, _ptr(r, self.n), _ptr(z, self.n), int(mode)))

    def pcg_solve(self, b, x, rtol=1e-8, raise_on_noconv=True):
        info = SolveInfo()
        st = lib().vsr_pcg_solve(self._h, _ptr(b, self.n), _ptr(x, self.n), float(rtol), ctypes.byref(info))
        if st != VSR_OK and (raise_on_noconv or st != VSR_ENOCONV):
            _check(st)
        out = info.as_dict()
        out["status"] = st
        return out

    def damping(self):
        w, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().vsr_get_damping(self._h, ctypes.byref(w), ctypes.byref(a), ctypes.byref(b)))
        return w.value, a.value, b.value

    def set_profiling(self, enable=True):
        _check(lib().vsr_set_profiling(self._h, int(bool(enable))))

    def kernel_stats(self):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(lib().vsr_kernel_stats(self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value

    def factor_info(self):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().vsr_factor_info(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


class Batch:
    """Independent problems solved together by the batched PCG (members on several streams,
    one lockstep iteration replayed from a hipGraph)."""

    def __init__(self, problems, progress=None, **options):
        """problems: list of dicts with keys vertices, p and optionally kappa, mu_override.
        Members are set up one at a time (progress(i, member) is called after each), then
        handed to the batch."""
        L = lib()
        members = []
        try:
            for i, d in enumerate(problems):
                members.append(Problem(d["vertices"], int(d["p"]), kappa=d.get("kappa"),
                                       mu_override=d.get("mu_override"), **options))
                if progress is not None:
                    progress(i, members[-1])
            opt = make_options(**options)
            handles = (ctypes.c_void_p * len(members))(*[m._h.value for m in members])
            h = ctypes.c_void_p()
            _check(L.vsr_batch_create(len(members), handles, ctypes.byref(opt), ctypes.byref(h)))
        except BaseException:
            for m in members:
                m.close()
            raise
        for m in members:
            m._owned = False   # the batch frees them
        self._h = h
        self.members = members

    def __len__(self):
        return len(self.members)

    def pcg_solve(self, bs, xs, rtol=1e-8, raise_on_noconv=True):
        count = len(self.members)
        if len(bs) != count or len(xs) != count:
            raise ValueError("one b and one x per member")
        bp = (ctypes.c_void_p * count)(*[_ptr(b, m.n).value for b, m in zip(bs, self.members)])
        xp = (ctypes.c_void_p * count)(*[_ptr(x, m.n).value for x, m in zip(xs, self.members)])
        infos = (SolveInfo * count)()
        st = lib().vsr_pcg_solve_batch(self._h, bp, xp, float(rtol), infos)
        if st != VSR_OK and (raise_on_noconv or st != VSR_ENOCONV):
            _check(st)
        return [dict(infos[i].as_dict(), status=st) for i in range(count)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            for m in self.members:
                m._h = None
            lib().vsr_destroy_batch(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned surrogate
def _setup_surrogate_signatures():
    L = lib()
    if getattr(L, "_surrogate_ready", False):
        return L
    P = ctypes.c_void_p
    dpp = ctypes.POINTER(ctypes.c_double)
    L.vsr_mlp_num_params.restype = ctypes.c_int32
    L.vsr_surrogate_features.argtypes = [ctypes.c_int64, dpp, dpp, ctypes.c_int32, P, dpp]
    L.vsr_surrogate_ratio.argtypes = [ctypes.c_int64, dpp, dpp, dpp]
    L.vsr_surrogate_labels.argtypes = [ctypes.c_int64, dpp, ctypes.c_int32, dpp, dpp]
    L.vsr_mlp_forward.argtypes = [P, ctypes.c_int32, P, ctypes.c_int64, P]
    L.vsr_mlp_gradient.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int64, P, P]
    L.vsr_mlp_train.argtypes = [P, P, P, ctypes.c_int32, P, P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_float, P]
    L.vsr_surrogate_scalings.argtypes = [ctypes.c_int64, dpp, dpp, ctypes.c_int32, P, ctypes.c_int32, dpp,
                                         ctypes.POINTER(ctypes.c_int32)]
    for name in ("vsr_surrogate_features", "vsr_surrogate_ratio", "vsr_surrogate_labels", "vsr_mlp_forward",
                 "vsr_mlp_gradient", "vsr_mlp_train", "vsr_surrogate_scalings"):
        getattr(L, name).restype = ctypes.c_int
    L._surrogate_ready = True
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tp(t, dtype, numel=None):
    """Device pointer of a contiguous CUDA tensor of `dtype` holding exactly `numel` values."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"tensor has {t.numel()} entries, expected {numel}")
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _rows(X, width, name):
    """Number of rows of a (rows, width) sample matrix."""
    if X.dim() != 2 or X.shape[1] != width:
        raise ValueError(f"{name} must have shape (n, {width}), got {tuple(X.shape)}")
    return int(X.shape[0])


def _cells(corners):
    C = np.ascontiguousarray(corners, dtype=np.float64)
    if C.ndim < 2 or C.size != 24 * C.shape[0]:
        raise ValueError(f"corners must hold 24 values per cell, got shape {C.shape}")
    return C


def mesh_corners(vertices):
    """Corners (ncell, 2, 2, 2, 3) [cell, c, b, a, coord] of a structured mesh's cells (indexing only)."""
    V = np.asarray(vertices, dtype=np.float64)
    nz, ny, nx = V.shape[0] - 1, V.shape[1] - 1, V.shape[2] - 1
    out = np.empty((nz, ny, nx, 2, 2, 2, 3))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                out[:, :, :, c, b, a, :] = V[c:c + nz, b:b + ny, a:a + nx, :]
    return np.ascontiguousarray(out.reshape(nz * ny * nx, 2, 2, 2, 3))


def mlp_num_params():
    return int(_setup_surrogate_signatures().vsr_mlp_num_params())


def surrogate_features(corners, p, kappa=None):
    import torch
    L = _setup_surrogate_signatures()
    C = _cells(corners)
    n = C.shape[0]
    k = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    if k is not None and k.size != n:
        raise ValueError("kappa must hold one value per cell")
    X = torch.empty((n, 74), dtype=torch.float32, device="cuda")
    mu = np.empty((n, 3))
    _check(L.vsr_surrogate_features(n, _dp(C), _dp(k), int(p), _tp(X, torch.float32), _dp(mu)))
    return X, mu


def surrogate_ratio(corners, mu):
    L = _setup_surrogate_signatures()
    C = _cells(corners)
    m = np.ascontiguousarray(mu, dtype=np.float64)
    if m.size != 3 * C.shape[0]:
        raise ValueError("mu must hold 3 values per cell")
    r = np.empty(C.shape[0])
    _check(L.vsr_surrogate_ratio(C.shape[0], _dp(C), _dp(m), _dp(r)))
    return r


def surrogate_labels(corners, p):
    L = _setup_surrogate_signatures()
    C = _cells(corners)
    d = np.empty((C.shape[0], 3))
    r = np.empty(C.shape[0])
    _check(L.vsr_surrogate_labels(C.shape[0], _dp(C), int(p), _dp(d), _dp(r)))
    return d, r


def mlp_forward(params, X, bf16=True):
    import torch
    L = _setup_surrogate_signatures()
    n = _rows(X, 74, "X")
    Y = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    _check(L.vsr_mlp_forward(_tp(params, torch.float32, mlp_num_params()), int(bool(bf16)), _tp(X, torch.float32), n,
                             _tp(Y, torch.float32)))
    return Y


def mlp_gradient(params, X, T, bf16=True):
    import torch
    L = _setup_surrogate_signatures()
    n = _rows(X, 74, "X")
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(L.vsr_mlp_gradient(_tp(params, torch.float32, mlp_num_params()), int(bool(bf16)), _tp(X, torch.float32),
                              _tp(T, torch.float32, 3 * n), n, _tp(g, torch.float32), _tp(loss, torch.float32)))
    return g, loss


def mlp_train(params, m, v, X, T, order, batch, steps, step0=0, lr=1e-3, bf16=True):
    import torch
    L = _setup_surrogate_signatures()
    n = _rows(X, 74, "X")
    npar = mlp_num_params()
    if order.numel() < int(steps) * int(batch):
        raise ValueError(f"order has {order.numel()} entries, {int(steps) * int(batch)} needed")
    if order.numel() and (int(order.min()) < 0 or int(order.max()) >= n):
        raise ValueError("order holds a row index outside [0, n)")
    losses = torch.empty(steps, dtype=torch.float32, device="cuda")
    _check(L.vsr_mlp_train(_tp(params, torch.float32, npar), _tp(m, torch.float32, npar), _tp(v, torch.float32, npar),
                           int(bool(bf16)), _tp(X, torch.float32), _tp(T, torch.float32, 3 * n), n,
                           _tp(order, torch.int32), int(batch), int(steps), int(step0), float(lr),
                           _tp(losses, torch.float32)))
    return losses


def surrogate_scalings(corners, p, params, kappa=None, bf16=True):
    import torch
    L = _setup_surrogate_signatures()
    C = _cells(corners)
    k = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    if k is not None and k.size != C.shape[0]:
        raise ValueError("kappa must hold one value per cell")
    mu = np.empty((C.shape[0], 3))
    used = np.empty(C.shape[0], dtype=np.int32)
    _check(L.vsr_surrogate_scalings(C.shape[0], _dp(C), _dp(k), int(p), _tp(params, torch.float32, mlp_num_params()),
                                    int(bool(bf16)),
                                    _dp(mu), used.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return mu, used


class Elasticity:
    """Primal linear elasticity (Sec. 3.1) with the SDC relaxation, resident on the GPU: Lame
    parameters mu, lam on a tensor grid of boxes; vectors hold 3 n values, component after
    component."""

    def __init__(self, vertices, p, mu, lam, **options):
        L = lib()
        self._in = _Inputs(vertices, None, None)
        opt = make_options(**options)
        h = ctypes.c_void_p()
        _check(L.vsr_elasticity_setup(ctypes.byref(self._in.mesh), int(p), float(mu), float(lam), ctypes.byref(opt),
                                      ctypes.byref(h)))
        self._h = h
        self.p = p
        self.n = int(L.vsr_elasticity_num_dofs(h))
        self.q = (3 * (p + 1) + 1) // 2
        nz, ny, nx = self._in.shape[0], self._in.shape[1], self._in.shape[2]
        self.ncell = nx * ny * nz

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().vsr_elasticity_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_vector(self, f, b):
        _check(lib().vsr_elasticity_load_vector(self._h, _ptr(f, 3 * self.ncell * self.q ** 3), _ptr(b, self.n)))

    def apply_operator(self, x, y):
        _check(lib().vsr_elasticity_apply_operator(self._h, _ptr(x, self.n), _ptr(y, self.n)))

    def apply_relaxation(self, r, z, mode=0):
        _check(lib().vsr_elasticity_apply_relaxation(self._h, _ptr(r, self.n), _ptr(z, self.n), int(mode)))

    def damping(self):
        w, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().vsr_elasticity_damping(self._h, ctypes.byref(w), ctypes.byref(a), ctypes.byref(b)))
        return w.value, a.value, b.value

    def pcg_solve(self, b, x, rtol=1e-8, raise_on_noconv=True):
        info = SolveInfo()
        st = lib().vsr_elasticity_pcg_solve(self._h, _ptr(b, self.n), _ptr(x, self.n), float(rtol), ctypes.byref(info))
        if st != VSR_OK and (raise_on_noconv or st != VSR_ENOCONV):
            _check(st)
        out = info.as_dict()
        out["status"] = st
        return out

