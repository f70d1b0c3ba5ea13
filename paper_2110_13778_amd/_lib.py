"""ctypes binding of libfagbi.so (the C ABI in include/fagbi.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  Device arrays are torch CUDA tensors (float64, contiguous); host
arrays are numpy arrays.  Errors raise FagbiError with the library message.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libfagbi.so")

OK, E_ARG, E_MESH, E_STATE, E_OOM, E_HIP, E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
W_NOT_CONVERGED = 1
FP64, MIXED = 0, 1
PRECOND_NONE, PRECOND_DIAG, PRECOND_BLOCK, PRECOND_GROUP = 0, 1, 2, 3
MLP_OFF, MLP_PRECOND, MLP_GATED = 0, 1, 2
RADII_LEVEL, RADII_CLUSTER = 0, 1
BASIS_S0, BASIS_S1 = 0, 1          # box functions (per panel) / hat functions (per vertex)
PART_NEAR, PART_FAR, PART_ALL = 1, 2, 3

EXPORTS = ["fagbi_default_params", "fagbi_create", "fagbi_build_tree",
           "fagbi_assemble_nearfield", "fagbi_matvec", "fagbi_matvec_parts",
           "fagbi_precond_apply", "fagbi_rhs", "fagbi_rhs_treecode", "fagbi_solve",
           "fagbi_solvation_energy", "fagbi_solvation_energy_treecode", "fagbi_get_tree_info",
           "fagbi_get_permutation", "fagbi_set_profiling", "fagbi_get_profile",
           "fagbi_mlp_dataset", "fagbi_mlp_train", "fagbi_mlp_forward", "fagbi_mlp_grad",
           "fagbi_mlp_get_weights", "fagbi_mlp_set_weights", "fagbi_get_mlp_stats",
           "fagbi_solvation_energy_noalloc", "fagbi_destroy", "fagbi_last_error"]
MLP_NIN, MLP_NOUT, MLP_NAUX, MLP_NPARAM, MLP_NBLOB = 16, 6, 8, 35974, 36093


class Params(C.Structure):
    _fields_ = [("eps_in", C.c_double), ("eps_out", C.c_double), ("kappa", C.c_double),
                ("eta0", C.c_double),
                ("leaf_size", C.c_int32), ("p_leaf", C.c_int32), ("adaptive", C.c_int32),
                ("p_max", C.c_int32),
                ("quad_duffy", C.c_int32), ("near_ratio", C.c_double),
                ("precision", C.c_int32), ("precond", C.c_int32), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("max_outer", C.c_int32), ("inner_tol", C.c_double),
                ("mlp_mode", C.c_int32), ("mlp_gate_tol", C.c_double), ("rhs_theta", C.c_double),
                ("rhs_pmax", C.c_int32), ("radii", C.c_int32), ("basis", C.c_int32)]


class TreeInfo(C.Structure):
    _fields_ = [("n_panels", C.c_int64), ("n_leaves", C.c_int64), ("levels", C.c_int32),
                ("lmin", C.c_int32), ("near_pairs", C.c_int64), ("m2l_pairs", C.c_int64),
                ("m2l_flops_fp", C.c_int64), ("singular_pairs", C.c_int64 * 4),
                ("order_leaf", C.c_int32), ("order_root", C.c_int32),
                ("rho_leaf", C.c_double), ("h_leaf", C.c_double),
                ("lev_clusters", C.c_int32 * 21), ("lev_order", C.c_int32 * 21),
                ("lev_offsets", C.c_int32 * 21), ("lev_pad", C.c_int32), ("lev_pairs", C.c_int64 * 21),
                ("device_bytes", C.c_int64), ("hat_rows", C.c_int64), ("hat_entries", C.c_int64)]


class SolveInfo(C.Structure):
    _fields_ = [("outer_iterations", C.c_int32), ("inner_iterations", C.c_int32),
                ("matvecs_fp64", C.c_int32), ("matvecs_fp32", C.c_int32),
                ("rel_residual", C.c_double), ("t_rhs_ms", C.c_double),
                ("t_solve_ms", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("matvecs", C.c_int64 * 2), ("ms_total", C.c_double * 2),
                ("ms_near", C.c_double * 2), ("ms_up", C.c_double * 2),
                ("ms_m2l", C.c_double * 2), ("ms_down", C.c_double * 2),
                ("ms_tree", C.c_double), ("ms_classify", C.c_double), ("ms_surrogate", C.c_double),
                ("ms_singular", C.c_double), ("ms_fmm_setup", C.c_double), ("ms_precond", C.c_double),
                ("ms_m2l_leaf", C.c_double * 2)]


class FagbiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fagbi error %d: %s" % (code, msg))
        self.code = code


_lib = None


def load():
    """Load libfagbi.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise ImportError("libfagbi.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(LIBPATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "fagbi_default_params": [C.POINTER(Params)],
        "fagbi_create": [C.POINTER(Params), C.POINTER(vp)],
        "fagbi_build_tree": [vp, vp, i64, vp, i64],
        "fagbi_assemble_nearfield": [vp, vp],
        "fagbi_matvec": [vp, vp, vp, i32, vp],
        "fagbi_matvec_parts": [vp, vp, vp, i32, i32, vp],
        "fagbi_precond_apply": [vp, vp, vp, vp],
        "fagbi_rhs": [vp, vp, vp, i64, vp, vp],
        "fagbi_rhs_treecode": [vp, vp, vp, i64, C.c_double, i32, vp, vp],
        "fagbi_solve": [vp, vp, vp, i64, vp, C.POINTER(SolveInfo), vp],
        "fagbi_solvation_energy": [vp, vp, vp, vp, i64, dp, vp],
        "fagbi_solvation_energy_treecode": [vp, vp, vp, vp, i64, C.c_double, i32, dp, vp],
        "fagbi_solvation_energy_noalloc": [vp, vp, vp, i64, vp, vp],
        "fagbi_get_tree_info": [vp, C.POINTER(TreeInfo)],
        "fagbi_get_permutation": [vp, vp],
        "fagbi_set_profiling": [vp, i32],
        "fagbi_get_profile": [vp, C.POINTER(Profile)],
        "fagbi_mlp_dataset": [vp, i64, vp, vp, vp, C.POINTER(i64), vp],
        "fagbi_mlp_train": [vp, vp, vp, vp, i64, i32, i32, C.c_float, C.c_uint64, vp, vp],
        "fagbi_mlp_forward": [vp, vp, vp, i64, vp],
        "fagbi_mlp_grad": [vp, vp, vp, vp, i32, C.POINTER(C.c_float), vp, vp],
        "fagbi_mlp_get_weights": [vp, vp, i64],
        "fagbi_mlp_set_weights": [vp, vp, i64],
        "fagbi_get_mlp_stats": [vp, C.POINTER(i64), C.POINTER(i64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.fagbi_destroy.argtypes = [vp]
    lib.fagbi_destroy.restype = None
    lib.fagbi_last_error.argtypes = []
    lib.fagbi_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(code):
    if code < 0:
        raise FagbiError(code, _lib.fagbi_last_error().decode())
    return code


def default_params(**kw):
    lib = load()
    p = Params()
    _check(lib.fagbi_default_params(C.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _dev(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _devf(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


class Handle:
    """One operator/solver instance (owns its device memory)."""

    def __init__(self, params=None, **kw):
        self.lib = load()
        self.params = params if params is not None else default_params(**kw)
        h = C.c_void_p()
        _check(self.lib.fagbi_create(C.byref(self.params), C.byref(h)))
        self.h = h
        self.n = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.fagbi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_tree(self, verts, tris):
        v, vp = _host(verts, np.float64)
        t, tp = _host(tris, np.int32)
        _check(self.lib.fagbi_build_tree(self.h, vp, len(v), tp, len(t)))
        self.n = len(t)
        return self

    def assemble_nearfield(self, stream=None):
        _check(self.lib.fagbi_assemble_nearfield(self.h, _stream(stream)))
        return self

    def matvec(self, x, y, precision=FP64, parts=PART_ALL, stream=None):
        _check(self.lib.fagbi_matvec_parts(self.h, _dev(x), _dev(y), precision, parts,
                                           _stream(stream)))
        return y

    def precond_apply(self, z, y, stream=None):
        _check(self.lib.fagbi_precond_apply(self.h, _dev(z), _dev(y), _stream(stream)))
        return y

    def rhs(self, xq, q, b, stream=None):
        xq_, xqp = _host(xq, np.float64)
        q_, qp = _host(q, np.float64)
        _check(self.lib.fagbi_rhs(self.h, xqp, qp, len(q_), _dev(b), _stream(stream)))
        return b

    def rhs_treecode(self, xq, q, theta, b, p_max=8, stream=None):
        xq_, xqp = _host(xq, np.float64)
        q_, qp = _host(q, np.float64)
        _check(self.lib.fagbi_rhs_treecode(self.h, xqp, qp, len(q_), float(theta), int(p_max), _dev(b),
                                           _stream(stream)))
        return b

    def solve(self, xq, q, x, stream=None):
        xq_, xqp = _host(xq, np.float64)
        q_, qp = _host(q, np.float64)
        info = SolveInfo()
        code = _check(self.lib.fagbi_solve(self.h, xqp, qp, len(q_), _dev(x), C.byref(info),
                                           _stream(stream)))
        return code, info

    def solvation_energy(self, x, xq, q, stream=None):
        xq_, xqp = _host(xq, np.float64)
        q_, qp = _host(q, np.float64)
        e = C.c_double()
        _check(self.lib.fagbi_solvation_energy(self.h, _dev(x), xqp, qp, len(q_), C.byref(e),
                                               _stream(stream)))
        return e.value

    def solvation_energy_noalloc(self, x, chg, E, stream=None):
        """chg: float64 CUDA tensor [nc, 4] (x, y, z, q); E: float64 CUDA tensor [1]
        receives the energy (asynchronous)."""
        if chg.dim() != 2 or chg.shape[1] != 4:
            raise ValueError("chg must be [nc, 4]")
        _check(self.lib.fagbi_solvation_energy_noalloc(self.h, _dev(x), _dev(chg), chg.shape[0], _dev(E),
                                                       _stream(stream)))
        return E

    def solvation_energy_treecode(self, x, xq, q, theta, p_max=8, stream=None):
        xq_, xqp = _host(xq, np.float64)
        q_, qp = _host(q, np.float64)
        e = C.c_double()
        _check(self.lib.fagbi_solvation_energy_treecode(self.h, _dev(x), xqp, qp, len(q_), float(theta),
                                                        int(p_max), C.byref(e), _stream(stream)))
        return e.value

    def tree_info(self):
        ti = TreeInfo()
        _check(self.lib.fagbi_get_tree_info(self.h, C.byref(ti)))
        return ti

    # ---- learned near-field surrogate ----
    def mlp_dataset(self, max_pairs, stream=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        X = torch.empty(max_pairs * MLP_NIN, dtype=torch.float32, device=dev)
        T = torch.empty(max_pairs * MLP_NOUT, dtype=torch.float32, device=dev)
        A = torch.empty(max_pairs * MLP_NAUX, dtype=torch.float32, device=dev)
        n = C.c_int64()
        _check(self.lib.fagbi_mlp_dataset(self.h, max_pairs, _devf(X), _devf(T), _devf(A),
                                          C.byref(n), _stream(stream)))
        n = n.value
        return (X[:n * MLP_NIN].view(n, MLP_NIN), T[:n * MLP_NOUT].view(n, MLP_NOUT),
                A[:n * MLP_NAUX].view(n, MLP_NAUX))

    @staticmethod
    def _rows(X, T=None, A=None):
        n = X.numel() // MLP_NIN
        if X.numel() != n * MLP_NIN or (T is not None and T.numel() != n * MLP_NOUT) or \
                (A is not None and A.numel() != n * MLP_NAUX):
            raise ValueError("expected X[n,16], T[n,6], aux[n,8]")
        return n

    def mlp_train(self, X, T, A, epochs=20, batch=4096, lr=2e-3, seed=1, stream=None):
        hist = np.zeros(epochs, np.float32)
        n = self._rows(X, T, A)
        _check(self.lib.fagbi_mlp_train(self.h, _devf(X), _devf(T), _devf(A), n, epochs,
                                        batch, lr, seed, hist.ctypes.data_as(C.c_void_p),
                                        _stream(stream)))
        return hist

    def mlp_forward(self, X, stream=None):
        import torch
        n = self._rows(X)
        Y = torch.empty(n * MLP_NOUT, dtype=torch.float32, device=X.device)
        _check(self.lib.fagbi_mlp_forward(self.h, _devf(X), _devf(Y), n, _stream(stream)))
        return Y.view(n, MLP_NOUT)

    def mlp_grad(self, theta, X, T, stream=None):
        th = np.ascontiguousarray(theta, np.float32)
        g = np.zeros(MLP_NPARAM, np.float32)
        loss = C.c_float()
        if th.size != MLP_NPARAM:
            raise ValueError("theta must hold %d floats" % MLP_NPARAM)
        n = self._rows(X, T)
        _check(self.lib.fagbi_mlp_grad(self.h, th.ctypes.data_as(C.c_void_p), _devf(X), _devf(T),
                                       n, C.byref(loss), g.ctypes.data_as(C.c_void_p),
                                       _stream(stream)))
        return loss.value, g

    def mlp_get_weights(self):
        b = np.zeros(MLP_NBLOB, np.float32)
        _check(self.lib.fagbi_mlp_get_weights(self.h, b.ctypes.data_as(C.c_void_p), MLP_NBLOB))
        return b

    def mlp_set_weights(self, blob):
        b = np.ascontiguousarray(blob, np.float32)
        _check(self.lib.fagbi_mlp_set_weights(self.h, b.ctypes.data_as(C.c_void_p), len(b)))

    def mlp_stats(self):
        g, c = C.c_int64(), C.c_int64()
        _check(self.lib.fagbi_get_mlp_stats(self.h, C.byref(g), C.byref(c)))
        return g.value, c.value

    def set_profiling(self, on):
        _check(self.lib.fagbi_set_profiling(self.h, 1 if on else 0))

    def profile(self):
        p = Profile()
        _check(self.lib.fagbi_get_profile(self.h, C.byref(p)))
        return {k: (list(getattr(p, k)) if hasattr(getattr(p, k), "__len__") else getattr(p, k))
                for k, _ in Profile._fields_}

    def permutation(self):
        p = np.zeros(self.n, np.int32)
        _check(self.lib.fagbi_get_permutation(self.h, p.ctypes.data_as(C.c_void_p)))
        return p
