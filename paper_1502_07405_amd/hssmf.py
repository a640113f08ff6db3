"""Python binding of libhssmf (include/hssmf.h): argument marshalling only.

Every step of factorization and solve runs in the HIP library; PyTorch only
provides device memory (float64 CUDA tensors) and the stream.  There is no
CPU fallback: if the library is missing or no GPU is present the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhssmf.so")

HSSMF_OK, HSSMF_EINVAL, HSSMF_ENOMEM, HSSMF_ESINGULAR, HSSMF_ERANK, HSSMF_ENOCONV, HSSMF_EDEVICE = 0, -1, -2, -3, -4, -5, -6
HSSMF_ETOOBIG = -7
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}
OUTER = {"ir": 0, "gmres": 1}

EXPORTS = ["hssmf_default_opts", "hssmf_factor", "hssmf_refactor", "hssmf_apply", "hssmf_solve",
           "hssmf_solve_transpose", "hssmf_adjoint", "hssmf_stats_get", "hssmf_hss_ranks",
           "hssmf_last_failed_front", "hssmf_destroy", "hssmf_strerror", "hssmf_profile_enable",
           "hssmf_profile_read", "hssmf_factor_batch", "hssmf_systems", "hssmf_measure_peaks",
           "hssmf_refactor_device", "hssmf_solve_batch", "hssmf_solve_noalloc",
           "hssmf_front_data", "hssmf_static_pivoting", "hssmf_nested_dissection", "hssmf_factor_z",
           "hssmf_refactor_z", "hssmf_refactor_z_device"]
KCLASS = {"id": 0, "gemm64": 1, "gemmlp": 2, "lupanel": 3, "idres": 4}


class HssmfError(RuntimeError):
    def __init__(self, code, what, front=-1):
        super().__init__(f"{what}: {strerror(code)} ({code})" + (f", front {front}" if front >= 0 else ""))
        self.code = code
        self.front = front


MEM_HOST, MEM_DEVICE = 0, 1


class CSRArg(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("mem", ctypes.c_int32)]


class OrderingArg(ctypes.Structure):
    _fields_ = [("perm", ctypes.c_void_p), ("nfront", ctypes.c_int32), ("sep_ptr", ctypes.c_void_p),
                ("parent", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("rel_tol", ctypes.c_double), ("leaf_size", ctypes.c_int32), ("min_sep_hss", ctypes.c_int32),
                ("d0", ctypes.c_int32), ("dd", ctypes.c_int32), ("p", ctypes.c_int32), ("d_max", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("gemm_prec", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("tol", ctypes.c_double), ("max_it", ctypes.c_int32),
                ("id_kernel", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("gemm_tile", ctypes.c_int32), ("abs_tol", ctypes.c_double),
                ("keep_stages", ctypes.c_int32), ("hss_update", ctypes.c_int32),
                ("power_q", ctypes.c_int32), ("srrqr_f", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("failed_front", ctypes.c_int32), ("outer_switched", ctypes.c_int32)]


class Peaks(ctypes.Structure):
    _fields_ = [("hbm_GBps", ctypes.c_double), ("fp64_valu_TFLOPs", ctypes.c_double),
                ("fp64_mfma_TFLOPs", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nfront", ctypes.c_int32), ("n_hss_fronts", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("max_d", ctypes.c_int32), ("growth_rounds", ctypes.c_int32),
                ("factor_bytes", ctypes.c_int64), ("t_plan_ms", ctypes.c_double),
                ("t_factor_ms", ctypes.c_double), ("flops_factor", ctypes.c_double),
                ("peak_bytes", ctypes.c_int64), ("trsv_multi_ops", ctypes.c_int32), ("srrqr_swaps", ctypes.c_int32)]


_lib = None


def load():
    """Load libhssmf.so (built in-tree by paper_1502_07405_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1502_07405_amd/build.py first")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        L.hssmf_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.hssmf_factor.argtypes = [ctypes.POINTER(CSRArg), ctypes.POINTER(OrderingArg), ctypes.POINTER(Opts), vp,
                                   ctypes.POINTER(vp)]
        L.hssmf_refactor.argtypes = [vp, vp]
        L.hssmf_factor_z.argtypes = [ctypes.POINTER(CSRArg), ctypes.POINTER(OrderingArg), ctypes.POINTER(Opts), vp,
                                     ctypes.POINTER(vp)]
        L.hssmf_refactor_z.argtypes = [vp, vp]
        L.hssmf_refactor_z_device.argtypes = [vp, vp]
        L.hssmf_refactor_device.argtypes = [vp, vp]
        L.hssmf_apply.argtypes = [vp, i32, vp, vp]
        L.hssmf_solve.argtypes = [vp, i32, vp, vp, ctypes.POINTER(Info)]
        L.hssmf_solve_transpose.argtypes = [vp, i32, vp, vp, ctypes.POINTER(Info)]
        L.hssmf_solve_batch.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(Info)]
        L.hssmf_solve_noalloc.argtypes = [vp, i32, vp, vp, ctypes.POINTER(Info)]
        L.hssmf_front_data.argtypes = [vp, i32, i32, vp, ctypes.c_int64, vp]
        L.hssmf_adjoint.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(Info)]
        L.hssmf_stats_get.argtypes = [vp, ctypes.POINTER(Stats)]
        L.hssmf_hss_ranks.argtypes = [vp, vp, i32]
        L.hssmf_last_failed_front.argtypes = [vp]
        L.hssmf_destroy.argtypes = [vp]
        L.hssmf_destroy.restype = None
        L.hssmf_strerror.argtypes = [i32]
        L.hssmf_strerror.restype = ctypes.c_char_p
        L.hssmf_factor_batch.argtypes = [i32, ctypes.POINTER(CSRArg), ctypes.POINTER(OrderingArg),
                                         ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
        L.hssmf_systems.argtypes = [vp, vp, i32]
        L.hssmf_profile_enable.argtypes = [i32]
        L.hssmf_measure_peaks.argtypes = [vp, ctypes.POINTER(Peaks)]
        L.hssmf_profile_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double)]
        L.hssmf_static_pivoting.argtypes = [ctypes.POINTER(CSRArg), vp, vp, vp]
        L.hssmf_nested_dissection.argtypes = [ctypes.POINTER(CSRArg), i32, i32, vp, vp, vp, ctypes.POINTER(i32)]
        _lib = L
    return _lib


def profile_enable(on=True):
    """Turn the library's kernel timing hooks on or off."""
    rc = load().hssmf_profile_enable(int(bool(on)))
    if rc != HSSMF_OK:
        raise HssmfError(rc, "hssmf_profile_enable")


def profile_read(kclass):
    """(ms, launches, flops) accumulated for a kernel class since the last read."""
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    rc = load().hssmf_profile_read(KCLASS.get(kclass, kclass), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl))
    if rc != HSSMF_OK:
        raise HssmfError(rc, "hssmf_profile_read")
    return ms.value, n.value, fl.value


def measure_peaks(stream=None):
    """Measured device rates: {"hbm_GBps", "fp64_valu_TFLOPs", "fp64_mfma_TFLOPs"}
    from the library's copy, FMA-loop and matrix-core-loop probes."""
    out = Peaks()
    rc = load().hssmf_measure_peaks(stream, ctypes.byref(out))
    if rc != HSSMF_OK:
        raise HssmfError(rc, "hssmf_measure_peaks")
    return {k: getattr(out, k) for k, _ in Peaks._fields_}


def strerror(code):
    return load().hssmf_strerror(int(code)).decode()


def default_opts(**kw):
    o = Opts()
    load().hssmf_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "gemm_prec" and isinstance(v, str):
            v = PREC[v]
        if k == "outer" and isinstance(v, str):
            v = OUTER[v]
        if k == "id_kernel" and isinstance(v, str):
            v = {"stepwise": 0, "cooperative": 1, "resident": 2}[v]
        if k == "hss_update" and isinstance(v, str):
            v = {"lowrank": 0, "dense": 1}[v]
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_f64(x, n, torch):
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()
            and x.numel() == n):
        raise ValueError(f"expected a contiguous float64 CUDA tensor with {n} entries")
    return x


def _args(A, ordering, keep):
    arrs = (np.ascontiguousarray(A.rowptr, dtype=np.int64), np.ascontiguousarray(A.colind, dtype=np.int32),
            np.ascontiguousarray(A.val, dtype=np.float64), np.ascontiguousarray(ordering.perm, dtype=np.int32),
            np.ascontiguousarray(ordering.sep_ptr, dtype=np.int32),
            np.ascontiguousarray(ordering.parent, dtype=np.int32))
    keep.append(arrs)
    rp, ci, va, pe, sp, pa = arrs
    return (CSRArg(int(A.n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data, MEM_HOST),
            OrderingArg(pe.ctypes.data, len(pa), sp.ctypes.data, pa.ctypes.data))


def _host_csr(A, keep):
    arrs = (np.ascontiguousarray(A.rowptr, dtype=np.int64), np.ascontiguousarray(A.colind, dtype=np.int32),
            np.ascontiguousarray(A.val, dtype=np.float64))
    keep.append(arrs)
    rp, ci, va = arrs
    return CSRArg(int(A.n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data, MEM_HOST)


def nested_dissection(A, leaf_size=64, sep_leaf=64):
    """hssmf_nested_dissection: a fill-reducing ordering of the graph of
    A + A^T with HSS-ordered separators, as an Ordering."""
    from .problems import Ordering
    keep = []
    csr = _host_csr(A, keep)
    n = int(A.n)
    perm = np.empty(n, dtype=np.int32)
    sep_ptr = np.empty(n + 1, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    nf = ctypes.c_int32()
    rc = load().hssmf_nested_dissection(ctypes.byref(csr), int(leaf_size), int(sep_leaf), perm.ctypes.data,
                                        sep_ptr.ctypes.data, parent.ctypes.data, ctypes.byref(nf))
    if rc != HSSMF_OK:
        raise HssmfError(rc, "hssmf_nested_dissection")
    k = nf.value
    return Ordering(perm, sep_ptr[:k + 1].copy(), parent[:k].copy(), [None] * k, None)


def static_pivoting(A):
    """hssmf_static_pivoting: (colperm, row_scale, col_scale) with
    B(:, i) = Dr A Dc (:, colperm[i]) carrying the matched entries, of
    magnitude 1, on its diagonal."""
    keep = []
    csr = _host_csr(A, keep)
    n = int(A.n)
    q = np.empty(n, dtype=np.int32)
    r = np.empty(n, dtype=np.float64)
    c = np.empty(n, dtype=np.float64)
    rc = load().hssmf_static_pivoting(ctypes.byref(csr), q.ctypes.data, r.ctypes.data, c.ctypes.data)
    if rc != HSSMF_OK:
        raise HssmfError(rc, "hssmf_static_pivoting")
    return q, r, c


def apply_static_pivoting(A, colperm, row_scale, col_scale):
    """The matrix B = Dr A Dc Q of static_pivoting's output as a CSR (host):
    B[i, k] = r_i a[i, colperm[k]] c[colperm[k]].  A solution y of B y = Dr b
    gives x[colperm[k]] = c[colperm[k]] y[k]."""
    from .problems import CSR
    S = A.to_scipy().tocoo()
    pos = np.empty(int(A.n), dtype=np.int64)
    pos[colperm] = np.arange(int(A.n))
    import scipy.sparse as sp
    B = sp.csr_matrix((S.data * row_scale[S.row] * col_scale[S.col], (S.row, pos[S.col])), shape=S.shape)
    B.sort_indices()
    return CSR(int(A.n), B.indptr.astype(np.int64), B.indices.astype(np.int32), B.data.astype(np.float64))


class Factorization:
    """hssmf_factor on CSR / ordering arrays; solves on CUDA tensors or host
    arrays.  device_csr=True hands the CSR arrays over in device memory
    (hssmf_csr.mem = HSSMF_MEM_DEVICE)."""

    def __init__(self, A, ordering, opts=None, stream=None, device_csr=False, **kw):
        import torch
        self._torch = torch
        self.lib = load()
        self.n = int(A.n)
        self.nnz = int(A.rowptr[-1])
        self._keep = []
        csr, ordg = _args(A, ordering, self._keep)
        if device_csr:
            dev = [torch.tensor(np.asarray(a), device="cuda") for a in (A.rowptr, A.colind, A.val)]
            dev = [dev[0].to(torch.int64), dev[1].to(torch.int32), dev[2].to(torch.float64)]
            self._keep.append(dev)
            csr = CSRArg(int(A.n), dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), MEM_DEVICE)
        self.opts = opts if opts is not None else default_opts(**kw)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.hssmf_factor(ctypes.byref(csr), ctypes.byref(ordg), ctypes.byref(self.opts),
                                   ctypes.c_void_p(stream), ctypes.byref(h))
        if rc != HSSMF_OK:
            raise HssmfError(rc, "hssmf_factor", self.lib.hssmf_last_failed_front(None))
        self.h = h
        self.offsets = [0, self.n]
        self._vals_host = np.array(A.val, dtype=np.float64, copy=True)
        self._vals_dev = None

    def factored_values(self, device):
        """The matrix values of the current factorization, as a float64 tensor
        on device."""
        torch = self._torch
        if self._vals_dev is None or self._vals_dev.device != torch.device(device):
            src = self._vals_dev if self._vals_dev is not None else torch.from_numpy(self._vals_host)
            self._vals_dev = src.to(device=device, dtype=torch.float64)
        return self._vals_dev

    def _check(self, rc, what, allow_noconv=False):
        if rc == HSSMF_OK or (allow_noconv and rc == HSSMF_ENOCONV):
            return rc
        raise HssmfError(rc, what, self.lib.hssmf_last_failed_front(self.h))

    def refactor(self, val):
        """New values, same pattern: a float64 CUDA tensor (read in place,
        hssmf_refactor_device) or host values (hssmf_refactor)."""
        torch = self._torch
        if torch is not None and isinstance(val, torch.Tensor) and val.is_cuda:
            _dev_f64(val, self.nnz, torch)
            self._vals_dev = self._vals_host = None
            self._check(self.lib.hssmf_refactor_device(self.h, _ptr(val)), "hssmf_refactor_device")
            self._vals_dev = val.detach().clone()
            return
        v = np.ascontiguousarray(val, dtype=np.float64)
        assert v.size == self.nnz
        self._vals_dev = self._vals_host = None
        self._check(self.lib.hssmf_refactor(self.h, v.ctypes.data), "hssmf_refactor")
        self._vals_host = v.copy()

    def apply(self, x, trans=False):
        torch = self._torch
        _dev_f64(x, self.n, torch)
        y = torch.empty_like(x)
        self._check(self.lib.hssmf_apply(self.h, int(bool(trans)), _ptr(x), _ptr(y)), "hssmf_apply")
        return y

    def _solve(self, fn, what, b, allow_noconv):
        """b: float64 CUDA tensor or numpy array of n entries (one right-hand
        side) or n x nrhs (columns = right-hand sides); the result has b's
        kind and shape.  Returns (x, info) for one right-hand side and
        (x, [info, ...]) for several."""
        torch = self._torch
        if isinstance(b, torch.Tensor):
            if not (b.dtype == torch.float64 and b.shape[0] == self.n and b.dim() in (1, 2)):
                raise ValueError(f"expected float64 with {self.n} rows")
            many = b.dim() == 2
            bc = b.t().contiguous() if many else b.contiguous()   # columns back to back
            xc = torch.empty_like(bc)
            ptr_b, ptr_x = bc.data_ptr(), xc.data_ptr()
        else:
            b = np.asarray(b, dtype=np.float64)
            if b.shape[0] != self.n or b.ndim not in (1, 2):
                raise ValueError(f"expected {self.n} rows")
            many = b.ndim == 2
            bc = np.ascontiguousarray(b.T if many else b)
            xc = np.empty_like(bc)
            ptr_b, ptr_x = bc.ctypes.data, xc.ctypes.data
        nrhs = bc.shape[0] if many else 1
        infos = (Info * max(nrhs, 1))()
        rc = fn(self.h, nrhs, ctypes.c_void_p(ptr_b), ctypes.c_void_p(ptr_x), infos)
        self._check(rc, what, allow_noconv)
        if many:
            return xc.T, [infos[j] for j in range(nrhs)]
        return xc, infos[0]

    def solve(self, b, allow_noconv=False):
        return self._solve(self.lib.hssmf_solve, "hssmf_solve", b, allow_noconv)

    def solve_transpose(self, g, allow_noconv=False):
        return self._solve(self.lib.hssmf_solve_transpose, "hssmf_solve_transpose", g, allow_noconv)

    def adjoint(self, x, g):
        torch = self._torch
        _dev_f64(x, self.n, torch)
        _dev_f64(g, self.n, torch)
        db = torch.empty_like(g)
        dval = torch.empty(self.nnz, dtype=torch.float64, device=g.device)
        info = Info()
        rc = self.lib.hssmf_adjoint(self.h, _ptr(x), _ptr(g), _ptr(db), _ptr(dval), ctypes.byref(info))
        self._check(rc, "hssmf_adjoint")
        return db, dval, info

    def stats(self):
        s = Stats()
        self._check(self.lib.hssmf_stats_get(self.h, ctypes.byref(s)), "hssmf_stats_get")
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    STAGES = {"random": 0, "samples_row": 1, "samples_col": 2, "theta_t": 3, "phi": 4, "update": 5}

    def front_data(self, front, what):
        """hssmf_front_data: an intermediate array of HSS front ``front``
        (``what`` in STAGES) as a numpy array."""
        dims = np.zeros(2, dtype=np.int32)
        w = self.STAGES[what]
        self._check(self.lib.hssmf_front_data(self.h, int(front), w, None, 0, dims.ctypes.data), "hssmf_front_data")
        out = np.zeros((int(dims[0]), int(dims[1])), dtype=np.float64, order="F")
        self._check(self.lib.hssmf_front_data(self.h, int(front), w, out.ctypes.data, out.size, dims.ctypes.data),
                    "hssmf_front_data")
        return out

    def hss_ranks(self):
        nf = self.lib.hssmf_hss_ranks(self.h, None, 0)
        out = np.zeros(5 * max(nf, 1), dtype=np.int32)
        self.lib.hssmf_hss_ranks(self.h, out.ctypes.data, nf)
        return [tuple(int(v) for v in out[5 * i:5 * i + 5]) for i in range(nf)]

    def close(self):
        if getattr(self, "h", None):
            self.lib.hssmf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ZFactorization(Factorization):
    """hssmf_factor_z: a complex system (problems.ZCSR, complex128 values)
    factored through its real-equivalent form.  Vectors are complex128 CUDA
    tensors or numpy arrays of n entries; they cross the boundary as their
    interleaved (real, imaginary) doubles, which is the real form's
    vector of 2n entries."""

    def __init__(self, A, ordering, opts=None, stream=None, **kw):
        import torch
        self._torch = torch
        self.lib = load()
        self.nz = int(A.n)
        self.n = 2 * self.nz
        self.nnz = 4 * int(A.rowptr[-1])
        self._keep = []
        zval = np.ascontiguousarray(A.val, dtype=np.complex128).view(np.float64)
        arrs = (np.ascontiguousarray(A.rowptr, dtype=np.int64), np.ascontiguousarray(A.colind, dtype=np.int32),
                zval, np.ascontiguousarray(ordering.perm, dtype=np.int32),
                np.ascontiguousarray(ordering.sep_ptr, dtype=np.int32),
                np.ascontiguousarray(ordering.parent, dtype=np.int32))
        self._keep.append(arrs)
        rp, ci, va, pe, sp, pa = arrs
        csr = CSRArg(self.nz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, MEM_HOST)
        ordg = OrderingArg(pe.ctypes.data, len(pa), sp.ctypes.data, pa.ctypes.data)
        self.opts = opts if opts is not None else default_opts(**kw)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.hssmf_factor_z(ctypes.byref(csr), ctypes.byref(ordg), ctypes.byref(self.opts),
                                     ctypes.c_void_p(stream), ctypes.byref(h))
        if rc != HSSMF_OK:
            raise HssmfError(rc, "hssmf_factor_z", self.lib.hssmf_last_failed_front(None))
        self.h = h
        self.offsets = [0, self.n]
        self._vals_host = None
        self._vals_dev = None

    def refactor(self, val):
        """New complex values: a complex128 CUDA tensor (read in place,
        hssmf_refactor_z_device) or host values (hssmf_refactor_z)."""
        torch = self._torch
        if isinstance(val, torch.Tensor) and val.is_cuda:
            if not (val.dtype == torch.complex128 and val.is_contiguous() and val.numel() == self.nnz // 4):
                raise ValueError(f"expected a contiguous complex128 tensor of {self.nnz // 4} values")
            self._check(self.lib.hssmf_refactor_z_device(self.h, val.data_ptr()), "hssmf_refactor_z_device")
            return
        v = np.ascontiguousarray(val, dtype=np.complex128).view(np.float64)
        assert v.size == self.nnz // 2
        self._check(self.lib.hssmf_refactor_z(self.h, v.ctypes.data), "hssmf_refactor_z")

    def _as_real(self, z):
        """One complex right-hand side as the real form's vector (a view of
        its interleaved doubles)."""
        torch = self._torch
        if isinstance(z, torch.Tensor):
            if not (z.dtype == torch.complex128 and z.dim() == 1 and z.shape[0] == self.nz):
                raise ValueError(f"expected a complex128 vector of {self.nz} entries")
            return torch.view_as_real(z.contiguous()).reshape(self.n)
        z = np.ascontiguousarray(z, dtype=np.complex128)
        if z.shape != (self.nz,):
            raise ValueError(f"expected a vector of {self.nz} entries")
        return z.view(np.float64)

    def _as_complex(self, x):
        torch = self._torch
        if isinstance(x, torch.Tensor):
            return torch.view_as_complex(x.contiguous().view(self.nz, 2))
        return np.ascontiguousarray(x).view(np.complex128)

    def apply(self, z, trans=False):
        return self._as_complex(Factorization.apply(self, self._as_real(z), trans))

    def solve(self, b, allow_noconv=False):
        x, info = Factorization.solve(self, self._as_real(b), allow_noconv)
        return self._as_complex(x), info

    def solve_transpose(self, g, allow_noconv=False):
        x, info = Factorization.solve_transpose(self, self._as_real(g), allow_noconv)
        return self._as_complex(x), info

    def adjoint(self, x, g):
        raise NotImplementedError("hssmf_adjoint is defined for real systems")


class BatchFactorization(Factorization):
    """hssmf_factor_batch over a list of (A, ordering) systems: one handle,
    vectors are the systems' vectors back to back (see offsets / split)."""

    def __init__(self, systems, opts=None, stream=None, **kw):
        import torch
        self._torch = torch
        self.lib = load()
        self._keep = []
        args = [_args(A, o, self._keep) for A, o in systems]
        csrs = (CSRArg * len(args))(*[a[0] for a in args])
        ords = (OrderingArg * len(args))(*[a[1] for a in args])
        self.n = int(sum(int(A.n) for A, _ in systems))
        self.nnz = int(sum(int(A.rowptr[-1]) for A, _ in systems))
        self.front_offsets = np.cumsum([0] + [len(o.parent) for _, o in systems])
        self.opts = opts if opts is not None else default_opts(**kw)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.hssmf_factor_batch(len(args), csrs, ords, ctypes.byref(self.opts), ctypes.c_void_p(stream),
                                         ctypes.byref(h))
        if rc != HSSMF_OK:
            raise HssmfError(rc, "hssmf_factor_batch", self.lib.hssmf_last_failed_front(None))
        self.h = h
        ns = self.lib.hssmf_systems(h, None, 0)
        off = np.zeros(ns + 1, dtype=np.int64)
        self.lib.hssmf_systems(h, off.ctypes.data, ns + 1)
        self.offsets = [int(v) for v in off]
        self._vals_host = np.concatenate([np.asarray(A.val, dtype=np.float64) for A, _ in systems])
        self._vals_dev = None

    def split(self, x):
        return [x[a:b] for a, b in zip(self.offsets[:-1], self.offsets[1:])]

    def solve_batch(self, bs, allow_noconv=False):
        """hssmf_solve_batch: bs = one right-hand side per system (float64
        CUDA tensors or numpy arrays, each of the system's size); returns
        ([x_s], info) with x_s of the same kind as b_s."""
        torch = self._torch
        sizes = [b - a for a, b in zip(self.offsets[:-1], self.offsets[1:])]
        if len(bs) != len(sizes):
            raise ValueError(f"expected {len(sizes)} right-hand sides")
        keep, xs = [], []
        for b, m in zip(bs, sizes):
            if isinstance(b, torch.Tensor):
                b = b.contiguous()
                if b.dtype != torch.float64 or b.numel() != m:
                    raise ValueError("bad right-hand side")
                x = torch.empty_like(b)
                keep.append((b, b.data_ptr(), x.data_ptr()))
            else:
                b = np.ascontiguousarray(b, dtype=np.float64)
                if b.size != m:
                    raise ValueError("bad right-hand side")
                x = np.empty_like(b)
                keep.append((b, b.ctypes.data, x.ctypes.data))
            xs.append(x)
        pb = (ctypes.c_void_p * len(keep))(*[k[1] for k in keep])
        px = (ctypes.c_void_p * len(keep))(*[k[2] for k in keep])
        info = Info()
        rc = self.lib.hssmf_solve_batch(self.h, pb, px, ctypes.byref(info))
        self._check(rc, "hssmf_solve_batch", allow_noconv)
        return xs, info

    def hss_ranks_by_system(self):
        """hss_ranks() with the fronts renumbered per system:
        {system: [(local front, row rank, col rank, d, rounds), ...]}."""
        out = {}
        for r in self.hss_ranks():
            s = int(np.searchsorted(self.front_offsets, r[0], side="right") - 1)
            out.setdefault(s, []).append((r[0] - int(self.front_offsets[s]),) + tuple(r[1:]))
        return out


class LinearSolve:
    """x = A(val)^{-1} b as a torch.autograd.Function whose backward is the
    hand-written adjoint: one transposed solve with the same factors gives
    dL/db = lambda and dL/dval = -lambda_i x_j on the pattern.  forward
    refactors (hssmf_refactor_device, same pattern and plan) whenever val
    differs from the values the handle holds factors of."""

    @staticmethod
    def make(fact):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, val, b):
                v = val.detach().to(dtype=torch.float64).contiguous()
                if fact.h is None:
                    raise HssmfError(HSSMF_EINVAL, "LinearSolve on a closed factorization")
                if not torch.equal(fact.factored_values(v.device), v):
                    fact.refactor(v)
                x, _ = fact.solve(b.contiguous())
                ctx.save_for_backward(x)
                return x

            @staticmethod
            def backward(ctx, gx):
                (x,) = ctx.saved_tensors
                db, dval, _ = fact.adjoint(x, gx.contiguous())
                return dval, db

        return _Fn.apply
