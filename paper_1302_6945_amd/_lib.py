"""ctypes marshalling for libtikh.so (include/tikh.h).  No compute here."""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libtikh.so")

if not os.path.exists(library_path):
    raise ImportError("libtikh.so is not built: run `python paper_1302_6945_amd/build.py` "
                      "(or __graft_entry__.build()) before using paper_1302_6945_amd")

lib = ctypes.CDLL(library_path)

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


class _Opts(ctypes.Structure):
    _fields_ = [("n_lim", ctypes.c_int32), ("refine", ctypes.c_int32), ("refine_max", ctypes.c_int32),
                ("leaf_wave_groups", ctypes.c_int32), ("refine_tol", ctypes.c_double), ("defer_tol", ctypes.c_double),
                ("record_short", ctypes.c_int32), ("streams", ctypes.c_int32), ("merge_tol", ctypes.c_double),
                ("fallback_nlim", ctypes.c_int32), ("chunk_groups", ctypes.c_int32),
                ("refine_skip", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("k", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("leaf_nodes", ctypes.c_int32), ("solves", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("refine_extra", ctypes.c_int64), ("deferred", ctypes.c_int64), ("host_syncs", ctypes.c_int64),
                ("fallback_groups", ctypes.c_int64), ("refine_skipped", ctypes.c_int64)]


def _sig(name, args, res=ctypes.c_int):
    f = getattr(lib, name)
    f.argtypes = args
    f.restype = res
    return f


_sig("tikh_init", [])
tikh_plan_info = _sig("tikh_plan_info", [_I64, _I64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64)])
_sig("tikh_release", [])
tikh_workspace_bytes = _sig("tikh_workspace_bytes", [_I64, _P, _P, _I64, _I64, ctypes.POINTER(ctypes.c_size_t)])
tikh_set_workspace = _sig("tikh_set_workspace", [_P, ctypes.c_size_t])
tikh_fft_batched = _sig("tikh_fft_batched", [_P, _I64, _I64, _I64, ctypes.c_int])
tikh_autotune_nlim = _sig("tikh_autotune_nlim", [_I64, _I64, _I64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_double)])
_sig("tikh_profile_kernel", [ctypes.c_char_p])
_sig("tikh_profile_read", [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)])
_sig("tikh_profile_units", [ctypes.POINTER(ctypes.c_double)])
_sig("tikh_set_stream", [_P])
_sig("tikh_set_options", [ctypes.POINTER(_Opts)])
_sig("tikh_get_options", [ctypes.POINTER(_Opts)])
_sig("tikh_get_stats", [ctypes.POINTER(_Stats)])
_sig("tikh_strerror", [ctypes.c_int], ctypes.c_char_p)
tikh_toeplitz_solve = _sig("tikh_toeplitz_solve", [_P, _P, _I64, _I64, _P, _D, _P])
tikh_toeplitz_solve_z = _sig("tikh_toeplitz_solve_z", [_P, _P, _I64, _I64, _P, _D, _P])
tikh_toeplitz_solve_normal = _sig("tikh_toeplitz_solve_normal", [_P, _P, _I64, _I64, _P, _D, _P])
tikh_toeplitz_solve_normal_z = _sig("tikh_toeplitz_solve_normal_z", [_P, _P, _I64, _I64, _P, _D, _P])
tikh_toeplitz_solve_batched = _sig("tikh_toeplitz_solve_batched",
                                   [_I64, _P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, ctypes.c_int])
tikh_toeplitz_solve_batched_noalloc = _sig("tikh_toeplitz_solve_batched_noalloc",
                                           [_I64, _P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, ctypes.c_int])
tikh_gramian_solve = _sig("tikh_gramian_solve", [_P, _P, _P, _I64, _I64, _P, _P])
tikh_gramian_solve_z = _sig("tikh_gramian_solve_z", [_P, _P, _P, _I64, _I64, _P, _P])
tikh_gramian_solve_batched = _sig("tikh_gramian_solve_batched",
                                  [_I64, _P, _P, _P, _P, _P, _I64, _P, _P, _P, ctypes.c_int])
tikh_toeplitz_solve_backward = _sig("tikh_toeplitz_solve_backward",
                                    [_P, _P, _I64, _I64, _P, _D, _P, _P, _P, _P, _P, _P])
tikh_toeplitz_solve_backward_z = _sig("tikh_toeplitz_solve_backward_z",
                                      [_P, _P, _I64, _I64, _P, _D, _P, _P, _P, _P, _P, _P])
tikh_toeplitz_solve_backward_batched = _sig("tikh_toeplitz_solve_backward_batched",
                                            [_I64, _P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P,
                                             _P, ctypes.c_int])
tikh_prepare_batched = _sig("tikh_prepare_batched", [_I64, _P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, ctypes.c_int,
                                                     ctypes.POINTER(ctypes.c_void_p)])
tikh_prepare_backward_batched = _sig("tikh_prepare_backward_batched",
                                     [_I64, _P, _P, _P, _P, _I64, _P, _I64, _P, _P, _P, _P, _P, _P, _P, _P,
                                      ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)])
tikh_prepared_run = _sig("tikh_prepared_run", [_P])
tikh_prepared_workspace = _sig("tikh_prepared_workspace", [_P, ctypes.POINTER(ctypes.c_size_t)])
tikh_prepared_free = _sig("tikh_prepared_free", [_P])


class TikhError(RuntimeError):
    def __init__(self, code, where):
        msg = lib.tikh_strerror(code).decode()
        super().__init__("%s failed: %s (code %d)" % (where, msg, code))
        self.code = code


def _check(code, where):
    if code != 0:
        raise TikhError(code, where)


def _stream():
    lib.tikh_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def set_options(n_lim=None, refine=None, refine_max=None, refine_tol=None, defer_tol=None,
                leaf_wave_groups=None, record_short=None, streams=None, merge_tol=None, fallback_nlim=None,
                chunk_groups=None, refine_skip=None):
    """Leaf cutoff, refinement steps for every solve, most refinement steps for a solve whose
    estimated error is above the target (see tikh_opts in include/tikh.h)."""
    o = _Opts()
    _check(lib.tikh_get_options(ctypes.byref(o)), "tikh_get_options")
    if n_lim is not None:
        o.n_lim = int(n_lim)
    if refine is not None:
        o.refine = int(refine)
    if refine_max is not None:
        o.refine_max = int(refine_max)
    if refine_tol is not None:
        o.refine_tol = float(refine_tol)
    if defer_tol is not None:
        o.defer_tol = float(defer_tol)
    if leaf_wave_groups is not None:
        o.leaf_wave_groups = int(leaf_wave_groups)
    if record_short is not None:
        o.record_short = int(record_short)
    if streams is not None:
        o.streams = int(streams)
    if merge_tol is not None:
        o.merge_tol = float(merge_tol)
    if fallback_nlim is not None:
        o.fallback_nlim = int(fallback_nlim)
    if chunk_groups is not None:
        o.chunk_groups = int(chunk_groups)
    if refine_skip is not None:
        o.refine_skip = int(refine_skip)
    _check(lib.tikh_set_options(ctypes.byref(o)), "tikh_set_options")


def get_options():
    o = _Opts()
    _check(lib.tikh_get_options(ctypes.byref(o)), "tikh_get_options")
    return dict(n_lim=o.n_lim, refine=o.refine, refine_max=o.refine_max, refine_tol=o.refine_tol,
                defer_tol=o.defer_tol, leaf_wave_groups=o.leaf_wave_groups, record_short=o.record_short,
                streams=o.streams, merge_tol=o.merge_tol, fallback_nlim=o.fallback_nlim,
                chunk_groups=o.chunk_groups, refine_skip=o.refine_skip)


def plan_info(m, n, n_lim=256):
    """(N, M, depth, k) of the extension plan (host-only, Alg. 2)."""
    N = ctypes.c_int64(); M = ctypes.c_int64(); p = ctypes.c_int32(); k = ctypes.c_int64()
    _check(tikh_plan_info(int(m), int(n), int(n_lim), ctypes.byref(N), ctypes.byref(M), ctypes.byref(p),
                          ctypes.byref(k)), "tikh_plan_info")
    return N.value, M.value, p.value, k.value


def profile_kernel(name):
    """Time every launch of one kernel kind with HIP events (None disables)."""
    _check(lib.tikh_profile_kernel(name.encode() if name else None), "tikh_profile_kernel")


def profile_read():
    """(total_ms, launches, algorithmic units) of the profiled kernel since profile_kernel()."""
    t = ctypes.c_double(); c = ctypes.c_int64(); u = ctypes.c_double()
    _check(lib.tikh_profile_read(ctypes.byref(t), ctypes.byref(c)), "tikh_profile_read")
    _check(lib.tikh_profile_units(ctypes.byref(u)), "tikh_profile_units")
    return t.value, c.value, u.value


def get_stats():
    s = _Stats()
    _check(lib.tikh_get_stats(ctypes.byref(s)), "tikh_get_stats")
    return dict(N=s.N, k=s.k, depth=s.depth, leaf_nodes=s.leaf_nodes, solves=s.solves, launches=s.launches,
                refine_extra=s.refine_extra, deferred=s.deferred, host_syncs=s.host_syncs,
                fallback_groups=s.fallback_groups, refine_skipped=s.refine_skipped)


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a HIP device tensor")
    if t.dtype != dtype:
        raise TypeError("expected dtype %s, got %s" % (dtype, t.dtype))
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dtype_of(*ts):
    return torch.complex128 if any(t.is_complex() for t in ts) else torch.float64


def fft_batched(x, sign=-1):
    """In-place batched FFT of a complex128 device tensor of shape (items, lines, len) along the last
    axis: X_k = sum_j x_j exp(sign 2 pi i j k / len), unnormalized.  Returns x."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != torch.complex128 or x.dim() != 3:
        raise TypeError("expected a complex128 HIP device tensor of shape (items, lines, len)")
    if not x.is_contiguous():
        raise ValueError("fft_batched works in place on a contiguous tensor")
    _stream()
    _check(tikh_fft_batched(_ptr(x), x.shape[0], x.shape[1], x.shape[2], int(sign)), "tikh_fft_batched")
    return x


def autotune_nlim(m, n, groups=64, nrhs=4):
    """Time one batched solve of an m x n synthetic problem for each leaf cutoff in
    (64, 128, 192, 256), keep the fastest in the options; returns (best, {cutoff: ms})."""
    _stream()
    best = ctypes.c_int32()
    ms = (ctypes.c_double * 4)()
    _check(tikh_autotune_nlim(int(m), int(n), int(groups), int(nrhs), ctypes.byref(best), ms), "tikh_autotune_nlim")
    return best.value, {c: ms[i] for i, c in enumerate((64, 128, 192, 256)) if ms[i] >= 0}


def solve(col, row, b, lam):
    """x = argmin ||T x - b||^2 + lam^2 ||x||^2 on the GPU (tikh_toeplitz_solve[_z])."""
    dt = _dtype_of(col, row, b)
    col, row, b = _dev(col.to(dt), dt), _dev(row.to(dt), dt), _dev(b.to(dt), dt)
    m, n = col.numel(), row.numel()
    x = torch.empty(n, dtype=dt, device=col.device)
    _stream()
    f = tikh_toeplitz_solve_z if dt == torch.complex128 else tikh_toeplitz_solve
    _check(f(_ptr(col), _ptr(row), m, n, _ptr(b), float(lam), _ptr(x)), f.__name__)
    return x


def solve_normal(col, row, y, lam):
    """x = (T^H T + lam^2 I)^{-1} y on the GPU (tikh_toeplitz_solve_normal[_z])."""
    dt = _dtype_of(col, row, y)
    col, row, y = _dev(col.to(dt), dt), _dev(row.to(dt), dt), _dev(y.to(dt), dt)
    m, n = col.numel(), row.numel()
    x = torch.empty(n, dtype=dt, device=col.device)
    _stream()
    f = tikh_toeplitz_solve_normal_z if dt == torch.complex128 else tikh_toeplitz_solve_normal
    _check(f(_ptr(col), _ptr(row), m, n, _ptr(y), float(lam), _ptr(x)), f.__name__)
    return x


def _i64(vals):
    arr = (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])
    return arr


def workspace_bytes(ms, ns, nlam, nrhs):
    """Bytes of workspace with which a batched solve or backward of these shapes runs in
    one chunk (tikh_workspace_bytes; host only)."""
    out = ctypes.c_size_t()
    _check(tikh_workspace_bytes(len(ms), _i64(ms), _i64(ns), int(nlam), int(nrhs), ctypes.byref(out)),
           "tikh_workspace_bytes")
    return out.value


_workspace_ref = None


def set_workspace(buf=None):
    """Hand the library a caller-owned device buffer (a CUDA tensor, kept referenced here
    until replaced) as its workspace, or None to return to the library's own."""
    global _workspace_ref
    if buf is None:
        _check(tikh_set_workspace(None, 0), "tikh_set_workspace")
        _workspace_ref = None
        return
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("workspace must be a contiguous device tensor")
    _check(tikh_set_workspace(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()),
           "tikh_set_workspace")
    _workspace_ref = buf


def solve_batched(ms, ns, col, row, lambdas, nrhs, b, complex_data=False, info=None, x=None):
    """Packed batched solve (tikh_toeplitz_solve_batched).  col/row/b are packed
    device tensors; lambdas is a host sequence of nprob*nlam values.  Returns
    (x, info) tensors; asynchronous on the current stream."""
    dt = torch.complex128 if complex_data else torch.float64
    nprob = len(ms)
    nlam = len(lambdas) // max(nprob, 1)
    assert nlam * nprob == len(lambdas)
    col, row, b = _dev(col, dt), _dev(row, dt), _dev(b, dt)
    xn = sum(nlam * nrhs * int(n) for n in ns)
    if x is None:
        x = torch.empty(xn, dtype=dt, device=col.device)
    if info is None:
        info = torch.zeros(nprob * nlam * nrhs, dtype=torch.int32, device=col.device)
    lam_arr = (ctypes.c_double * len(lambdas))(*[float(v) for v in lambdas])
    _stream()
    _check(tikh_toeplitz_solve_batched(nprob, _i64(ms), _i64(ns), _ptr(col), _ptr(row), nlam, lam_arr, int(nrhs),
                                       _ptr(b), _ptr(x), _ptr(info), 1 if complex_data else 0),
           "tikh_toeplitz_solve_batched")
    return x, info


def solve_batched_noalloc(ms, ns, col, row, lambdas, nrhs, b, x, info, complex_data=False):
    """Allocation-free batched solve (tikh_toeplitz_solve_batched_noalloc): like solve_batched,
    with the outputs x and info supplied by the caller; the library allocates nothing."""
    dt = torch.complex128 if complex_data else torch.float64
    nprob = len(ms)
    nlam = len(lambdas) // max(nprob, 1)
    assert nlam * nprob == len(lambdas)
    col, row, b = _dev(col, dt), _dev(row, dt), _dev(b, dt)
    assert x.dtype == dt and x.is_contiguous() and x.numel() == sum(nlam * nrhs * int(n) for n in ns)
    assert info.dtype == torch.int32 and info.is_contiguous() and info.numel() == nprob * nlam * nrhs
    lam_arr = (ctypes.c_double * len(lambdas))(*[float(v) for v in lambdas])
    _stream()
    _check(tikh_toeplitz_solve_batched_noalloc(nprob, _i64(ms), _i64(ns), _ptr(col), _ptr(row), nlam, lam_arr,
                                               int(nrhs), _ptr(b), _ptr(x), _ptr(info), 1 if complex_data else 0),
           "tikh_toeplitz_solve_batched_noalloc")
    return x, info


def gramian_solve(gram, lcol, lrow, y):
    """Toeplitz-Gramian problem x = (G + L^H L)^{-1} y (tikh_gramian_solve[_z]); G Hermitian
    Toeplitz with first column gram, L Toeplitz (lcol, lrow).  Synchronizes."""
    dt = _dtype_of(gram, lcol, lrow, y)
    gram, lcol, lrow, y = (_dev(t.to(dt), dt) for t in (gram, lcol, lrow, y))
    x = torch.empty_like(y)
    fn = tikh_gramian_solve_z if dt == torch.complex128 else tikh_gramian_solve
    _stream()
    _check(fn(_ptr(gram), _ptr(lcol), _ptr(lrow), lcol.numel(), gram.numel(), _ptr(y), _ptr(x)), "tikh_gramian_solve")
    return x


def gramian_solve_batched(ps, ns, gram, lcol, lrow, nrhs, y, complex_data=False):
    """Packed batched Toeplitz-Gramian solves (tikh_gramian_solve_batched); returns (x, info),
    asynchronous on the current stream."""
    dt = torch.complex128 if complex_data else torch.float64
    gram, lcol, lrow, y = _dev(gram, dt), _dev(lcol, dt), _dev(lrow, dt), _dev(y, dt)
    x = torch.empty_like(y)
    info = torch.zeros(len(ps) * nrhs, dtype=torch.int32, device=y.device)
    _stream()
    _check(tikh_gramian_solve_batched(len(ps), _i64(ps), _i64(ns), _ptr(gram), _ptr(lcol), _ptr(lrow), int(nrhs),
                                      _ptr(y), _ptr(x), _ptr(info), 1 if complex_data else 0),
           "tikh_gramian_solve_batched")
    return x, info


def backward(col, row, b, lam, x, gx):
    """Adjoint of solve: returns (g_col, g_row, g_b, g_lam) (tikh_toeplitz_solve_backward[_z])."""
    dt = _dtype_of(col, row, b, x, gx)
    col, row, b, x, gx = [_dev(t.to(dt), dt) for t in (col, row, b, x, gx)]
    m, n = col.numel(), row.numel()
    g_col = torch.empty(m, dtype=dt, device=col.device)
    g_row = torch.empty(n, dtype=dt, device=col.device)
    g_b = torch.empty(m, dtype=dt, device=col.device)
    g_lam = torch.empty(1, dtype=torch.float64, device=col.device)
    _stream()
    f = tikh_toeplitz_solve_backward_z if dt == torch.complex128 else tikh_toeplitz_solve_backward
    _check(f(_ptr(col), _ptr(row), m, n, _ptr(b), float(lam), _ptr(x), _ptr(gx), _ptr(g_col), _ptr(g_row),
             _ptr(g_b), _ptr(g_lam)), f.__name__)
    return g_col, g_row, g_b, g_lam[0]


def backward_batched(ms, ns, col, row, lambdas, nrhs, b, x, gx, complex_data=False):
    """Packed batched backward (tikh_toeplitz_solve_backward_batched); asynchronous."""
    dt = torch.complex128 if complex_data else torch.float64
    nprob = len(ms)
    nlam = len(lambdas) // max(nprob, 1)
    col, row, b, x, gx = [_dev(t, dt) for t in (col, row, b, x, gx)]
    nsol = nprob * nlam * nrhs
    g_col = torch.empty(sum(nlam * nrhs * int(m) for m in ms), dtype=dt, device=col.device)
    g_row = torch.empty(sum(nlam * nrhs * int(n) for n in ns), dtype=dt, device=col.device)
    g_b = torch.empty(sum(nlam * nrhs * int(m) for m in ms), dtype=dt, device=col.device)
    g_lam = torch.empty(nsol, dtype=torch.float64, device=col.device)
    info = torch.zeros(nsol, dtype=torch.int32, device=col.device)
    lam_arr = (ctypes.c_double * len(lambdas))(*[float(v) for v in lambdas])
    _stream()
    _check(tikh_toeplitz_solve_backward_batched(nprob, _i64(ms), _i64(ns), _ptr(col), _ptr(row), nlam, lam_arr,
                                                int(nrhs), _ptr(b), _ptr(x), _ptr(gx), _ptr(g_col), _ptr(g_row),
                                                _ptr(g_b), _ptr(g_lam), _ptr(info), 1 if complex_data else 0),
           "tikh_toeplitz_solve_backward_batched")
    return g_col, g_row, g_b, g_lam, info


class PreparedBatch:
    """A prepared batch (tikh_prepare_batched / tikh_prepare_backward_batched): the batch's
    plan, workspace and recorded transform lengths are fixed once; run() enqueues it on the
    current stream with kernel launches only, so it can be captured into a CUDA/HIP graph
    (torch.cuda.graph).  The lambdas are read from the device tensor `lam` at every run.
    The tensors passed in are kept referenced for the handle's lifetime; the outputs are
    the attributes x/info (forward) or g_col/g_row/g_b/g_lam/info (backward)."""

    def __init__(self, handle, keep, outputs):
        self._h = handle
        self._keep = keep
        for k, v in outputs.items():
            setattr(self, k, v)

    def run(self):
        if self._h is None:
            raise TikhError(-1, "tikh_prepared_run (freed handle)")
        _stream()
        _check(tikh_prepared_run(self._h), "tikh_prepared_run")

    def workspace_bytes(self):
        out = ctypes.c_size_t()
        _check(tikh_prepared_workspace(self._h, ctypes.byref(out)), "tikh_prepared_workspace")
        return out.value

    def free(self):
        if self._h is not None:
            tikh_prepared_free(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _lam_dev(lam, nvals):
    if not isinstance(lam, torch.Tensor) or not lam.is_cuda or lam.dtype != torch.float64 or not lam.is_contiguous():
        raise TypeError("expected a contiguous float64 HIP device tensor of lambdas")
    if lam.numel() != nvals:
        raise ValueError("expected %d lambdas, got %d" % (nvals, lam.numel()))
    return lam


def prepare_batched(ms, ns, col, row, lam, nrhs, b, complex_data=False):
    """Prepared forward batch: like solve_batched, with the lambdas in the device tensor
    `lam` [nprob*nlam].  Runs the batch once (synchronously); returns a PreparedBatch whose
    x/info hold the results of every run."""
    dt = torch.complex128 if complex_data else torch.float64
    nprob = len(ms)
    nlam = lam.numel() // max(nprob, 1)
    lam = _lam_dev(lam, nprob * nlam)
    col, row, b = _dev(col, dt), _dev(row, dt), _dev(b, dt)
    x = torch.empty(sum(nlam * nrhs * int(n) for n in ns), dtype=dt, device=col.device)
    info = torch.zeros(nprob * nlam * nrhs, dtype=torch.int32, device=col.device)
    h = ctypes.c_void_p()
    mm, nn = _i64(ms), _i64(ns)
    _stream()
    _check(tikh_prepare_batched(nprob, mm, nn, _ptr(col), _ptr(row), nlam, _ptr(lam), int(nrhs), _ptr(b), _ptr(x),
                                _ptr(info), 1 if complex_data else 0, ctypes.byref(h)), "tikh_prepare_batched")
    return PreparedBatch(h, (col, row, b, lam, mm, nn), dict(x=x, info=info))


def prepare_backward_batched(ms, ns, col, row, lam, nrhs, b, x, gx, complex_data=False):
    """Prepared backward batch: like backward_batched, with the lambdas in the device tensor
    `lam`; x and gx are read at every run (the caller updates them in place)."""
    dt = torch.complex128 if complex_data else torch.float64
    nprob = len(ms)
    nlam = lam.numel() // max(nprob, 1)
    lam = _lam_dev(lam, nprob * nlam)
    col, row, b = _dev(col, dt), _dev(row, dt), _dev(b, dt)
    for t in (x, gx):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
            raise TypeError("x and gx must be contiguous device tensors of the batch's dtype (kept in place)")
    nsol = nprob * nlam * nrhs
    g_col = torch.empty(sum(nlam * nrhs * int(m) for m in ms), dtype=dt, device=col.device)
    g_row = torch.empty(sum(nlam * nrhs * int(n) for n in ns), dtype=dt, device=col.device)
    g_b = torch.empty(sum(nlam * nrhs * int(m) for m in ms), dtype=dt, device=col.device)
    g_lam = torch.empty(nsol, dtype=torch.float64, device=col.device)
    info = torch.zeros(nsol, dtype=torch.int32, device=col.device)
    h = ctypes.c_void_p()
    mm, nn = _i64(ms), _i64(ns)
    _stream()
    _check(tikh_prepare_backward_batched(nprob, mm, nn, _ptr(col), _ptr(row), nlam, _ptr(lam), int(nrhs), _ptr(b),
                                         _ptr(x), _ptr(gx), _ptr(g_col), _ptr(g_row), _ptr(g_b), _ptr(g_lam),
                                         _ptr(info), 1 if complex_data else 0, ctypes.byref(h)),
           "tikh_prepare_backward_batched")
    return PreparedBatch(h, (col, row, b, lam, x, gx, mm, nn), dict(g_col=g_col, g_row=g_row, g_b=g_b, g_lam=g_lam,
                                                                   info=info))
