"""Python binding of libmpcare (argument marshalling only).

Dense matrices are torch float64 CUDA tensors of shape (rows, cols) in
COLUMN-major storage (stride (1, ld)); `colmajor()` converts.  Sparse A is a
`DeviceCSR` (CSR of A itself, int32 indices, float64 values).  Every call goes
through the C ABI of include/mpcare.h; nothing here computes.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import (CARE_AUTO, CARE_BF16_SPMM, CARE_FP16_SPMM, CARE_FP32, CARE_FP64, care_csr, care_opts,  # noqa: F401
                   care_shift, care_stats)

PREC = {"fp64": CARE_FP64, "fp32": CARE_FP32, "bf16": CARE_BF16_SPMM, "fp16": CARE_FP16_SPMM, "auto": CARE_AUTO,
        CARE_FP64: CARE_FP64, CARE_FP32: CARE_FP32, CARE_BF16_SPMM: CARE_BF16_SPMM, CARE_FP16_SPMM: CARE_FP16_SPMM,
        CARE_AUTO: CARE_AUTO}


class CareError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.name = L.STATUS_NAMES.get(status, str(status))


def _lib():
    return L.load()


def _check(st):
    if st < 0:
        raise CareError(st, _lib().care_last_error().decode())
    return st


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def colmajor(t: torch.Tensor) -> torch.Tensor:
    """Same values, column-major storage (stride (1, rows))."""
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.stride(0) == 1 and t.stride(1) >= max(t.shape[0], 1):
        return t
    return t.t().contiguous().t()


def tight(t: torch.Tensor) -> torch.Tensor:
    """Column-major copy with leading dimension exactly rows."""
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    return t.t().contiguous().t()


def empty_colmajor(rows, cols, device, dtype=torch.float64):
    return torch.empty((max(cols, 1), rows), device=device, dtype=dtype).t()[:, :cols]


def _ld(t):
    return max(t.stride(1), t.shape[0], 1) if t.dim() == 2 else max(t.shape[0], 1)


class DeviceCSR:
    """CSR of A on the GPU (the caller's buffers, passed to the ABI as-is)."""

    def __init__(self, row_ptr, col_idx, val, n):
        self.row_ptr, self.col_idx, self.val, self.n = row_ptr, col_idx, val, int(n)
        self.nnz = int(col_idx.numel())
        self._c = care_csr(self.n, self.nnz, row_ptr.data_ptr(), col_idx.data_ptr(), val.data_ptr())

    @classmethod
    def from_scipy(cls, A, device="cuda"):
        A = A.tocsr()
        A.sort_indices()
        return cls(torch.as_tensor(A.indptr.astype(np.int32), device=device),
                   torch.as_tensor(A.indices.astype(np.int32), device=device),
                   torch.as_tensor(A.data.astype(np.float64), device=device), A.shape[0])

    @property
    def c(self):
        return C.byref(self._c)


class TorchAllocator:
    """Device-memory hooks that draw the library's workspace from PyTorch's
    caching allocator (torch.cuda.caching_allocator_alloc / _delete), so the
    library and torch share one pool.  Counts the calls (for tests)."""

    def __init__(self, device: int):
        self.device = device
        self.allocs = 0
        self.frees = 0
        self.live = {}

        def alloc(nbytes, stream, user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0))
            except Exception:      # out of memory: the library reports CARE_ERR_NOMEM
                return None
            self.allocs += 1
            self.live[ptr] = int(nbytes)
            return ptr

        def dealloc(ptr, nbytes, stream, user):
            self.frees += 1
            self.live.pop(ptr, None)
            torch.cuda.caching_allocator_delete(ptr)

        # the ctypes callback objects must outlive the context
        self.c_alloc = L.ALLOC_FN(alloc)
        self.c_dealloc = L.DEALLOC_FN(dealloc)


class Context:
    """A library context bound to one device and one HIP stream (torch's
    current stream by default).  allocator="torch" (default) backs the
    library's device workspace with PyTorch's caching allocator through the
    context's allocator hooks; allocator=None lets the library use hipMalloc."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, allocator: str | None = "torch"):
        self.device = device
        self.stream = stream or torch.cuda.current_stream(device)
        self.allocator = TorchAllocator(device) if allocator == "torch" else None
        if allocator not in ("torch", None):
            raise ValueError(f"unknown allocator {allocator!r}")
        h = C.c_void_p()
        if self.allocator is not None:
            _check(_lib().care_ctx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream),
                                          self.allocator.c_alloc, self.allocator.c_dealloc, None))
        else:
            _check(_lib().care_ctx_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream),
                                          L.ALLOC_FN(), L.DEALLOC_FN(), None))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            _lib().care_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def default_opts(prec="fp64", **kw) -> care_opts:
    o = care_opts()
    _lib().care_opts_default(C.byref(o), PREC[prec])
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _shift(p) -> care_shift:
    p = complex(p)
    return care_shift(p.real, p.imag)


def _shift_array(shifts):
    s = list(shifts)
    arr = (care_shift * max(len(s), 1))()
    for i, p in enumerate(s):
        arr[i] = _shift(p)
    return arr, len(s)


def version():
    return _lib().care_version().decode()


def spmm(ctx: Context, A: DeviceCSR, X: torch.Tensor, shift=0.0, prec="fp64") -> torch.Tensor:
    """Y = (A^T + p I) X (complex p: X, Y hold [Re | Im] blocks)."""
    X = colmajor(X)
    k = X.shape[1] // 2 if complex(shift).imag != 0 else X.shape[1]
    Y = empty_colmajor(A.n, X.shape[1], X.device)
    _check(_lib().care_spmm(ctx.h, A.c, PREC[prec], _shift(shift), _ptr(X), _ld(X), k, _ptr(Y), _ld(Y)))
    return Y


def spmm_timing(ctx: Context, A: DeviceCSR, k: int, shift=0.0, prec="fp32", nsets=4, reps=5, panel=0, pg=0):
    """Mean microseconds per product Y = (A^T + p I) X over `nsets` rotated
    operator / panel sets, and the algorithmic bytes of one product."""
    us, nb = C.c_double(0), C.c_double(0)
    _check(_lib().care_spmm_timing(ctx.h, A.c, PREC[prec], _shift(shift), k, nsets, reps, panel, pg, C.byref(us),
                                   C.byref(nb)))
    return us.value, nb.value


def gram(ctx, X, Y):
    """C = X^T Y (FP64 matrix cores).  Passing the same tensor twice gives an
    exactly symmetric X^T X."""
    same = X is Y
    X = colmajor(X)
    Y = X if same else colmajor(Y)
    C_ = empty_colmajor(X.shape[1], Y.shape[1], X.device)
    _check(_lib().care_gram(ctx.h, X.shape[0], _ptr(X), _ld(X), X.shape[1], _ptr(Y), _ld(Y), Y.shape[1], _ptr(C_),
                            _ld(C_)))
    return C_


def gram_noalloc(ctx, X, Y, C_=None):
    """C = X^T Y through the allocation-free entry point (the library's own
    MFMA kernel, partials in its fixed device array).  C_ (a x b, column-major
    FP64) may be passed in, so that the call itself allocates nothing."""
    X = colmajor(X)
    Y = colmajor(Y)
    if C_ is None:
        C_ = empty_colmajor(X.shape[1], Y.shape[1], X.device)
    _check(_lib().care_gram_noalloc(ctx.h, X.shape[0], _ptr(X), _ld(X), X.shape[1], _ptr(Y), _ld(Y), Y.shape[1],
                                    _ptr(C_), _ld(C_)))
    return C_


def tsgemm(ctx, X, S, alpha=1.0, beta=0.0, Y=None):
    """Y = alpha X S + beta Y (FP64 matrix cores)."""
    X, S = colmajor(X), colmajor(S)
    if Y is None:
        Y = empty_colmajor(X.shape[0], S.shape[1], X.device)
    else:
        Y = colmajor(Y)
    _check(_lib().care_tsgemm(ctx.h, X.shape[0], _ptr(X), _ld(X), X.shape[1], _ptr(S), _ld(S), S.shape[1], alpha,
                              beta, _ptr(Y), _ld(Y)))
    return Y


def shifted_solve(ctx, A, W, shift, B=None, K=None, prec="fp64", tol=0.0, maxit=0, opts=None):
    """V = (A_k^T + p I)^{-1} W with A_k = A - B K^T (SMW); complex p returns [Re | Im].
    opts (care_opts, optional) selects the Krylov method (krylov_method,
    krylov_restart, krylov_compact, krylov_rb, krylov_precond)."""
    W = colmajor(W)
    w = W.shape[1]
    m = 0 if K is None else K.shape[1]
    B = colmajor(B) if B is not None else None
    K = colmajor(K) if K is not None else None
    vc = 2 * w if complex(shift).imag != 0 else w
    V = empty_colmajor(A.n, vc, W.device)
    it = C.c_int32(0)
    args = (ctx.h, A.c, _ptr(B), _ld(B) if B is not None else A.n, _ptr(K), _ld(K) if K is not None else A.n, m,
            _shift(shift), _ptr(W), _ld(W), w, PREC[prec], tol, maxit)
    if opts is None:
        st = _check(_lib().care_shifted_solve(*args, _ptr(V), _ld(V), C.byref(it)))
    else:
        st = _check(_lib().care_shifted_solve_opts(*args, C.byref(opts), _ptr(V), _ld(V), C.byref(it)))
    return V, dict(status=st, iters=it.value)


def ilu0_factor(ctx, A, shift, prec="fp64"):
    """ILU(0) of A^T + p I in the library's multicolour order: returns
    (colours, off, udiag) as numpy arrays (off at A^T's off-diagonal nonzeros
    in row-major order)."""
    rows = torch.repeat_interleave(torch.arange(A.n, device=A.row_ptr.device),
                                   (A.row_ptr[1:] - A.row_ptr[:-1]).long())
    noff = A.nnz - int((A.col_idx.long() == rows).sum().item())
    colours = np.zeros(A.n, dtype=np.int32)
    off = np.zeros(max(noff, 1), dtype=np.float64)
    udiag = np.zeros(A.n, dtype=np.float64)
    _check(_lib().care_ilu0_factor(ctx.h, A.c, PREC[prec], float(shift),
                                   colours.ctypes.data_as(C.POINTER(C.c_int32)),
                                   off.ctypes.data_as(C.POINTER(C.c_double)), noff,
                                   udiag.ctypes.data_as(C.POINTER(C.c_double))))
    return colours, off[:noff], udiag


def ilu0_colouring(A):
    """The library's first-fit colouring of a host sparse matrix's pattern
    (host-only call, no device): returns (colours, number of colours)."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    rp = np.ascontiguousarray(A.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.indices, dtype=np.int32)
    colours = np.zeros(A.shape[0], dtype=np.int32)
    nc = C.c_int32(0)
    p32 = C.POINTER(C.c_int32)
    _check(_lib().care_ilu0_colouring(A.shape[0], A.nnz, rp.ctypes.data_as(p32), ci.ctypes.data_as(p32),
                                      colours.ctypes.data_as(p32), C.byref(nc)))
    return colours, nc.value


def ilu0_apply(ctx, A, X, shift, prec="fp64"):
    """Z = (L U)^{-1} X with the ILU(0) factors of A^T + p I."""
    X = colmajor(X)
    Z = empty_colmajor(A.n, X.shape[1], X.device)
    _check(_lib().care_ilu0_apply(ctx.h, A.c, PREC[prec], float(shift), _ptr(X), _ld(X), X.shape[1], _ptr(Z),
                                  _ld(Z)))
    return Z


def lyap_lradi(ctx, A, W, shifts, B=None, K=None, tol=0.0, opts=None, rmax=None):
    """LR-ADI for A_k^T X + X A_k + W W^T = 0; returns (Z, stats, status)."""
    W = colmajor(W)
    n, w = W.shape
    m = 0 if K is None else K.shape[1]
    Bc = tight(B) if B is not None else None            # the ABI takes B, K with ld = n
    Kc = tight(K) if K is not None else None
    opts = opts or default_opts()
    rmax = rmax or w * (opts.j_max + 2)
    Z = empty_colmajor(n, rmax, W.device)
    r = C.c_int32(0)
    stats = care_stats()
    arr, ns = _shift_array(shifts)
    st = _check(_lib().lyap_lradi(ctx.h, A.c, _ptr(Bc), _ptr(Kc), m, _ptr(W), _ld(W), w, arr, ns, tol,
                                  C.byref(opts), _ptr(Z), _ld(Z), rmax, C.byref(r), C.byref(stats)))
    return Z[:, :r.value], stats.to_dict(), st


def residual_factor(ctx, A, B, C_, Z, eta_r_rel=1e-4, cap=None):
    """Algorithm 1: returns (C+, C-, ||R||_F)."""
    n = A.n
    Bc = tight(B) if B is not None and B.shape[1] else None
    Cr = C_.contiguous()                                    # p x n row-major
    Z = colmajor(Z)
    r = Z.shape[1]
    p = Cr.shape[0]
    m = 0 if Bc is None else Bc.shape[1]
    cap = cap or (2 * r + m + p)
    Cp = empty_colmajor(n, cap, Z.device)
    Cm = empty_colmajor(n, cap, Z.device)
    rp, rm, res = C.c_int32(0), C.c_int32(0), C.c_double(0)
    _check(_lib().care_residual_factor(ctx.h, A.c, _ptr(Bc), m, _ptr(Cr), p, _ptr(Z) if r else None, _ld(Z), r,
                                       eta_r_rel, _ptr(Cp), C.byref(rp), _ptr(Cm), C.byref(rm), _ld(Cp), cap,
                                       C.byref(res)))
    return Cp[:, :rp.value], Cm[:, :rm.value], res.value


def lowrank_truncate(ctx, G, sign, eta_s_rel=1.1102230246251565e-15, cap=None):
    """Algorithm 2 with signature diag(sign): returns (Z, eta_n)."""
    G = colmajor(G)
    n, s = G.shape
    sg = (C.c_int8 * max(s, 1))(*[int(v) for v in sign])
    cap = cap or max(s, 1)
    Z = empty_colmajor(n, cap, G.device)
    r, eta_n = C.c_int32(0), C.c_double(0)
    _check(_lib().lowrank_truncate(ctx.h, n, _ptr(G), _ld(G), s, sg, eta_s_rel, _ptr(Z), _ld(Z), cap, C.byref(r),
                                   C.byref(eta_n)))
    return Z[:, :r.value], eta_n.value


def care_solve(ctx, A, B, C_, tol=1e-10, shifts=None, prec="fp32", opts=None, rmax=None, **kw):
    """Framework 1.  B: n x m, C_: p x n.  Returns (Z, stats dict, status)."""
    B = tight(B)
    Cr = C_.contiguous()
    n, m = B.shape
    p = Cr.shape[0]
    opts = opts or default_opts(prec, **kw)
    rmax = rmax or min(n, 4096)
    Z = empty_colmajor(n, rmax, B.device)
    r = C.c_int32(0)
    stats = care_stats()
    arr, ns = _shift_array(shifts if shifts is not None else [])
    st = _check(_lib().care_solve(ctx.h, A.c, _ptr(B), m, _ptr(Cr), p, tol, arr, ns, C.byref(opts), _ptr(Z),
                                  _ld(Z), rmax, C.byref(r), C.byref(stats)))
    return Z[:, :r.value], stats.to_dict(), st


def care_solve_dense(ctx, A, B, C_, tol=1e-10, shifts=None, prec="fp32", opts=None, rmax=None, **kw):
    """Framework 1 for a dense A (n x n device tensor, FP64).  Returns
    (Z, stats dict, status)."""
    A = colmajor(A.to(torch.float64))
    B = tight(B)
    Cr = C_.contiguous()
    n, m = B.shape
    p = Cr.shape[0]
    opts = opts or default_opts(prec, **kw)
    rmax = rmax or min(n, 4096)
    Z = empty_colmajor(n, rmax, B.device)
    r = C.c_int32(0)
    stats = care_stats()
    arr, ns = _shift_array(shifts if shifts is not None else [])
    st = _check(_lib().care_solve_dense(ctx.h, _ptr(A), n, _ld(A), _ptr(B), m, _ptr(Cr), p, tol, arr, ns,
                                        C.byref(opts), _ptr(Z), _ld(Z), rmax, C.byref(r), C.byref(stats)))
    return Z[:, :r.value], stats.to_dict(), st


def care_solve_batch(ctx, problems, tol=1e-10, prec="fp32", opts=None, rmax=None, workers=0, **kw):
    """Batched Framework 1.  problems: list of (A, B n x m tensor, C p x n
    tensor, shifts or None) with A a DeviceCSR or a dense n x n FP64 device
    tensor.  Returns a list of
    (Z, stats dict, status, message), one per problem; raises CareError only
    for a batch-level failure (use the per-instance status otherwise)."""
    from ._lib import care_instance, care_instance_result
    opts = opts or default_opts(prec, **kw)
    count = len(problems)
    inst = (care_instance * max(count, 1))()
    res = (care_instance_result * max(count, 1))()
    keep = []
    for k, (A, B, Cm, shifts) in enumerate(problems):
        B = tight(B)
        Cr = Cm.contiguous()
        n, m = B.shape
        rk = rmax or min(n, 4096)
        Z = empty_colmajor(n, rk, B.device)
        arr, ns = _shift_array(shifts if shifts is not None else [])
        if isinstance(A, DeviceCSR):
            inst[k].A = C.pointer(A._c)
        else:
            A = colmajor(A.to(torch.float64))
            inst[k].A_dense, inst[k].n_dense, inst[k].lda_dense = A.data_ptr(), A.shape[0], _ld(A)
        keep.append((A, B, Cr, Z, arr))
        inst[k].B, inst[k].m = (B.data_ptr() if m > 0 else None), m
        inst[k].C, inst[k].p = Cr.data_ptr(), Cr.shape[0]
        inst[k].shifts, inst[k].nshifts = (C.cast(arr, C.POINTER(care_shift)) if ns else None), ns
        inst[k].Z, inst[k].ldz, inst[k].rmax = Z.data_ptr(), _ld(Z), rk
    st = _lib().care_solve_batch(ctx.h, count, inst, tol, C.byref(opts), workers, res)
    if st < 0 and all(res[k].status >= 0 for k in range(count)):
        raise CareError(st, _lib().care_last_error().decode())
    out = []
    for k in range(count):
        Z = keep[k][3]
        r = res[k].r if res[k].status >= 0 else 0
        out.append((Z[:, :r], res[k].stats.to_dict(), res[k].status, res[k].message.decode()))
    return out


def penzl_shifts(ctx, A, l0=16, kp=20, km=10, real_only=False):
    """Heuristic shift set from Ritz values of A^T and A^-T (GPU Arnoldi)."""
    out = (care_shift * (l0 + 1))()
    cnt = C.c_int32(0)
    _check(_lib().care_penzl_shifts(ctx.h, A.c, l0, kp, km, 1 if real_only else 0, out, C.byref(cnt)))
    return np.array([complex(out[i].re, out[i].im) for i in range(cnt.value)])


def projection_shifts(ctx, A, V, l0=16, B=None, K=None, prec="fp64"):
    """Projection shifts: Ritz values of A^T - K B^T on span(V) (n x s device
    tensor), mirrored into the left half-plane, at most l0 chosen."""
    V = colmajor(V.to(torch.float64))
    smw = B is not None and K is not None and B.shape[1] > 0
    Bt = tight(B) if smw else None
    Kt = tight(K) if smw else None
    m = Bt.shape[1] if smw else 0
    out = (care_shift * (l0 + 1))()
    cnt = C.c_int32(0)
    _check(_lib().care_projection_shifts(ctx.h, A.c, _ptr(Bt) if smw else None, _ptr(Kt) if smw else None, m,
                                         _ptr(V), _ld(V), V.shape[1], l0, PREC[prec], out, C.byref(cnt)))
    return np.array([complex(out[i].re, out[i].im) for i in range(cnt.value)])


def ritz_values(H):
    """Eigenvalues of a small upper Hessenberg matrix (host, no device work)."""
    H = np.asfortranarray(np.asarray(H, dtype=np.float64))
    k = H.shape[0]
    if H.shape != (k, k):
        raise ValueError("H must be square")
    re = np.zeros(max(k, 1))
    im = np.zeros(max(k, 1))
    dp = C.POINTER(C.c_double)
    _check(_lib().care_ritz_values(H.ctypes.data_as(dp), k, max(k, 1), re.ctypes.data_as(dp),
                                   im.ctypes.data_as(dp)))
    return (re + 1j * im)[:k]


def penzl_select(candidates, l0):
    """Greedy min-max choice of l0 shifts among candidate values (host)."""
    R = np.asarray(candidates, dtype=np.complex128).ravel()
    re = np.ascontiguousarray(R.real)
    im = np.ascontiguousarray(R.imag)
    out = (care_shift * (l0 + 1))()
    cnt = C.c_int32(0)
    dp = C.POINTER(C.c_double)
    _check(_lib().care_penzl_select(re.ctypes.data_as(dp), im.ctypes.data_as(dp), R.size, l0, out,
                                    C.byref(cnt)))
    return np.array([complex(out[i].re, out[i].im) for i in range(cnt.value)])


def shifted_lu_factor(ctx, M0, shifts, prec="fp32"):
    """LU with partial pivoting of M0 + p I for every real p in `shifts`, one
    launch.  M0: n x n on the GPU (cast to prec's type, column-major).
    Returns (F, perm, info): F (nshifts, n, n) holding each factor column-major
    (F[s].T is the n x n matrix of factors in row-major torch indexing), perm
    (nshifts, n) int32 with (P M)[i] = M[perm[i]], and info, a list of 0 or
    the 1-based first zero pivot."""
    code = PREC[prec]
    if code not in (L.CARE_FP32, L.CARE_FP64):
        raise ValueError("prec must be fp32 or fp64")
    dt = torch.float32 if code == L.CARE_FP32 else torch.float64
    n = int(M0.shape[0])
    Mc = colmajor(M0.to(dt))
    if _ld(Mc) != n:
        Mc = Mc.t().contiguous().t()
    sh = np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(-1))
    ns = int(sh.size)
    F = torch.empty((max(ns, 1), n, n), device=M0.device, dtype=dt)
    perm = torch.empty((max(ns, 1), n), device=M0.device, dtype=torch.int32)
    info = (C.c_int32 * max(ns, 1))()
    _check(_lib().care_shifted_lu_factor(ctx.h, code, n, _ptr(Mc), sh.ctypes.data_as(C.POINTER(C.c_double)), ns,
                                         _ptr(F), _ptr(perm), info))
    return F[:ns], perm[:ns], [int(info[i]) for i in range(ns)]


def shifted_lu_solve(ctx, F, perm, Bm, prec="fp32"):
    """X = M^{-1} B with one factor F (n x n storage as returned in
    shifted_lu_factor's F[s]) and its perm; B: n x k on the GPU."""
    code = PREC[prec]
    dt = torch.float32 if code == L.CARE_FP32 else torch.float64
    n = int(F.shape[-1])
    Bc = colmajor(Bm.to(dt))
    X = empty_colmajor(n, Bc.shape[1], Bm.device, dtype=dt)
    _check(_lib().care_shifted_lu_solve(ctx.h, code, n, _ptr(F), _ptr(perm), Bc.shape[1], _ptr(Bc), _ld(Bc),
                                        _ptr(X), _ld(X)))
    return X
