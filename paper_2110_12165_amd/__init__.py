"""Lattice H-matrix products for boundary-element earthquake-sequence models
on AMD Instinct MI355X (gfx950).

Thin Python binding over ``libhmat.so`` (C ABI in ``include/hmat.h``).  All
computation runs in the library's native code: the host construction
(cluster tree, partition, ACA) in C++, the products and the rate-and-state
right-hand side in HIP kernels.  PyTorch provides device memory and streams.
There is no fallback path: if the library is not built, importing the
binding's entry points raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import HmatError, check

__all__ = ["HMatrix", "rs_rhs", "RK45", "HmatError", "library"]


def library():
    return _lib.load()


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def _gpu_f64(t, shape, name, contiguous=True):
    """Raise unless t is a float64 GPU tensor of the given shape (and
    contiguous): its address goes to the device kernels unchecked."""
    torch = _torch()
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and tuple(t.shape) == tuple(shape) and (t.is_contiguous() or not contiguous)):
        raise ValueError(f"{name} must be a {'contiguous ' if contiguous else ''}float64 GPU tensor of shape "
                         f"{tuple(shape)}")


class HMatrix:
    """Handle on a lattice H-matrix held on the current GPU."""

    def __init__(self, handle):
        self._h = handle
        self._lib = _lib.load()
        self._n = None

    # -- construction -------------------------------------------------------
    @staticmethod
    def _opts(aca_eps=1e-6, eta=2.0, leaf=32, lattice=1, max_rank=0, prec="f64", kernel="auto",
              n_threads=0, wg_waves=0, unit_kib=0, wg_waves_p1=0, max_nrhs=0, transpose=1, build_device=0,
              mm_groups=0):
        lib = _lib.load()
        o = _lib.HmatOpts()
        lib.hmat_default_opts(C.byref(o))
        o.aca_eps, o.eta, o.leaf, o.lattice, o.max_rank = aca_eps, eta, leaf, lattice, max_rank
        o.prec = _lib.PREC[prec]
        o.kernel = _lib.KERNEL[kernel]
        o.n_threads, o.wg_waves, o.unit_kib, o.wg_waves_p1 = n_threads, wg_waves, unit_kib, wg_waves_p1
        o.max_nrhs = max_nrhs
        o.transpose = transpose
        o.build_device = build_device
        o.mm_groups = mm_groups
        return o

    @classmethod
    def build(cls, verts, slip_dir, mu, nu, component=0, stream=None, **opts):
        """hmat_build from element vertices (N, 4, 3) (coplanar rectangles) or
        (N, 3, 3) (triangles, any orientation) and slip directions (N, 3).
        component 0: shear tractions (A); 1: normal tractions (B)."""
        lib = _lib.load()
        verts = np.ascontiguousarray(verts, dtype=np.float64)
        slip_dir = np.ascontiguousarray(slip_dir, dtype=np.float64)
        if verts.ndim != 3 or slip_dir.shape != (verts.shape[0], 3):
            raise ValueError("verts must be (N, nvert, 3) and slip_dir (N, 3)")
        mesh = _lib.HmatMesh(verts.shape[0], verts.shape[1],
                             verts.ctypes.data_as(C.POINTER(C.c_double)),
                             slip_dir.ctypes.data_as(C.POINTER(C.c_double)))
        kind = _lib.GF_FS_TRIANGLE if verts.shape[1] == 3 else _lib.GF_FS_RECT_COPLANAR
        green = _lib.HmatGreen(kind, component, mu, nu)
        o = cls._opts(**opts)
        h = C.c_void_p()
        check(lib.hmat_build(C.byref(mesh), C.byref(green), C.byref(o), _stream_ptr(stream), C.byref(h)))
        return cls(h)

    @classmethod
    def from_blocks(cls, n, perm, desc, off, values, stream=None, **opts):
        """hmat_import from host arrays in the hmat_host_blocks layout."""
        lib = _lib.load()
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        desc = np.ascontiguousarray(desc, dtype=np.int64)
        off = np.ascontiguousarray(off, dtype=np.int64)
        values = np.ascontiguousarray(values, dtype=np.float64)
        hb = _lib.HmatHostBlocks(n, off.shape[0], values.shape[0],
                                 perm.ctypes.data_as(C.POINTER(C.c_int32)),
                                 desc.ctypes.data_as(C.POINTER(C.c_int64)),
                                 off.ctypes.data_as(C.POINTER(C.c_int64)),
                                 values.ctypes.data_as(C.POINTER(C.c_double)))
        o = cls._opts(**opts)
        h = C.c_void_p()
        check(lib.hmat_import(C.byref(hb), C.byref(o), _stream_ptr(stream), C.byref(h)))
        return cls(h)

    # -- products -----------------------------------------------------------
    def _apply(self, fn, x, y, alpha, beta, stream):
        torch = _torch()
        n = self.n
        if not (x.is_cuda and x.dtype == torch.float64):
            raise TypeError("x must be a float64 GPU tensor")
        if x.dim() == 1:
            if x.shape[0] != n:
                raise ValueError("x has the wrong length")
            xc = x.contiguous()
            out = torch.empty_like(xc) if y is None else y
            _gpu_f64(out, (n,), "y")
            check(fn(self._h, _dptr(xc), _dptr(out), 1, n, alpha, 0.0 if y is None else beta, _stream_ptr(stream)))
            return out
        if x.dim() != 2 or x.shape[0] != n:
            raise ValueError("x must be (n,) or (n, k)")
        k = x.shape[1]
        if y is not None:
            _gpu_f64(y, (n, k), "y", contiguous=False)
        xt = x.t().contiguous()                       # (k, n): column-major n x k, ld = n
        yt = torch.empty_like(xt) if y is None else y.t().contiguous()
        check(fn(self._h, _dptr(xt), _dptr(yt), k, n, alpha, 0.0 if y is None else beta, _stream_ptr(stream)))
        res = yt.t()
        if y is not None:
            y.copy_(res)
            return y
        return res

    def matvec(self, x, y=None, alpha=1.0, beta=0.0, stream=None):
        """y = alpha H x + beta y (x: float64 GPU tensor (n,) or (n, k))."""
        return self._apply(self._lib.hmat_matvec, x, y, alpha, beta, stream)

    def matvec_T(self, x, y=None, alpha=1.0, beta=0.0, stream=None):
        return self._apply(self._lib.hmat_matvec_T, x, y, alpha, beta, stream)

    def matmat(self, X, Y=None, alpha=1.0, beta=0.0, mode="x6", stream=None):
        """Y = alpha H X + beta Y on MFMA (hmat_matmat).  X: float64 GPU tensor
        (n, k), row-major (element-major: the k members of an element are
        contiguous)."""
        torch = _torch()
        n = self.n
        if not (X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[0] == n):
            raise ValueError("X must be a float64 GPU tensor of shape (n, k)")
        Xc = X.contiguous()
        out = torch.empty_like(Xc) if Y is None else Y
        _gpu_f64(out, Xc.shape, "Y")
        k = Xc.shape[1]
        check(self._lib.hmat_matmat(self._h, _dptr(Xc), k, _dptr(out), k, k, alpha, 0.0 if Y is None else beta,
                                    _lib.MM_MODE[mode], _stream_ptr(stream)))
        return out

    def matvec_raw(self, x_ptr, y_ptr, nrhs=1, ld=None, alpha=1.0, beta=0.0, stream_ptr=None, transpose=False):
        """Direct call with device addresses (no tensor checks)."""
        fn = self._lib.hmat_matvec_T if transpose else self._lib.hmat_matvec
        check(fn(self._h, C.c_void_p(x_ptr), C.c_void_p(y_ptr), nrhs, self.n if ld is None else ld, alpha, beta,
                 C.c_void_p(stream_ptr)))

    # -- inspection ---------------------------------------------------------
    def info(self):
        st = _lib.HmatStats()
        check(self._lib.hmat_info(self._h, C.byref(st)))
        d = {name: getattr(st, name) for name, _ in _lib.HmatStats._fields_}
        d["kernel"] = _lib.KERNEL_NAME.get(d["kernel"], d["kernel"])
        d["prec"] = "f32" if d["prec"] == 1 else "f64"
        g = d.pop("mm_groups")
        d["mm_groups"] = {"x3": ((g >> 0) & 15, (g >> 4) & 15), "x6": ((g >> 8) & 15, (g >> 12) & 15)} if g else None
        return d

    @property
    def n(self):
        if self._n is None:
            self._n = self.info()["n"]
        return self._n

    def export(self):
        """Copies of the FP64 host blocks: dict(n, perm, desc (nb, 6), off, values)."""
        hb = _lib.HmatHostBlocks()
        check(self._lib.hmat_export(self._h, C.byref(hb)))
        n, nb, nv = hb.n, hb.nblocks, hb.nvalues
        return dict(n=n,
                    perm=np.ctypeslib.as_array(hb.perm, shape=(n,)).copy(),
                    desc=np.ctypeslib.as_array(hb.desc, shape=(nb * 6,)).copy().reshape(nb, 6),
                    off=np.ctypeslib.as_array(hb.off, shape=(nb,)).copy(),
                    values=np.ctypeslib.as_array(hb.values, shape=(nv,)).copy() if nv else np.zeros(0))

    def profile(self, x, y, reps=50, stream=None):
        """hmat_profile: per-launch mean durations (ms) and algorithmic bytes."""
        _gpu_f64(x, (self.n,), "x")
        _gpu_f64(y, (self.n,), "y")
        pr = _lib.HmatProfile()
        check(self._lib.hmat_profile(self._h, _dptr(x), _dptr(y), reps, _stream_ptr(stream), C.byref(pr)))
        nl = pr.n_launches
        return dict(n_launches=nl, reps=pr.reps, ms=[pr.ms[i] for i in range(nl)], ms_product=pr.ms_product,
                    alg_bytes=[pr.alg_bytes[i] for i in range(nl)])

    def check(self, stream=None):
        """hmat_check: raise HmatError if a persistent product on this handle
        since the last check gave up (waits for the stream only then)."""
        check(self._lib.hmat_check(self._h, _stream_ptr(stream)))

    def autotune(self, reps=20, stream=None):
        check(self._lib.hmat_autotune(self._h, reps, _stream_ptr(stream)))
        return self.info()

    def close(self):
        if self._h:
            self._lib.hmat_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rs_rhs(A: HMatrix, B, y, a, b, dc, V0, f0, eta_rad, V_pl, dydt=None, V_out=None, stream=None):
    """dy/dt of the 3N rate-and-state ODEs; y = (phi | tau | sigma) float64 GPU tensor."""
    torch = _torch()
    n = A.n
    if y.shape != (3 * n,) or y.dtype != torch.float64 or not y.is_cuda:
        raise ValueError("y must be a float64 GPU tensor of length 3n")
    for t, name in ((a, "a"), (b, "b"), (dc, "dc")):
        _gpu_f64(t, (n,), name)
    y = y.contiguous()
    out = torch.empty_like(y) if dydt is None else dydt
    _gpu_f64(out, (3 * n,), "dydt")
    if V_out is not None:
        _gpu_f64(V_out, (n,), "V_out")
    p = _lib.RsParams(n, V0, f0, eta_rad, V_pl, a.data_ptr(), b.data_ptr(), dc.data_ptr())
    lib = _lib.load()
    check(lib.rs_rhs(A._h, None if B is None else B._h, C.byref(p), _dptr(y), _dptr(out),
                     None if V_out is None else _dptr(V_out), _stream_ptr(stream)))
    return out


class RK45:
    """Adaptive Runge-Kutta 5(4) integration of the rate-and-state ODEs on the
    GPU (rs_rk45_attempt / rs_rk45_step): the stage combinations, the products
    with A (and B), the right-hand side, the error estimate and the slip
    update all run in the library; the step control of eqs. (14)-(15) is
    applied after each attempt."""

    def __init__(self, A, B, a, b, dc, V0, f0, eta_rad, V_pl, eps_rk=1e-4, dt0=1.0):
        torch = _torch()
        self.A, self.B = A, B
        n = A.n
        for t, name in ((a, "a"), (b, "b"), (dc, "dc")):
            _gpu_f64(t, (n,), name)
        self._keep = (a, b, dc)
        self.params = _lib.RsParams(n, V0, f0, eta_rad, V_pl, a.data_ptr(), b.data_ptr(), dc.data_ptr())
        nbytes = _lib.load().rs_rk45_workspace_bytes(n)
        self.workspace = torch.empty(nbytes // 8, dtype=torch.float64, device=a.device)
        self.state = _lib.RsRk45State(0.0, dt0, eps_rk, 0.0, 0, 0)

    def _check(self, y, D):
        n = self.A.n
        _gpu_f64(y, (3 * n,), "y")
        _gpu_f64(D, (n,), "D")

    def attempt(self, y, D, force=-1, stream=None):
        self._check(y, D)
        lib = _lib.load()
        check(lib.rs_rk45_attempt(self.A._h, None if self.B is None else self.B._h, C.byref(self.params),
                                  _dptr(y), _dptr(D), _dptr(self.workspace), C.byref(self.state), force,
                                  _stream_ptr(stream)))
        return self.state.last_err

    def step(self, y, D, max_attempts=64, stream=None):
        self._check(y, D)
        lib = _lib.load()
        check(lib.rs_rk45_step(self.A._h, None if self.B is None else self.B._h, C.byref(self.params),
                               _dptr(y), _dptr(D), _dptr(self.workspace), C.byref(self.state), max_attempts,
                               _stream_ptr(stream)))

    def run(self, y, D, n_accept, max_attempts=0, use_graph=True, stream=None, dt_log=None):
        """Advance n_accept accepted steps with the step control on the GPU
        (rs_rk45_run).  The graph path needs a non-default stream.  dt_log:
        optional float64 GPU tensor of n_accept entries receiving the
        accepted steps (the list replay() and adjoint() take)."""
        self._check(y, D)
        if dt_log is not None and (dt_log.dtype != _torch().float64 or not dt_log.is_cuda
                                   or dt_log.numel() < n_accept or not dt_log.is_contiguous()):
            raise ValueError("dt_log must be a contiguous float64 GPU tensor of at least n_accept entries")
        lib = _lib.load()
        check(lib.rs_rk45_run(self.A._h, None if self.B is None else self.B._h, C.byref(self.params),
                              _dptr(y), _dptr(D), _dptr(self.workspace), C.byref(self.state), n_accept,
                              max_attempts, None if dt_log is None else _dptr(dt_log), 1 if use_graph else 0,
                              _stream_ptr(stream)))

    def _check_handles(self, stream):
        self.A.check(stream)
        if self.B is not None and self.B is not self.A:
            self.B.check(stream)

    def run_timed(self, y, D, n_accept, max_attempts=0, use_graph=True, stream=None, dt_log=None):
        """run() with the products' share of the GPU time measured inside the
        run (rs_rk45_run_timed).  Returns dict(product_ms, attempt_ms,
        attempts, hmvm_share)."""
        self._check(y, D)
        if dt_log is not None and (dt_log.dtype != _torch().float64 or not dt_log.is_cuda
                                   or dt_log.numel() < n_accept or not dt_log.is_contiguous()):
            raise ValueError("dt_log must be a contiguous float64 GPU tensor of at least n_accept entries")
        tm = _lib.RsRk45Timing()
        check(_lib.load().rs_rk45_run_timed(self.A._h, None if self.B is None else self.B._h, C.byref(self.params),
                                            _dptr(y), _dptr(D), _dptr(self.workspace), C.byref(self.state),
                                            n_accept, max_attempts, None if dt_log is None else _dptr(dt_log),
                                            1 if use_graph else 0, _stream_ptr(stream), C.byref(tm)))
        share = tm.product_ms / tm.attempt_ms if tm.attempt_ms > 0 else float("nan")
        return dict(product_ms=tm.product_ms, attempt_ms=tm.attempt_ms, attempts=tm.attempts, hmvm_share=share)

    def replay(self, y, D, dts, ckpt_every=0, stream=None, noalloc=False):
        """The integration on the frozen steps dts (rs_rk45_replay): y (and D,
        unless None) advance in place.  With ckpt_every > 0 returns the
        checkpoints (the state before every ckpt_every-th step) for adjoint().
        noalloc: rs_rk45_replay_noalloc (the library's static scratch instead
        of this object's workspace)."""
        torch = _torch()
        n = self.A.n
        _gpu_f64(y, (3 * n,), "y")
        if D is not None:
            _gpu_f64(D, (n,), "D")
        d = np.ascontiguousarray(dts, dtype=np.float64)
        m = d.shape[0]
        ckpt = None
        if ckpt_every > 0:
            ckpt = torch.empty(((m + ckpt_every - 1) // ckpt_every) * 3 * n, dtype=torch.float64, device=y.device)
        lib = _lib.load()
        args = (self.A._h, None if self.B is None else self.B._h, C.byref(self.params), _dptr(y),
                None if D is None else _dptr(D), d.ctypes.data_as(C.POINTER(C.c_double)), m,
                None if ckpt is None else _dptr(ckpt), max(ckpt_every, 1))
        if noalloc:
            check(lib.rs_rk45_replay_noalloc(*args, _stream_ptr(stream)))
        else:
            check(lib.rs_rk45_replay(*args, _dptr(self.workspace), _stream_ptr(stream)))
        self._check_handles(stream)
        return ckpt

    def adjoint(self, ckpt, dts, ckpt_every, y_bar, D_bar=None, a_bar=None, dc_bar=None, stream=None):
        """Reverse sweep of replay() (rs_rk45_adjoint).  y_bar: dL/dy_M on
        entry, dL/dy_0 on return (in place); D_bar: dL/dD_M or None.
        a_bar, dc_bar accumulate dL/da and dL/dd_c (new zero tensors when
        None).  Returns (y_bar, a_bar, dc_bar)."""
        torch = _torch()
        n = self.A.n
        d = np.ascontiguousarray(dts, dtype=np.float64)
        m = d.shape[0]
        dev = y_bar.device
        if a_bar is None:
            a_bar = torch.zeros(n, dtype=torch.float64, device=dev)
        if dc_bar is None:
            dc_bar = torch.zeros(n, dtype=torch.float64, device=dev)
        for t, k, name in ((y_bar, 3 * n, "y_bar"), (a_bar, n, "a_bar"), (dc_bar, n, "dc_bar")) + (
                () if D_bar is None else ((D_bar, n, "D_bar"),)):
            _gpu_f64(t, (k,), name)
        if ckpt is not None and ckpt_every > 0:
            _gpu_f64(ckpt, (((m + ckpt_every - 1) // ckpt_every) * 3 * n,), "ckpt")
        lib = _lib.load()
        nbytes = lib.rs_rk45_adjoint_workspace_bytes(n, max(1, min(ckpt_every, m)))
        if nbytes < 0:
            raise ValueError("bad adjoint sizes")
        if getattr(self, "_adj_ws", None) is None or self._adj_ws.numel() * 8 < nbytes:
            self._adj_ws = torch.empty(nbytes // 8, dtype=torch.float64, device=dev)
        check(lib.rs_rk45_adjoint(self.A._h, None if self.B is None else self.B._h, C.byref(self.params),
                                  None if ckpt is None else _dptr(ckpt), ckpt_every,
                                  d.ctypes.data_as(C.POINTER(C.c_double)), m,
                                  None if D_bar is None else _dptr(D_bar), _dptr(y_bar), _dptr(a_bar),
                                  _dptr(dc_bar), _dptr(self._adj_ws), self._adj_ws.numel() * 8,
                                  _stream_ptr(stream)))
        self._check_handles(stream)
        return y_bar, a_bar, dc_bar

    @property
    def t(self):
        return self.state.t

    @property
    def dt(self):
        return self.state.dt

    @dt.setter
    def dt(self, v):
        self.state.dt = v


class EnsembleRK45:
    """Up to 64 rate-and-state simulations on one fault advanced together
    (rs_ens_rk45_run): per-member FP64 state, parameters and step control on
    the GPU, one MFMA ensemble product with A (and B) per stage for all
    members.  a, b, dc: float64 GPU tensors (n, members); states y (3, n,
    members) and slip D (n, members), contiguous."""

    def __init__(self, A, B, a, b, dc, V0, f0, eta_rad, V_pl, mode="x3", eps_rk=1e-4, dt0=1.0):
        torch = _torch()
        n = A.n
        if a.dim() != 2 or a.shape[0] != n or not 1 <= a.shape[1] <= 64:
            raise ValueError("a must be (n, members) with 1 <= members <= 64")
        m = a.shape[1]
        for t in (a, b, dc):
            if t.shape != (n, m) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
                raise ValueError("a, b, dc must be contiguous float64 GPU tensors of shape (n, members)")
        self.A, self.B, self.members = A, B, m
        self._keep = (a, b, dc)
        self.params = _lib.RsEnsParams(n, m, _lib.MM_MODE[mode], V0, f0, eta_rad, V_pl, a.data_ptr(),
                                       b.data_ptr(), dc.data_ptr())
        nbytes = _lib.load().rs_ens_workspace_bytes(n, m)
        if nbytes < 0:
            raise ValueError("bad ensemble size")
        self.workspace = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=a.device)
        self.state = _lib.RsEnsState()
        self.state.eps_rk = eps_rk
        for r in range(64):
            self.state.dt[r] = dt0

    def run(self, y, D, n_accept, max_attempts=0, use_graph=True, stream=None):
        """Advance every member by n_accept accepted steps (graph replay needs
        a non-default stream)."""
        n, m = self.A.n, self.members
        _gpu_f64(y, (3, n, m), "y")
        _gpu_f64(D, (n, m), "D")
        check(_lib.load().rs_ens_rk45_run(self.A._h, None if self.B is None else self.B._h, C.byref(self.params),
                                          _dptr(y), _dptr(D), _dptr(self.workspace), C.byref(self.state), n_accept,
                                          max_attempts, 1 if use_graph else 0, _stream_ptr(stream)))

    @property
    def t(self):
        return np.array(self.state.t[:self.members])

    @property
    def dt(self):
        return np.array(self.state.dt[:self.members])

    @property
    def accepted(self):
        return np.array(self.state.accepted[:self.members])

    @property
    def rejected(self):
        return np.array(self.state.rejected[:self.members])


def kernel_entries(verts, slip_dir, mu, nu, rows, cols, component=0):
    """Kernel entries A[rows[k], cols[k]] (component 0) or B (component 1),
    evaluated on the host by the library's closed forms (hmat_kernel_entries)."""
    lib = _lib.load()
    verts = np.ascontiguousarray(verts, dtype=np.float64)
    slip_dir = np.ascontiguousarray(slip_dir, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows and cols must be 1-D arrays of equal length")
    mesh = _lib.HmatMesh(verts.shape[0], verts.shape[1], verts.ctypes.data_as(C.POINTER(C.c_double)),
                         slip_dir.ctypes.data_as(C.POINTER(C.c_double)))
    kind = _lib.GF_FS_TRIANGLE if verts.shape[1] == 3 else _lib.GF_FS_RECT_COPLANAR
    green = _lib.HmatGreen(kind, component, mu, nu)
    out = np.empty(rows.shape[0])
    check(lib.hmat_kernel_entries(C.byref(mesh), C.byref(green), rows.shape[0],
                                  rows.ctypes.data_as(C.POINTER(C.c_int64)),
                                  cols.ctypes.data_as(C.POINTER(C.c_int64)),
                                  out.ctypes.data_as(C.POINTER(C.c_double))))
    return out
