"""Python binding of libgnk (ctypes). Argument marshalling only: every step of
the solver runs in the HIP library; PyTorch provides device memory and the
stream. The library must be built (``python -m paper_1308_5351_amd.build``);
there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgnk.so")

# status codes (include/gnk.h)
OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_ODD_N, ERR_ZERO_A, ERR_ZERO_ETAP, ERR_NONFINITE, ERR_HIP, ERR_OOM = -1, -2, -3, -4, -5, -10, -11
FP64, MIXED = 0, 1
OP_FB, OP_FC, OP_GB, OP_FB_T, OP_FC_T, OP_GB_T, OP_LHAT, OP_FB_U, OP_GB_U = range(9)

EXPORTED = ("gnk_create", "gnk_destroy", "gnk_set_stream", "gnk_last_error", "gnk_version",
            "gnk_profile", "gnk_profile_read", "gnk_cauchy_sum", "gnk_apply", "gnk_fbie", "gnk_fbie_ad",
            "gnk_fbie_batched", "gnk_fbie_adjoint", "gnk_geom_vjp", "gnk_fourier_curve", "gnk_fourier_vjp",
            "gnk_fcau", "gnk_cauchy_sum_tree", "gnk_circular_slit_map", "gnk_slit_map", "gnk_fcau_tree",
            "gnk_cauchy_sum_noalloc")


class GnkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gnk status {status}: {msg}")
        self.status = status


class _Domain(C.Structure):
    _fields_ = [("m1", C.c_int64), ("n", C.c_int64), ("eta", C.c_void_p), ("etap", C.c_void_p),
                ("etapp", C.c_void_p), ("A", C.c_void_p), ("Ap", C.c_void_p), ("c", C.c_int)]


class _Opts(C.Structure):
    _fields_ = [("restart", C.c_int), ("maxit", C.c_int), ("tol", C.c_double), ("prec", C.c_int),
                ("inner_tol", C.c_double), ("max_refine", C.c_int), ("x0", C.c_void_p),
                ("no_subtraction", C.c_int), ("far_tol", C.c_double), ("hist", C.c_void_p),
                ("hist_len", C.c_int)]


class Info(C.Structure):
    _fields_ = [("flag", C.c_int), ("outer_it", C.c_int), ("inner_it", C.c_int), ("mixed_steps", C.c_int),
                ("relres", C.c_double), ("true_relres", C.c_double), ("refine_steps", C.c_int),
                ("hist_count", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Prof(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("pair_cols", C.c_double), ("flops", C.c_double),
                ("launches1", C.c_int64), ("ms1", C.c_double), ("pairs1", C.c_double),
                ("launches_mixed", C.c_int64), ("ms_mixed", C.c_double), ("pair_cols_mixed", C.c_double),
                ("launches_tree", C.c_int64), ("ms_tree", C.c_double), ("flops_tree", C.c_double),
                ("launches_fft", C.c_int64), ("ms_fft", C.c_double), ("bytes_fft", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgnk.so and declare the C signatures. Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1308_5351_amd.build`")
    lib = C.CDLL(path)
    P = C.c_void_p
    lib.gnk_create.argtypes = [C.POINTER(P), C.c_int]
    lib.gnk_destroy.argtypes = [P]
    lib.gnk_set_stream.argtypes = [P, P]
    lib.gnk_last_error.argtypes = [P]
    lib.gnk_last_error.restype = C.c_char_p
    lib.gnk_version.restype = C.c_char_p
    lib.gnk_profile.argtypes = [P, C.c_int]
    lib.gnk_profile_read.argtypes = [P, C.POINTER(Prof), C.c_int]
    lib.gnk_cauchy_sum.argtypes = [P, C.c_int64, P, P, C.c_int, P]
    lib.gnk_cauchy_sum_noalloc.argtypes = [P, C.c_int64, P, P, C.c_int, P]
    lib.gnk_apply.argtypes = [P, C.POINTER(_Domain), C.c_int, C.c_int, P, C.c_int, P]
    lib.gnk_fbie.argtypes = [P, C.POINTER(_Domain), P, C.c_int, C.POINTER(_Opts), P, P, C.POINTER(Info)]
    lib.gnk_fbie_ad.argtypes = [P, C.POINTER(_Domain), P, C.c_int, C.POINTER(_Opts), P, C.POINTER(Info)]
    lib.gnk_fbie_batched.argtypes = [P, C.c_int, C.POINTER(_Domain), C.POINTER(P), C.POINTER(C.c_int),
                                     C.POINTER(_Opts), C.POINTER(P), C.POINTER(P), C.POINTER(Info)]
    lib.gnk_fbie_adjoint.argtypes = [P, C.POINTER(_Domain), P, P, C.c_int, C.POINTER(_Opts), P, P,
                                     C.POINTER(Info)]
    lib.gnk_geom_vjp.argtypes = [P, C.POINTER(_Domain), C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double),
                                 C.POINTER(P), C.POINTER(P), P, P, P]
    lib.gnk_fourier_curve.argtypes = [P, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int, P, P, P, P]
    lib.gnk_fourier_vjp.argtypes = [P, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int, P, P, P, P]
    lib.gnk_fcau.argtypes = [P, C.c_int64, C.c_int64, P, P, P, C.c_int, P, C.c_int64, P, P]
    lib.gnk_cauchy_sum_tree.argtypes = [P, C.c_int64, P, P, C.c_int, C.c_double, P]
    lib.gnk_fcau_tree.argtypes = [P, C.c_int64, C.c_int64, P, P, P, C.c_int, P, C.c_int64, P, C.c_double, P]
    lib.gnk_circular_slit_map.argtypes = [P, C.c_int64, C.c_int64, P, P, C.POINTER(C.c_double), C.POINTER(_Opts), P,
                                          C.POINTER(C.c_double), C.POINTER(Info)]
    lib.gnk_slit_map.argtypes = [P, C.c_int64, C.c_int64, P, P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(_Opts), P, C.POINTER(C.c_double), C.POINTER(Info)]
    for f in EXPORTED:
        if f not in ("gnk_last_error", "gnk_version"):
            getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


@dataclass
class DeviceDomain:
    """Boundary data resident on the GPU (complex128 tensors of length N)."""
    m1: int
    n: int
    eta: torch.Tensor
    etap: torch.Tensor
    A: torch.Tensor
    etapp: Optional[torch.Tensor] = None
    Ap: Optional[torch.Tensor] = None
    c: int = 1

    @property
    def N(self):
        return self.m1 * self.n

    @classmethod
    def from_host(cls, dom, device="cuda"):
        """From a workloads.Domain (NumPy arrays)."""
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)
        return cls(dom.m1, dom.n, t(dom.eta), t(dom.etap), t(dom.A), t(dom.etapp), t(dom.Ap), dom.c)

    def _struct(self):
        p = lambda x: None if x is None else x.data_ptr()
        return _Domain(self.m1, self.n, p(self.eta), p(self.etap), p(self.etapp), p(self.A), p(self.Ap), self.c)


def _check_real(x: torch.Tensor, N: int, name: str):
    if x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if x.dim() == 1:
        x = x.unsqueeze(1)
    if x.shape[0] != N:
        raise ValueError(f"{name} has {x.shape[0]} rows, expected N = {N}")
    # column-major N x nrhs == row-major nrhs x N
    return x.t().contiguous(), x.shape[1]


def _from_cols(buf: torch.Tensor, like_1d: bool):
    out = buf.t()
    return out[:, 0] if like_1d else out


class Context:
    """A libgnk context bound to one device and to torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        st = self.lib.gnk_create(C.byref(h), device)
        if st != OK:
            raise GnkError(st, "gnk_create failed")
        self.h = h
        self._stream = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.gnk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind_stream(self):
        # torch's default stream is the legacy null stream, which cannot be
        # captured: the context then keeps its own blocking stream (ordered
        # with the null stream); another current stream is passed through.
        s = torch.cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            self.lib.gnk_set_stream(self.h, C.c_void_p(s) if s else None)
            self._stream = s

    def _raise(self, st, allow_not_converged=True):
        if st == OK or (allow_not_converged and st == NOT_CONVERGED):
            return
        raise GnkError(st, self.lib.gnk_last_error(self.h).decode())

    # ------------------------------------------------------------------ calls
    def profile(self, enable: bool):
        """Start/stop HIP-event timing of the Cauchy-sum launches."""
        self._raise(self.lib.gnk_profile(self.h, 1 if enable else 0), False)

    def profile_read(self, reset: bool = True) -> dict:
        p = Prof()
        self._raise(self.lib.gnk_profile_read(self.h, C.byref(p), 1 if reset else 0), False)
        return p.as_dict()

    def cauchy_sum(self, eta: torch.Tensor, w: torch.Tensor, far_tol: float = 0.0) -> torch.Tensor:
        """S = E w, S_i = sum_{j != i} w_j / (eta_i - eta_j); w: (N,) or (N, nrhs) complex128.
        far_tol > 0: the far field from the treecode's expansions (gnk_cauchy_sum_tree)."""
        self._bind_stream()
        N = eta.shape[0]
        one = w.dim() == 1
        wc = (w.unsqueeze(1) if one else w).t().contiguous()
        S = torch.empty_like(wc)
        if far_tol > 0:
            st = self.lib.gnk_cauchy_sum_tree(self.h, N, eta.data_ptr(), wc.data_ptr(), wc.shape[0], far_tol,
                                              S.data_ptr())
            self._raise(st, False)
            return _from_cols(S, one)
        st = self.lib.gnk_cauchy_sum(self.h, N, eta.data_ptr(), wc.data_ptr(), wc.shape[0], S.data_ptr())
        self._raise(st, False)
        return _from_cols(S, one)

    def fcau(self, eta: torch.Tensor, etap: torch.Tensor, f: torch.Tensor, z: torch.Tensor, m1: int, n: int,
             finf=None, far_tol: float = 0.0) -> torch.Tensor:
        """f at the points z of G by the Cauchy integral formula (Sec. 7): eta, etap (N,) and f (N,) or
        (N, nrhs) complex128 on the device, N = m1 n; z (nz,) complex128. finf: None for bounded G, else
        f(infinity) (a number or nrhs numbers) for unbounded G. far_tol > 0: the sums by the treecode
        (gnk_fcau_tree). Returns (nz,) or (nz, nrhs)."""
        self._bind_stream()
        N = m1 * n
        for name, t in (("eta", eta), ("etap", etap)):
            if t.dtype != torch.complex128 or t.shape != (N,) or not t.is_cuda:
                raise ValueError(f"{name} must be a complex128 CUDA tensor of shape ({N},)")
        if f.dtype != torch.complex128 or f.shape[0] != N or f.dim() > 2 or not f.is_cuda:
            raise ValueError(f"f must be complex128 of shape ({N},) or ({N}, nrhs) on the GPU")
        if z.dtype != torch.complex128 or z.dim() != 1 or not z.is_cuda:
            raise ValueError("z must be a 1-D complex128 CUDA tensor")
        one = f.dim() == 1
        fc = (f.unsqueeze(1) if one else f).t().contiguous()
        nrhs = fc.shape[0]
        zc = z.contiguous()
        out = torch.empty((nrhs, zc.shape[0]), dtype=torch.complex128, device=z.device)
        fin = None
        if finf is not None:
            v = np.broadcast_to(np.asarray(finf, np.complex128), (nrhs,))
            fin = np.ascontiguousarray(v).view(np.float64)
        ec, pc = eta.contiguous(), etap.contiguous()
        fptr = None if fin is None else fin.ctypes.data
        if far_tol > 0.0:
            st = self.lib.gnk_fcau_tree(self.h, m1, n, ec.data_ptr(), pc.data_ptr(), fc.data_ptr(), nrhs,
                                        zc.data_ptr(), zc.shape[0], fptr, far_tol, out.data_ptr())
        else:
            st = self.lib.gnk_fcau(self.h, m1, n, ec.data_ptr(), pc.data_ptr(), fc.data_ptr(), nrhs,
                                   zc.data_ptr(), zc.shape[0], fptr, out.data_ptr())
        self._raise(st, False)
        return _from_cols(out, one)

    def circular_slit_map(self, eta: torch.Tensor, etap: torch.Tensor, m1: int, n: int, alpha: complex,
                          restart=25, maxit=40, tol=1e-12, far_tol=0.0):
        """Boundary values f (N,) complex128 of the map of a bounded domain onto the unit disc with circular
        slits (f(alpha) = 0, f'(alpha) > 0) and the slit radii (m1,) (R_0 = 1). Returns (f, radii, info, status)."""
        self._bind_stream()
        N = m1 * n
        for name, t in (("eta", eta), ("etap", etap)):
            if t.dtype != torch.complex128 or t.shape != (N,) or not t.is_cuda:
                raise ValueError(f"{name} must be a complex128 CUDA tensor of shape ({N},)")
        ec, pc = eta.contiguous(), etap.contiguous()
        f = torch.empty(N, dtype=torch.complex128, device=eta.device)
        al = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        radii = (C.c_double * m1)()
        info = (Info * 1)()
        o = self._opts(restart, maxit, tol, FP64, 0.0, 0, None, True, far_tol)
        st = self.lib.gnk_circular_slit_map(self.h, m1, n, ec.data_ptr(), pc.data_ptr(), al, C.byref(o),
                                            f.data_ptr(), radii, info)
        self._raise(st)
        return f, np.array(radii[:]), info[0].as_dict(), st

    def slit_map(self, eta: torch.Tensor, etap: torch.Tensor, m1: int, n: int, alpha: complex, theta,
                 restart=25, maxit=40, tol=1e-12, far_tol=0.0, bounded=True):
        """Boundary values f (N,) complex128 of the map of a bounded domain onto the unit disc (theta[0] = pi/2)
        or of an unbounded one onto the extended plane (f(z) = z + O(1)) with slits on
        Re[exp(i (pi/2 - theta_j)) log w] = level_j (circular for theta_j = pi/2, radial at angle -level_j for
        theta_j = 0); theta: m1 reals. Returns (f, level, info, status)."""
        self._bind_stream()
        N = m1 * n
        for name, t in (("eta", eta), ("etap", etap)):
            if t.dtype != torch.complex128 or t.shape != (N,) or not t.is_cuda:
                raise ValueError(f"{name} must be a complex128 CUDA tensor of shape ({N},)")
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.shape != (m1,):
            raise ValueError(f"theta must hold {m1} values")
        ec, pc = eta.contiguous(), etap.contiguous()
        f = torch.empty(N, dtype=torch.complex128, device=eta.device)
        al = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
        tha = (C.c_double * m1)(*th.tolist())
        level = (C.c_double * m1)()
        info = (Info * 1)()
        o = self._opts(restart, maxit, tol, FP64, 0.0, 0, None, True, far_tol)
        st = self.lib.gnk_slit_map(self.h, m1, n, ec.data_ptr(), pc.data_ptr(), int(bool(bounded)), al, tha, C.byref(o),
                                   f.data_ptr(), level, info)
        self._raise(st)
        return f, np.array(level[:]), info[0].as_dict(), st

    def apply(self, dom: DeviceDomain, op: int, x: torch.Tensor, prec: int = FP64) -> torch.Tensor:
        self._bind_stream()
        one = x.dim() == 1
        xc, nrhs = _check_real(x, dom.N, "x")
        y = torch.empty_like(xc)
        d = dom._struct()
        st = self.lib.gnk_apply(self.h, C.byref(d), op, prec, xc.data_ptr(), nrhs, y.data_ptr())
        self._raise(st, False)
        return _from_cols(y, one)

    @staticmethod
    def _opts(restart, maxit, tol, prec, inner_tol, max_refine, x0, subtract=True, far_tol=0.0, hist=None):
        hl = 0 if hist is None else hist[1]
        return _Opts(restart, maxit, tol, prec, inner_tol, max_refine, None if x0 is None else x0.data_ptr(),
                     0 if subtract else 1, far_tol, None if hist is None else C.addressof(hist[0]), hl)

    @staticmethod
    def _hist(ncol, hist_len):
        """(host buffer, hist_len) for the residual history of ncol columns, or None."""
        if not hist_len:
            return None
        return (C.c_double * (ncol * hist_len))(), int(hist_len)

    @staticmethod
    def _infos(infos, hist):
        out = [i.as_dict() for i in infos]
        if hist is not None:
            buf, hl = hist
            for q, d in enumerate(out):
                d["hist"] = list(buf[q * hl:q * hl + d["hist_count"]])
        return out

    def fbie(self, dom: DeviceDomain, gam: torch.Tensor, restart=25, maxit=40, tol=1e-12, prec=FP64,
             inner_tol=0.0, max_refine=0, x0=None, want_h=True, subtract=True, far_tol=0.0, hist_len=0):
        """Solve (I - N) mu = -M gamma and h = [M mu - (I - N) gamma]/2. Returns (mu, h, infos, status).
        subtract=False: without singularity subtraction (Example 2's comparison; needs etapp, Ap).
        hist_len > 0: each info also holds "hist", the column's residual history."""
        self._bind_stream()
        one = gam.dim() == 1
        g, nrhs = _check_real(gam, dom.N, "gam")
        mu = torch.empty_like(g)
        h = torch.empty_like(g) if want_h else None
        x0c = None if x0 is None else _check_real(x0, dom.N, "x0")[0]
        hist = self._hist(nrhs, hist_len)
        o = self._opts(restart, maxit, tol, prec, inner_tol, max_refine, x0c, subtract, far_tol, hist)
        infos = (Info * nrhs)()
        d = dom._struct()
        st = self.lib.gnk_fbie(self.h, C.byref(d), g.data_ptr(), nrhs, C.byref(o), mu.data_ptr(),
                               None if h is None else h.data_ptr(), infos)
        self._raise(st)
        return (_from_cols(mu, one), None if h is None else _from_cols(h, one), self._infos(infos, hist), st)

    def fbie_ad(self, dom: DeviceDomain, gam: torch.Tensor, restart=25, maxit=40, tol=1e-12, prec=FP64,
                inner_tol=0.0, max_refine=0, x0=None, subtract=True, far_tol=0.0, hist_len=0):
        """Solve (I + N* + J) mu = gamma. Returns (mu, infos, status).
        subtract=False: without singularity subtraction (Example 2's comparison)."""
        self._bind_stream()
        one = gam.dim() == 1
        g, nrhs = _check_real(gam, dom.N, "gam")
        mu = torch.empty_like(g)
        x0c = None if x0 is None else _check_real(x0, dom.N, "x0")[0]
        hist = self._hist(nrhs, hist_len)
        o = self._opts(restart, maxit, tol, prec, inner_tol, max_refine, x0c, subtract, far_tol, hist)
        infos = (Info * nrhs)()
        d = dom._struct()
        st = self.lib.gnk_fbie_ad(self.h, C.byref(d), g.data_ptr(), nrhs, C.byref(o), mu.data_ptr(), infos)
        self._raise(st)
        return _from_cols(mu, one), self._infos(infos, hist), st

    def fbie_batched(self, doms, gams, restart=25, maxit=40, tol=1e-12, prec=FP64, inner_tol=0.0, want_h=True,
                     subtract=True, max_refine=0, hist_len=0):
        """Batched FBIE over several domains. gams[d]: (N_d,) or (N_d, nrhs_d) float64 CUDA.
        Returns (mus, hs, infos, status) with one entry per domain (infos: list of lists)."""
        self._bind_stream()
        nd = len(doms)
        if nd != len(gams) or nd == 0:
            raise ValueError("need one gamma per domain")
        cols, ones = [], []
        for d, g in zip(doms, gams):
            gc, k = _check_real(g, d.N, "gam")
            cols.append((gc, k))
            ones.append(g.dim() == 1)
        mus = [torch.empty_like(gc) for gc, _ in cols]
        hs = [torch.empty_like(gc) for gc, _ in cols] if want_h else None
        D = (_Domain * nd)(*[d._struct() for d in doms])
        G = (C.c_void_p * nd)(*[gc.data_ptr() for gc, _ in cols])
        R = (C.c_int * nd)(*[k for _, k in cols])
        MU = (C.c_void_p * nd)(*[m.data_ptr() for m in mus])
        H = (C.c_void_p * nd)(*[h.data_ptr() for h in hs]) if want_h else None
        ncol = sum(k for _, k in cols)
        infos = (Info * ncol)()
        hist = self._hist(ncol, hist_len)
        o = self._opts(restart, maxit, tol, prec, inner_tol, max_refine, None, subtract, 0.0, hist)
        st = self.lib.gnk_fbie_batched(self.h, nd, D, G, R, C.byref(o), MU, H, infos)
        self._raise(st)
        flat = self._infos(infos, hist)
        out_i, q = [], 0
        for _, k in cols:
            out_i.append(flat[q:q + k])
            q += k
        mus = [_from_cols(m, one) for m, one in zip(mus, ones)]
        hs = [_from_cols(h, one) for h, one in zip(hs, ones)] if want_h else None
        return mus, hs, out_i, st

    # ------------------------------------------------------- differentiation
    def fbie_adjoint(self, dom: DeviceDomain, g_mu: Optional[torch.Tensor] = None, g_h: Optional[torch.Tensor] = None,
                     restart=25, maxit=40, tol=1e-12, prec=FP64, inner_tol=0.0, want_g_gam=True, max_refine=0,
                     hist_len=0):
        """Adjoint solve of FBIE: lam = Aop^-T (Cop^T g_h / 2 + g_mu) and
        dL/dgamma = -Aop^T g_h / 2 - Cop^T lam. Returns (lam, g_gam, infos, status)."""
        self._bind_stream()
        ref = g_h if g_h is not None else g_mu
        if ref is None:
            raise ValueError("need g_mu or g_h")
        one = ref.dim() == 1
        gm = _check_real(g_mu, dom.N, "g_mu") if g_mu is not None else None
        gh = _check_real(g_h, dom.N, "g_h") if g_h is not None else None
        nrhs = (gm or gh)[1]
        if gm is not None and gh is not None and gm[1] != gh[1]:
            raise ValueError("g_mu and g_h have different column counts")
        lam = torch.empty((nrhs, dom.N), dtype=torch.float64, device=ref.device)
        g_gam = torch.empty_like(lam) if want_g_gam else None
        hist = self._hist(nrhs, hist_len)
        o = self._opts(restart, maxit, tol, prec, inner_tol, max_refine, None, True, 0.0, hist)
        infos = (Info * nrhs)()
        d = dom._struct()
        st = self.lib.gnk_fbie_adjoint(self.h, C.byref(d), None if gm is None else gm[0].data_ptr(),
                                       None if gh is None else gh[0].data_ptr(), nrhs, C.byref(o), lam.data_ptr(),
                                       None if g_gam is None else g_gam.data_ptr(), infos)
        self._raise(st)
        return (_from_cols(lam, one), None if g_gam is None else _from_cols(g_gam, one),
                self._infos(infos, hist), st)

    def geom_vjp(self, dom: DeviceDomain, terms, want=(True, True, True)):
        """Gradients of s = sum_t c_t u_t^T Op_t v_t with respect to (eta, eta', A).
        terms: list of (op, c, u, v) with op OP_FB or OP_FC, c a float and u, v
        contiguous float64 CUDA vectors of length N. Returns three complex128
        tensors (None where not wanted)."""
        self._bind_stream()
        nt = len(terms)
        for _, _, u, v in terms:
            for x in (u, v):
                if x.dtype != torch.float64 or not x.is_cuda or x.dim() != 1 or x.shape[0] != dom.N \
                        or not x.is_contiguous():
                    raise ValueError("term vectors must be contiguous float64 CUDA vectors of length N")
        ops = (C.c_int * nt)(*[int(t[0]) for t in terms])
        cf = (C.c_double * nt)(*[float(t[1]) for t in terms])
        U = (C.c_void_p * nt)(*[t[2].data_ptr() for t in terms])
        V = (C.c_void_p * nt)(*[t[3].data_ptr() for t in terms])
        outs = [torch.empty(dom.N, dtype=torch.complex128, device=dom.eta.device) if w else None for w in want]
        d = dom._struct()
        st = self.lib.gnk_geom_vjp(self.h, C.byref(d), nt, ops, cf, U, V,
                                   *[None if o is None else o.data_ptr() for o in outs])
        self._raise(st, False)
        return tuple(outs)

    def fourier_curve(self, coef: torch.Tensor, kmin: int, n: int, ccw: bool = False):
        """eta, eta', eta'' (complex128, length m1*n) of the curves
        eta_j(t) = sum_k coef[j, k - kmin] e^{i s k t}, s = +1 (ccw) or -1, at t_p = 2 pi p / n."""
        self._bind_stream()
        if coef.dtype != torch.complex128 or not coef.is_cuda or coef.dim() != 2:
            raise TypeError("coef must be an (m1, nk) complex128 CUDA tensor")
        coef = coef.contiguous()
        m1, nk = coef.shape
        out = [torch.empty(m1 * n, dtype=torch.complex128, device=coef.device) for _ in range(3)]
        st = self.lib.gnk_fourier_curve(self.h, m1, n, kmin, nk, 1 if ccw else 0, coef.data_ptr(),
                                        *[o.data_ptr() for o in out])
        self._raise(st, False)
        return tuple(out)

    def fourier_vjp(self, g_eta, g_etap, g_etapp, m1: int, nk: int, kmin: int, n: int, ccw: bool = False):
        """Reverse mode of fourier_curve: the (m1, nk) complex gradient of the coefficients."""
        self._bind_stream()
        ptr = lambda x: None if x is None else x.contiguous().data_ptr()
        keep = [None if x is None else x.contiguous() for x in (g_eta, g_etap, g_etapp)]
        ref = next(x for x in keep if x is not None)
        g = torch.empty((m1, nk), dtype=torch.complex128, device=ref.device)
        st = self.lib.gnk_fourier_vjp(self.h, m1, n, kmin, nk, 1 if ccw else 0, *[ptr(x) for x in keep],
                                      g.data_ptr())
        self._raise(st, False)
        return g
