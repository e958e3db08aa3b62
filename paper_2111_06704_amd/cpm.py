"""ctypes binding of libcpm (include/cpm.h).

Argument marshalling only: every computation runs in the HIP library. Device
arrays are torch tensors on the current HIP device; their data pointers and
the current torch stream are passed through the C ABI. The library must be
built (``paper_2111_06704_amd.build``); a missing library is an error, there
is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcpm.so")

CPM_OK, CPM_EINVAL, CPM_ENOMEM, CPM_EDEVICE, CPM_ENOTSPD, CPM_ENOTCONV, CPM_ESTATE = 0, -1, -2, -3, -4, -5, -6
STORE_F32, STORE_BF16 = 1, 2
PREC_F64, PREC_F32, PREC_BF16 = 0, 1, 2
WARM_ZERO, WARM_CHI, WARM_MLP = 0, 1, 2
PRECOND_JACOBI, PRECOND_DC = 0, 1
MLP_IN, MLP_HIDDEN = 26, 64
MLP_NPARAM = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1

EXPORTS = [
    "cpm_build_E", "cpm_free", "cpm_set_stream", "cpm_describe", "cpm_rhs", "cpm_rhs_noalloc",
    "cpm_solve",
    "cpm_get_E", "cpm_get_E_block", "cpm_get_dprime", "cpm_matvec", "cpm_mlp_init", "cpm_mlp_neighbours",
    "cpm_mlp_set_params", "cpm_mlp_get_params", "cpm_mlp_features", "cpm_mlp_forward",
    "cpm_mlp_loss_grad", "cpm_mlp_train_step", "cpm_mlp_train_epoch", "cpm_set_warm_chi",
    "cpm_warm_start",
    "cpm_profile_enable", "cpm_profile_read", "cpm_precond_dc", "cpm_precond_apply",
    "cpm_precond_sparse_inverse", "cpm_precond_gap", "cpm_precond_coarse",
    "cpm_mi_build", "cpm_mi_solve", "cpm_gcd_build", "cpm_gcd_solve",
    "cpm_status_str", "cpm_last_error",
]
PROFILE_BUILD = 4


class CpmError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {message} (status {status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [("gauss_inv_width", C.c_double), ("gauss_inv_width_per_atom", C.POINTER(C.c_double)),
                ("ewald_split", C.c_double), ("rcut", C.c_double), ("kspace_eps", C.c_double),
                ("kmax_override", C.c_double), ("store_mask", C.c_uint),
                ("slab_correction", C.c_int), ("point_charge_self", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int),
                ("warm_start", C.c_int), ("inner_tol", C.c_double), ("check_every", C.c_int),
                ("preconditioner", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer", C.c_int), ("max_rel_resid", C.c_double),
                ("initial_rel_resid", C.c_double), ("max_abs_sum_q", C.c_double),
                ("warm_ms", C.c_double), ("solve_ms", C.c_double), ("fell_back", C.c_int),
                ("frame_iters", C.POINTER(C.c_int)), ("frame_rel_resid", C.POINTER(C.c_double))]


class ProfileInfo(C.Structure):
    _fields_ = [("launches", C.c_int64 * 5), ("ms", C.c_double * 5), ("work", C.c_double * 5)]


_lib = None


def lib():
    """Load libcpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2111_06704_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp, i64, dbl, f32 = C.c_void_p, C.c_int64, C.c_double, C.c_float
    L.cpm_build_E.argtypes = [vp, i64, vp, C.POINTER(Params), vp, C.POINTER(vp)]
    L.cpm_free.argtypes = [vp]
    L.cpm_free.restype = None
    L.cpm_set_stream.argtypes = [vp, vp]
    L.cpm_describe.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(dbl), C.POINTER(i64)]
    L.cpm_rhs.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp]
    L.cpm_rhs_noalloc.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp]
    L.cpm_solve.argtypes = [vp, vp, vp, i64, C.POINTER(SolveOpts), vp, C.POINTER(SolveInfo)]
    L.cpm_get_E.argtypes = [vp, C.c_int, vp, i64]
    L.cpm_get_E_block.argtypes = [vp, C.c_int, i64, i64, i64, i64, vp, i64]
    L.cpm_get_dprime.argtypes = [vp, vp, C.POINTER(dbl)]
    L.cpm_precond_sparse_inverse.argtypes = [vp, dbl]
    L.cpm_precond_gap.argtypes = [vp, C.c_int, C.POINTER(dbl)]
    L.cpm_precond_coarse.argtypes = [vp, dbl, C.POINTER(C.c_int64)]
    L.cpm_matvec.argtypes = [vp, C.c_int, vp, i64, vp]
    L.cpm_mlp_init.argtypes = [vp, vp, C.c_int32, f32, f32, f32]
    L.cpm_mlp_neighbours.argtypes = [vp, vp]
    L.cpm_mlp_set_params.argtypes = [vp, vp]
    L.cpm_mlp_get_params.argtypes = [vp, vp]
    L.cpm_mlp_features.argtypes = [vp, vp, i64, vp]
    L.cpm_mlp_forward.argtypes = [vp, vp, i64, vp]
    L.cpm_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp, C.POINTER(dbl)]
    L.cpm_mlp_train_step.argtypes = [vp, vp, vp, i64, f32, f32, f32, f32, C.POINTER(dbl)]
    L.cpm_mlp_train_epoch.argtypes = [vp, vp, vp, i64, vp, i64, f32, f32, f32, f32, C.POINTER(dbl)]
    L.cpm_set_warm_chi.argtypes = [vp, vp, C.POINTER(SolveOpts)]
    L.cpm_warm_start.argtypes = [vp, C.c_int, vp, vp, i64, vp, vp]
    L.cpm_gcd_build.argtypes = [vp, vp, C.c_int32, C.POINTER(SolveOpts), vp, C.POINTER(dbl),
                                C.POINTER(dbl), C.POINTER(SolveInfo)]
    L.cpm_gcd_solve.argtypes = [vp, vp, vp, i64, C.POINTER(SolveOpts), vp, vp,
                                C.POINTER(SolveInfo)]
    L.cpm_profile_enable.argtypes = [vp, C.c_int]
    L.cpm_profile_read.argtypes = [vp, C.POINTER(ProfileInfo)]
    L.cpm_status_str.argtypes = [C.c_int]
    L.cpm_status_str.restype = C.c_char_p
    L.cpm_last_error.argtypes = []
    L.cpm_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("cpm_free", "cpm_status_str", "cpm_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st: int, where: str, allow=()):
    if st != CPM_OK and st not in allow:
        msg = lib().cpm_last_error().decode(errors="replace")
        raise CpmError(st, where, msg)
    return st


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


class System:
    """An assembled Ewald matrix for one electrode geometry (cpm_build_E)."""

    def __init__(self, pos, box, gauss_inv_width=1.979, ewald_split=0.3, rcut=12.0,
                 kspace_eps=1e-6, kmax_override=0.0, store=(), per_atom_width=None,
                 profile_build=False, slab=False, point_charge_self=False):
        L = lib()
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        box = np.ascontiguousarray(box, dtype=np.float64)
        self.n = int(pos.shape[0])
        p = Params()
        p.gauss_inv_width = float(gauss_inv_width)
        self._widths = None
        if per_atom_width is not None:
            self._widths = np.ascontiguousarray(per_atom_width, dtype=np.float64)
            p.gauss_inv_width_per_atom = self._widths.ctypes.data_as(C.POINTER(C.c_double))
        p.ewald_split = float(ewald_split)
        p.rcut = float(rcut)
        p.kspace_eps = float(kspace_eps)
        p.kmax_override = float(kmax_override)
        mask = 0
        for s in store:
            mask |= {"f32": STORE_F32, "bf16": STORE_BF16}[s]
        p.store_mask = mask | (PROFILE_BUILD if profile_build else 0)
        p.slab_correction = 1 if slab else 0
        p.point_charge_self = 1 if point_charge_self else 0
        self.store = tuple(store)
        h = C.c_void_p()
        st = L.cpm_build_E(pos.ctypes.data, self.n, box.ctypes.data, C.byref(p), _stream(), C.byref(h))
        _check(st, "cpm_build_E")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().cpm_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, on=True, stride=1):
        """Time launches of the block product, the assembly contraction and the
        structure factors (every stride-th of each kind)."""
        _check(lib().cpm_profile_enable(self._h, max(1, int(stride)) if on else 0),
               "cpm_profile_enable")

    def profile_read(self):
        """Per kind (0 FP64, 1 FP32, 2 BF16 matvec, 3 assembly, 4 structure
        factors): launches, ms, work."""
        pi = ProfileInfo()
        _check(lib().cpm_profile_read(self._h, C.byref(pi)), "cpm_profile_read")
        return [dict(launches=pi.launches[k], ms=pi.ms[k], work=pi.work[k]) for k in range(5)]

    def describe(self):
        n, nk, dev = C.c_int64(), C.c_int64(), C.c_int64()
        km = C.c_double()
        _check(lib().cpm_describe(self._h, C.byref(n), C.byref(nk), C.byref(km), C.byref(dev)),
               "cpm_describe")
        return dict(n=n.value, n_kvec=nk.value, kmax=km.value, device_bytes=dev.value)

    def set_stream(self):
        _check(lib().cpm_set_stream(self._h, _stream()), "cpm_set_stream")

    def rhs(self, ion_pos, ion_q, chi, b_out=None, qsol_out=None):
        """b (F, N) and Q_sol (F,) for ion frames (F, M, 3), (F, M) and chi (N,) volts."""
        import torch
        f = int(ion_pos.shape[0]) if ion_pos is not None else 1
        m = int(ion_pos.shape[1]) if ion_pos is not None else 0
        dev = chi.device
        if b_out is None:
            b_out = torch.empty((f, self.n), dtype=torch.float64, device=dev)
        if qsol_out is None:
            qsol_out = torch.empty((f,), dtype=torch.float64, device=dev)
        st = lib().cpm_rhs(self._h, _ptr(ion_pos, torch.float64) if m else None,
                           _ptr(ion_q, torch.float64) if m else None, m, f,
                           _ptr(chi, torch.float64), _ptr(b_out, torch.float64),
                           _ptr(qsol_out, torch.float64))
        _check(st, "cpm_rhs")
        return b_out, qsol_out

    def rhs_noalloc(self, ion_pos, ion_q, chi, b_out, qsol_out):
        """cpm_rhs with the library's static scratch (allocates nothing; b_out
        (F, N) and qsol_out (F,) are the caller's)."""
        import torch
        f = int(ion_pos.shape[0]) if ion_pos is not None else int(b_out.shape[0])
        m = int(ion_pos.shape[1]) if ion_pos is not None else 0
        st = lib().cpm_rhs_noalloc(self._h, _ptr(ion_pos, torch.float64) if m else None,
                                   _ptr(ion_q, torch.float64) if m else None, m, f,
                                   _ptr(chi, torch.float64), _ptr(b_out, torch.float64),
                                   _ptr(qsol_out, torch.float64))
        _check(st, "cpm_rhs_noalloc")
        return b_out, qsol_out

    def solve(self, b, qsol, tol=1e-10, max_iter=5000, precision=PREC_F64, warm_start=WARM_ZERO,
              inner_tol=1e-3, check_every=8, q_out=None, allow_notconv=False,
              preconditioner=PRECOND_JACOBI):
        """Electrode charges (F, N) and a dict of solve statistics."""
        import torch
        f = int(b.shape[0])
        if q_out is None:
            q_out = torch.empty_like(b)
        o = SolveOpts(tol=tol, max_iter=max_iter, precision=precision, warm_start=warm_start,
                      inner_tol=inner_tol, check_every=check_every, preconditioner=preconditioner)
        fit = (C.c_int * f)()
        frr = (C.c_double * f)()
        info = SolveInfo()
        info.frame_iters = C.cast(fit, C.POINTER(C.c_int))
        info.frame_rel_resid = C.cast(frr, C.POINTER(C.c_double))
        st = lib().cpm_solve(self._h, _ptr(b, torch.float64), _ptr(qsol, torch.float64), f,
                             C.byref(o), _ptr(q_out, torch.float64), C.byref(info))
        _check(st, "cpm_solve", allow=(CPM_ENOTCONV,) if allow_notconv else ())
        stats = dict(status=st, iterations=info.iterations, outer=info.outer,
                     max_rel_resid=info.max_rel_resid, initial_rel_resid=info.initial_rel_resid,
                     max_abs_sum_q=info.max_abs_sum_q, warm_ms=info.warm_ms,
                     solve_ms=info.solve_ms, fell_back=info.fell_back,
                     frame_iters=list(fit), frame_rel_resid=list(frr))
        return q_out, stats

    def get_E(self, precision=PREC_F64):
        import torch
        dt = {PREC_F64: torch.float64, PREC_F32: torch.float32, PREC_BF16: torch.bfloat16}[precision]
        out = torch.empty((self.n, self.n), dtype=dt, device="cuda")
        _check(lib().cpm_get_E(self._h, precision, C.c_void_p(out.data_ptr()), self.n), "cpm_get_E")
        return out

    def get_E_block(self, row0, col0, rows, cols, precision=PREC_F64):
        """E[row0:row0+rows, col0:col0+cols] as a device tensor."""
        import torch
        dt = {PREC_F64: torch.float64, PREC_F32: torch.float32, PREC_BF16: torch.bfloat16}[precision]
        out = torch.empty((rows, cols), dtype=dt, device="cuda")
        _check(lib().cpm_get_E_block(self._h, precision, int(row0), int(col0), int(rows),
                                     int(cols), C.c_void_p(out.data_ptr()), int(cols)),
               "cpm_get_E_block")
        return out

    def dprime(self):
        import torch
        out = torch.empty((self.n,), dtype=torch.float64, device="cuda")
        c = C.c_double()
        _check(lib().cpm_get_dprime(self._h, _ptr(out), C.byref(c)), "cpm_get_dprime")
        return out, c.value

    def matvec(self, p, precision=PREC_F64):
        import torch
        v = torch.empty_like(p)
        _check(lib().cpm_matvec(self._h, precision, _ptr(p, torch.float64), int(p.shape[0]),
                                _ptr(v, torch.float64)), "cpm_matvec")
        return v

    def precond_dc(self, screening_g=0.083, rcut=8.0):
        """Build the PCG-DC preconditioner (Sec. III.B.2, Eq. 36)."""
        _check(lib().cpm_precond_dc(self._h, C.c_double(screening_g), C.c_double(rcut)),
               "cpm_precond_dc")

    def precond_sparse_inverse(self, rcut):
        """PCG-Normal / PCG-Full: E^-1 (from mi_build) sparsified at rcut."""
        _check(lib().cpm_precond_sparse_inverse(self._h, float(rcut)), "cpm_precond_sparse_inverse")

    def precond_gap(self, enable=True):
        """Eq. 37 fill of the current sparse preconditioner; returns p_gap."""
        g = C.c_double()
        _check(lib().cpm_precond_gap(self._h, 1 if enable else 0, C.byref(g)), "cpm_precond_gap")
        return g.value

    def precond_coarse(self, edge):
        """Coarse-space correction of the sparse preconditioner: patches of
        in-plane edge `edge` (A) per z-slab; edge <= 0 disables it. Returns
        the number of patches."""
        m = C.c_int64()
        _check(lib().cpm_precond_coarse(self._h, float(edge), C.byref(m)), "cpm_precond_coarse")
        return m.value

    def precond_apply(self, r):
        """z = P r for vectors r (F, N) on the device."""
        import torch
        z = torch.empty_like(r)
        _check(lib().cpm_precond_apply(self._h, _ptr(r, torch.float64), int(r.shape[0]),
                                       _ptr(z, torch.float64)), "cpm_precond_apply")
        return z

    def mi_build(self, tol=1e-13, max_iter=20000, precision=PREC_F64,
                 preconditioner=PRECOND_JACOBI):
        """Form S = E^-1 (I - 1 d^T) (Eq. 33) with the block solver."""
        o = SolveOpts(tol=tol, max_iter=max_iter, precision=precision, warm_start=WARM_ZERO,
                      inner_tol=1e-2, check_every=8, preconditioner=preconditioner)
        _check(lib().cpm_mi_build(self._h, C.byref(o)), "cpm_mi_build")

    def mi_solve(self, b, qsol, q_out=None):
        """q = S b - Q_sol d (Eq. 35) for frames b (F, N); asynchronous."""
        import torch
        if q_out is None:
            q_out = torch.empty_like(b)
        _check(lib().cpm_mi_solve(self._h, _ptr(b, torch.float64), _ptr(qsol, torch.float64),
                                  int(b.shape[0]), _ptr(q_out, torch.float64)), "cpm_mi_solve")
        return q_out

    def gcd_build(self, labels, m, tol=1e-12, max_iter=20000, precision=PREC_F64,
                  preconditioner=PRECOND_JACOBI, check_every=8, inner_tol=1e-3):
        """Capacitance coefficients C_E (Supplementary Eq. S22-S24) of the m
        electrodes given by labels (N,); returns (C_E, |C_E|, C(Q, -Q), stats)."""
        labels = np.ascontiguousarray(labels, dtype=np.int32)
        if labels.shape != (self.n,):
            raise ValueError(f"labels must have shape ({self.n},)")
        o = SolveOpts(tol=tol, max_iter=max_iter, precision=precision, warm_start=WARM_ZERO,
                      inner_tol=inner_tol, check_every=check_every, preconditioner=preconditioner)
        cmat = np.empty((int(m), int(m)), dtype=np.float64)
        det, joint = C.c_double(), C.c_double()
        info = SolveInfo()
        _check(lib().cpm_gcd_build(self._h, labels.ctypes.data, int(m), C.byref(o),
                                   cmat.ctypes.data, C.byref(det), C.byref(joint), C.byref(info)),
               "cpm_gcd_build")
        self._gcd_m = int(m)
        stats = dict(iterations=info.iterations, max_rel_resid=info.max_rel_resid,
                     solve_ms=info.solve_ms)
        return cmat, det.value, joint.value, stats

    def gcd_solve(self, b, Q, tol=1e-10, max_iter=5000, precision=PREC_F64,
                  preconditioner=PRECOND_JACOBI, check_every=8, inner_tol=1e-3, q_out=None,
                  dmu_out=None):
        """Charges (F, N) under prescribed electrode totals Q (F, M) (Eq. S15-S20),
        the multipliers Delta mu (F, M) and a dict of solve statistics."""
        import torch
        f = int(b.shape[0])
        m = getattr(self, "_gcd_m", None)
        if m is None:
            raise RuntimeError("gcd_build first")
        if tuple(b.shape) != (f, self.n) or tuple(Q.shape) != (f, m):
            raise ValueError(f"need b ({f}, {self.n}) and Q ({f}, {m})")
        if q_out is None:
            q_out = torch.empty_like(b)
        if dmu_out is None:
            dmu_out = torch.empty_like(Q)
        if tuple(q_out.shape) != (f, self.n) or tuple(dmu_out.shape) != (f, m):
            raise ValueError("output shapes do not match b and Q")
        o = SolveOpts(tol=tol, max_iter=max_iter, precision=precision, warm_start=WARM_ZERO,
                      inner_tol=inner_tol, check_every=check_every, preconditioner=preconditioner)
        info = SolveInfo()
        _check(lib().cpm_gcd_solve(self._h, _ptr(b, torch.float64), _ptr(Q, torch.float64), f,
                                   C.byref(o), _ptr(q_out, torch.float64),
                                   _ptr(dmu_out, torch.float64), C.byref(info)), "cpm_gcd_solve")
        stats = dict(iterations=info.iterations, max_rel_resid=info.max_rel_resid,
                     max_abs_sum_q=info.max_abs_sum_q, solve_ms=info.solve_ms)
        return q_out, dmu_out, stats

    def set_warm_chi(self, chi, tol=1e-12, max_iter=5000, preconditioner=PRECOND_JACOBI):
        import torch
        o = SolveOpts(tol=tol, max_iter=max_iter, precision=PREC_F64, warm_start=WARM_ZERO,
                      inner_tol=1e-3, check_every=8, preconditioner=preconditioner)
        _check(lib().cpm_set_warm_chi(self._h, _ptr(chi, torch.float64), C.byref(o)), "cpm_set_warm_chi")

    def warm_start(self, b, qsol, warm_start=WARM_MLP):
        """The solver's start x0 (F, N) and its FP64 residual r0 = b - E x0."""
        import torch
        x0 = torch.empty_like(b)
        r0 = torch.empty_like(b)
        _check(lib().cpm_warm_start(self._h, int(warm_start), _ptr(b, torch.float64),
                                    _ptr(qsol, torch.float64), int(b.shape[0]),
                                    _ptr(x0, torch.float64), _ptr(r0, torch.float64)),
               "cpm_warm_start")
        return x0, r0

    # ---- learned warm start
    def mlp_init(self, layer, n_layers, b_scale, r_scale, q_scale):
        layer = np.ascontiguousarray(layer, dtype=np.int32)
        _check(lib().cpm_mlp_init(self._h, layer.ctypes.data, int(n_layers), float(b_scale),
                                  float(r_scale), float(q_scale)), "cpm_mlp_init")

    def mlp_neighbours(self):
        out = np.empty((self.n, 12), dtype=np.int32)
        _check(lib().cpm_mlp_neighbours(self._h, out.ctypes.data), "cpm_mlp_neighbours")
        return out

    def mlp_set_params(self, params):
        params = np.ascontiguousarray(params, dtype=np.float32)
        assert params.size == MLP_NPARAM
        _check(lib().cpm_mlp_set_params(self._h, params.ctypes.data), "cpm_mlp_set_params")

    def mlp_get_params(self):
        out = np.empty(MLP_NPARAM, dtype=np.float32)
        _check(lib().cpm_mlp_get_params(self._h, out.ctypes.data), "cpm_mlp_get_params")
        return out

    def mlp_features(self, b):
        import torch
        out = torch.empty((b.shape[0] * self.n, MLP_IN), dtype=torch.float32, device=b.device)
        _check(lib().cpm_mlp_features(self._h, _ptr(b, torch.float64), int(b.shape[0]),
                                      _ptr(out, torch.float32)), "cpm_mlp_features")
        return out

    def mlp_forward(self, feat):
        import torch
        y = torch.empty((feat.shape[0],), dtype=torch.float32, device=feat.device)
        _check(lib().cpm_mlp_forward(self._h, _ptr(feat, torch.float32), int(feat.shape[0]),
                                     _ptr(y, torch.float32)), "cpm_mlp_forward")
        return y

    def mlp_loss_grad(self, feat, target):
        import torch
        g = torch.empty((MLP_NPARAM,), dtype=torch.float32, device=feat.device)
        loss = C.c_double()
        _check(lib().cpm_mlp_loss_grad(self._h, _ptr(feat, torch.float32), _ptr(target, torch.float32),
                                       int(feat.shape[0]), _ptr(g, torch.float32), C.byref(loss)),
               "cpm_mlp_loss_grad")
        return loss.value, g

    def mlp_train_step(self, feat, target, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        loss = C.c_double()
        _check(lib().cpm_mlp_train_step(self._h, _ptr(feat, torch.float32), _ptr(target, torch.float32),
                                        int(feat.shape[0]), lr, beta1, beta2, eps, C.byref(loss)),
               "cpm_mlp_train_step")
        return loss.value

    def mlp_train_epoch(self, b, q, perm, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        loss = C.c_double()
        _check(lib().cpm_mlp_train_epoch(self._h, _ptr(b, torch.float64), _ptr(q, torch.float64),
                                         int(b.shape[0]), _ptr(perm, torch.int64), int(batch), lr,
                                         beta1, beta2, eps, C.byref(loss)), "cpm_mlp_train_epoch")
        return loss.value
