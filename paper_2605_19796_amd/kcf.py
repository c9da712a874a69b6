"""ctypes binding of libkcf (argument marshalling only; every step runs in the HIP library).

Tensors are torch CUDA (ROCm) tensors used as device buffers; the context enqueues on the
current torch stream unless another stream is given. The library file is the in-tree
``libkcf.so`` built by ``paper_2605_19796_amd.build``; importing this module does not load
it, ``lib()`` does and raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkcf.so")

BOX, GAUSS = 0, 1
OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED, EIO = 0, -1, -2, -3, -4, -5


class KcfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kcf error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double)]


class Filter(C.Structure):
    _fields_ = [("kind", C.c_int), ("delta_over_h", C.c_int), ("precision", C.c_int)]


class Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in
                ("rho_bar", "ut", "tau", "grad", "tau_gm", "tau_smag", "k_sgs", "nu_t", "omega_t",
                 "q_crit")]


class ClosureParams(C.Structure):
    _fields_ = [("c_s", C.c_double), ("c_nu", C.c_double), ("theta", C.c_double),
                ("nu_mol", C.c_double), ("dt", C.c_double), ("gm_form", C.c_int),
                ("m2_mode", C.c_int), ("ksgs_rho_ref", C.c_int)]


class WidthStats(C.Structure):
    _fields_ = [("delta", C.c_double), ("m2", C.c_double), ("mean_rho_bar", C.c_double),
                ("ke_resolved", C.c_double), ("pi", C.c_double), ("pi_gm", C.c_double),
                ("pi_smag", C.c_double), ("corr_tau_gm", C.c_double * 6), ("corr_pi", C.c_double),
                ("mean_tau", C.c_double * 6), ("n_points", C.c_int64), ("n_nonfinite", C.c_int64),
                ("raw", C.c_double * 40)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


class CarrierStats(C.Structure):
    _fields_ = [("sgs_l2", C.c_double), ("err_l2", C.c_double), ("rel_err", C.c_double),
                ("hermite", C.c_double * 5), ("n_points", C.c_int64), ("n_nonfinite", C.c_int64),
                ("raw", C.c_double * 9)]

    as_dict = WidthStats.as_dict


class Moment3Stats(C.Structure):
    _fields_ = [("mean_m3", C.c_double * 10), ("rms_m3", C.c_double * 10),
                ("mean_theta_t", C.c_double), ("n_points", C.c_int64), ("n_nonfinite", C.c_int64),
                ("raw", C.c_double * 23)]

    as_dict = WidthStats.as_dict


class KcParams(C.Structure):
    _fields_ = [("nu", C.c_double), ("dt", C.c_double), ("theta", C.c_double),
                ("c_nu", C.c_double), ("rho_ref_one", C.c_int)]


class KcStats(C.Structure):
    _fields_ = [("corr", C.c_double * 6), ("rel_err", C.c_double), ("mean_m", C.c_double * 6),
                ("mean_tau", C.c_double * 6), ("mean_k", C.c_double), ("mean_k_exact", C.c_double),
                ("mean_omega", C.c_double), ("mean_omega_exact", C.c_double),
                ("clip", C.c_double), ("clip_exact", C.c_double), ("n_points", C.c_int64),
                ("n_nonfinite", C.c_int64), ("raw", C.c_double * 40)]

    as_dict = WidthStats.as_dict


class LbmParams(C.Structure):
    _fields_ = [("model", C.c_int), ("nu", C.c_double), ("c_nu", C.c_double)]


class LbmStats(C.Structure):
    _fields_ = [("mass", C.c_double), ("momentum", C.c_double * 3), ("kinetic_energy", C.c_double),
                ("mean_omega_sgs", C.c_double), ("clip_fraction", C.c_double),
                ("mean_k_sgs", C.c_double), ("n_nodes", C.c_int64), ("raw", C.c_double * 8)]

    as_dict = WidthStats.as_dict


LBM_BGK, LBM_KCRB, LBM_KCRB_RAW, LBM_KCMP, LBM_KCRR = range(5)
LBM_MODELS = {"bgk": LBM_BGK, "kcrb": LBM_KCRB, "kcrb_raw": LBM_KCRB_RAW, "kcmp": LBM_KCMP,
              "kcrr": LBM_KCRR}


class InputSummary(C.Structure):
    _fields_ = [("mean_rho", C.c_double), ("ek", C.c_double), ("enstrophy", C.c_double),
                ("n_nonfinite", C.c_int64)]


# exported symbol -> (restype, argtypes)
_SIGS = {
    "kcf_version": (C.c_int, []),
    "kcf_last_error": (C.c_char_p, []),
    "kcf_ctx_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "kcf_ctx_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "kcf_ctx_destroy": (None, [C.c_void_p]),
    "kcf_ctx_enable_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "kcf_ctx_kernel_ms": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "kcf_ctx_kernel_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_int,
                                       C.POINTER(C.c_int)]),
    "kcf_filter_taps": (C.c_int, [C.c_int, C.c_int, C.c_double, C.POINTER(C.c_float), C.c_int,
                                  C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "kcf_filter_favre": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.POINTER(Filter), C.c_int,
                                   C.c_void_p, C.c_void_p, C.POINTER(Outputs),
                                   C.POINTER(ClosureParams), C.POINTER(WidthStats)]),
    "kcf_filter_favre_noalloc": (C.c_int, [C.POINTER(Grid), C.POINTER(Filter), C.c_int,
                                           C.c_void_p, C.c_void_p, C.POINTER(Outputs),
                                           C.POINTER(ClosureParams), C.POINTER(WidthStats),
                                           C.c_int, C.c_void_p]),
    "kcf_grad_closure": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_double, C.c_double, C.POINTER(ClosureParams),
                                   C.POINTER(Outputs), C.POINTER(WidthStats)]),
    "kcf_sgs_carrier": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.POINTER(Filter), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(CarrierStats)]),
    "kcf_sgs_moment3": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.POINTER(Filter), C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.POINTER(Moment3Stats)]),
    "kcf_kc_mp": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.POINTER(Filter), C.c_void_p,
                            C.c_void_p, C.POINTER(KcParams), C.c_void_p, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_void_p, C.POINTER(KcStats)]),
    "kcf_lbm_equilibrium": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.c_void_p, C.c_void_p,
                                      C.c_void_p]),
    "kcf_lbm_step": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.POINTER(LbmParams), C.c_void_p,
                               C.c_void_p, C.POINTER(LbmStats)]),
    "kcf_input_stats": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.c_void_p, C.c_void_p,
                                  C.POINTER(InputSummary)]),
    "kcf_reduce_check": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                   C.POINTER(C.c_double)]),
    "kcf_stream_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                   C.c_int64]),
    "kcf_mlp_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "kcf_mlp_destroy": (None, [C.c_void_p]),
    "kcf_mlp_set_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "kcf_mlp_get_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "kcf_mlp_set_norm": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "kcf_mlp_get_norm": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "kcf_mlp_step_count": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "kcf_mlp_features": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_double, C.c_void_p, C.c_void_p]),
    "kcf_mlp_column_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "kcf_mlp_fit_norm": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64]),
    "kcf_mlp_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_int, C.c_float, C.c_void_p]),
    "kcf_mlp_grads": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int,
                                C.POINTER(C.c_float), C.POINTER(C.c_double)]),
    "kcf_mlp_predict": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "kcf_mlp_infer_field": (C.c_int, [C.c_void_p, C.POINTER(Grid), C.c_void_p, C.c_void_p,
                                      C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_int64)]),
    "kcf_mlp_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "kcf_mlp_load": (C.c_int, [C.c_void_p, C.c_char_p]),
}

_lib = None


def lib():
    """Load libkcf.so (in-tree). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run python -m paper_2605_19796_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def check(rc):
    if rc != OK:
        raise KcfError(rc, lib().kcf_last_error().decode())
    return rc


def filter_taps(kind, delta_over_h, h):
    """Host-side taps of the GPU filter: (float32 list w, radius R, second moment M2)."""
    buf = (C.c_float * 129)()
    R = C.c_int()
    m2 = C.c_double()
    check(lib().kcf_filter_taps(kind, delta_over_h, h, buf, 129, C.byref(R), C.byref(m2)))
    return [buf[i] for i in range(2 * R.value + 1)], R.value, m2.value


def _ptr(t, dtype=None):
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if t.dtype != (dtype or torch.float32):
        raise ValueError(f"expected {dtype or torch.float32}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _need(*specs):
    """Checks (tensor, numel, name) triples: each tensor that is given must hold exactly numel
    elements. Every wrapper runs this on all its tensors before it takes a pointer or calls
    the library, so a mismatched buffer never reaches a kernel."""
    for t, numel, name in specs:
        if t is not None and t.numel() != numel:
            raise ValueError(f"{name}: expected {numel} elements, got {t.numel()} (shape "
                             f"{tuple(t.shape)})")


def _sized(t, numel, name, dtype=None):
    """Device pointer of t after its size check (None stays None)."""
    _need((t, numel, name))
    return _ptr(t, dtype)


def _grid3(t, name="rho"):
    """(nz, ny, nx) of a scalar field given as (nz, ny, nx) or (1, nz, ny, nx)."""
    if t is None or t.dim() not in (3, 4) or (t.dim() == 4 and t.shape[0] != 1):
        raise ValueError(f"{name}: expected a (nz, ny, nx) field")
    return tuple(int(v) for v in t.shape[-3:])


def params(c_s=0.11, c_nu=0.02, theta=1.0, nu_mol=0.0, dt=0.0, gm_form=0, m2_mode=0,
           ksgs_rho_ref=0):
    return ClosureParams(c_s, c_nu, theta, nu_mol, dt, gm_form, m2_mode, ksgs_rho_ref)


OUT_SIZES = dict(rho_bar=1, ut=3, tau=6, grad=9, tau_gm=6, tau_smag=6, k_sgs=1, nu_t=1, omega_t=1,
                 q_crit=1)


def alloc_outputs(shape, device, fields=("rho_bar", "ut", "tau", "grad", "tau_gm")):
    """Device tensors for the requested outputs: dict name -> tensor (comp, nz, ny, nx)."""
    import torch
    nz, ny, nx = shape
    return {f: torch.empty((OUT_SIZES[f], nz, ny, nx), dtype=torch.float32, device=device)
            for f in fields}


def filter_favre_noalloc(rho, u, h, filters, outs, cp=None, stats=True, device=0, stream=None):
    """kcf_filter_favre_noalloc: the box path of Context.filter_favre without a context and
    without device allocation (see include/kcf.h); same arguments and results."""
    import torch
    nz, ny, nx = _grid3(rho)
    n = nx * ny * nz
    nf = len(filters)
    if not 1 <= nf <= 4:
        raise ValueError(f"1 to 4 filters per call, got {nf}")
    if len(outs) != nf:
        raise ValueError(f"{nf} filters but {len(outs)} output sets")
    _need((rho, n, "rho"), (u, 3 * n, "u"))
    for o in outs:
        _outputs_need(o, n)
    g = Grid(nx, ny, nz, h)
    fa = (Filter * nf)(*[Filter(*f) if len(f) == 3 else Filter(f[0], f[1], 0) for f in filters])
    oa = (Outputs * nf)(*[_outputs_struct(o, n) for o in outs])
    pr, pu = _ptr(rho), _ptr(u)
    if stream is None:
        stream = torch.cuda.current_stream(device)
    st = (WidthStats * nf)() if stats else None
    check(lib().kcf_filter_favre_noalloc(C.byref(g), fa, nf, pr, pu, oa,
                                         C.byref(cp) if cp is not None else None, st, device,
                                         C.c_void_p(stream.cuda_stream)))
    return [s.as_dict() for s in st] if stats else None


def _outputs_need(d, n):
    """Size checks of an output dict name -> tensor on a grid of n points."""
    if d:
        bad = set(d) - set(OUT_SIZES)
        if bad:
            raise ValueError(f"unknown output fields {sorted(bad)}")
        _need(*[(t, OUT_SIZES[k] * n, k) for k, t in d.items()])


def _outputs_struct(d, n=None):
    """Outputs struct of a dict name -> tensor; with n (points of the grid) every tensor must
    hold OUT_SIZES[name] * n elements."""
    if n is not None:
        _outputs_need(d, n)
    o = Outputs()
    for name in OUT_SIZES:
        t = d.get(name) if d else None
        p = _ptr(t)
        setattr(o, name, p.value if p is not None else None)
    return o


class Context:
    """A libkcf context bound to one device and stream."""

    def __init__(self, device=0, stream=None):
        import torch
        self._lib = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        check(self._lib.kcf_ctx_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)))
        self.handle = h
        self._children = []  # weak references to MLPs that use this context

    def close(self):
        """Destroys the context after every MLP created on it (they must not outlive it)."""
        if self.handle:
            for ref in self._children:
                m = ref()
                if m is not None:
                    m.close()
            self._children = []
            self._lib.kcf_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def enable_timing(self, on=True):
        check(self._lib.kcf_ctx_enable_timing(self.handle, 1 if on else 0))

    def kernel_ms(self):
        ms = C.c_double()
        n = C.c_int()
        check(self._lib.kcf_ctx_kernel_ms(self.handle, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def kernel_times(self, cap=4096):
        """Per-launch times (ms) of the timed launches since the last reset, in launch order."""
        buf = (C.c_float * cap)()
        n = C.c_int()
        check(self._lib.kcf_ctx_kernel_times(self.handle, buf, cap, C.byref(n)))
        return list(buf[:n.value])

    def filter_favre(self, rho, u, h, filters, outs, cp=None, stats=True):
        """rho (nz,ny,nx), u (3,nz,ny,nx) device float32; filters: list of (kind, n[, precision]);
        outs: list (one per filter) of dicts name -> tensor. Returns list of stats dicts."""
        nz, ny, nx = _grid3(rho)
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        nf = len(filters)
        if not 1 <= nf <= 4:
            raise ValueError(f"1 to 4 filters per call, got {nf}")
        if len(outs) != nf:
            raise ValueError(f"{nf} filters but {len(outs)} output sets")
        _need((rho, n, "rho"), (u, 3 * n, "u"))
        for o in outs:
            _outputs_need(o, n)
        fa = (Filter * nf)(*[Filter(*f) if len(f) == 3 else Filter(f[0], f[1], 0) for f in filters])
        oa = (Outputs * nf)(*[_outputs_struct(o, n) for o in outs])
        pr, pu = _sized(rho, n, "rho"), _sized(u, 3 * n, "u")
        st = (WidthStats * nf)() if stats else None
        check(self._lib.kcf_filter_favre(self.handle, C.byref(g), fa, nf, pr, pu, oa,
                                         C.byref(cp) if cp is not None else None, st))
        return [s.as_dict() for s in st] if stats else None

    def grad_closure(self, rho_bar, ut, tau, h, delta, m2, outs, cp=None, stats=True):
        nz, ny, nx = _grid3(rho_bar, "rho_bar")
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        _need((rho_bar, n, "rho_bar"), (ut, 3 * n, "ut"), (tau, 6 * n, "tau"))
        o = _outputs_struct(outs, n)
        pr, pu, pt = _sized(rho_bar, n, "rho_bar"), _sized(ut, 3 * n, "ut"), _sized(tau, 6 * n, "tau")
        st = WidthStats() if stats else None
        check(self._lib.kcf_grad_closure(self.handle, C.byref(g), pr, pu, pt,
                                         delta, m2, C.byref(cp) if cp is not None else None,
                                         C.byref(o), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def sgs_carrier(self, rho, u, h, filt, f_sgs=None, f_h2=None, stats=True):
        """D3Q27 SGS carrier of one filter (kind, n[, precision]): f_sgs and f_h2 are optional
        (27, nz, ny, nx) device float32 tensors; returns the statistics dict or None."""
        nz, ny, nx = _grid3(rho)
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        fl = Filter(*filt) if len(filt) == 3 else Filter(filt[0], filt[1], 0)
        _need((rho, n, "rho"), (u, 3 * n, "u"), (f_sgs, 27 * n, "f_sgs"), (f_h2, 27 * n, "f_h2"))
        ptrs = (_sized(rho, n, "rho"), _sized(u, 3 * n, "u"), _sized(f_sgs, 27 * n, "f_sgs"),
                _sized(f_h2, 27 * n, "f_h2"))
        st = CarrierStats() if stats else None
        check(self._lib.kcf_sgs_carrier(self.handle, C.byref(g), C.byref(fl), *ptrs,
                                        C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def sgs_moment3(self, rho, u, h, filt, theta=None, m3=None, theta_t=None, stats=True):
        """Third-order SGS moment of one filter (kind, n[, precision]): m3 is an optional
        (10, nz, ny, nx) device float32 tensor, theta_t an optional (nz, ny, nx) one (needs
        theta); returns the statistics dict or None."""
        nz, ny, nx = _grid3(rho)
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        fl = Filter(*filt) if len(filt) == 3 else Filter(filt[0], filt[1], 0)
        _need((rho, n, "rho"), (u, 3 * n, "u"), (theta, n, "theta"), (m3, 10 * n, "m3"),
              (theta_t, n, "theta_t"))
        ptrs = (_sized(rho, n, "rho"), _sized(u, 3 * n, "u"), _sized(theta, n, "theta"),
                _sized(m3, 10 * n, "m3"), _sized(theta_t, n, "theta_t"))
        st = Moment3Stats() if stats else None
        check(self._lib.kcf_sgs_moment3(self.handle, C.byref(g), C.byref(fl), *ptrs,
                                        C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def kc_mp(self, rho, u, h, filt, nu, dt=0.0, theta=1.0, c_nu=0.035, rho_ref_one=1,
              m_sgs=None, m_ce=None, k_sgs=None, nu_t_eff=None, omega_sgs=None, stats=True):
        """A priori KC-MP SGS moment and relaxation-rate field of one filter (kind, n[,
        precision]); outputs are optional device float32 tensors ((6, nz, ny, nx) for m_sgs and m_ce,
        (nz, ny, nx) for the rates). Returns the statistics dict or None."""
        nz, ny, nx = _grid3(rho)
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        fl = Filter(*filt) if len(filt) == 3 else Filter(filt[0], filt[1], 0)
        kp = KcParams(nu, dt, theta, c_nu, rho_ref_one)
        _need((rho, n, "rho"), (u, 3 * n, "u"), (m_sgs, 6 * n, "m_sgs"), (m_ce, 6 * n, "m_ce"),
              (k_sgs, n, "k_sgs"), (nu_t_eff, n, "nu_t_eff"), (omega_sgs, n, "omega_sgs"))
        pr, pu = _sized(rho, n, "rho"), _sized(u, 3 * n, "u")
        outs = (_sized(m_sgs, 6 * n, "m_sgs"), _sized(m_ce, 6 * n, "m_ce"),
                _sized(k_sgs, n, "k_sgs"), _sized(nu_t_eff, n, "nu_t_eff"),
                _sized(omega_sgs, n, "omega_sgs"))
        st = KcStats() if stats else None
        check(self._lib.kcf_kc_mp(self.handle, C.byref(g), C.byref(fl), pr, pu, C.byref(kp), *outs,
                                  C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def lbm_equilibrium(self, rho, u, f_out=None):
        """Equilibrium populations (27, nz, ny, nx) of rho (nz, ny, nx) and u (3, nz, ny, nx),
        lattice units."""
        import torch
        nz, ny, nx = _grid3(rho)
        n = nx * ny * nz
        _need((rho, n, "rho"), (u, 3 * n, "u"), (f_out, 27 * n, "f_out"))
        if f_out is None:
            f_out = torch.empty((27, nz, ny, nx), dtype=torch.float32, device=rho.device)
        g = Grid(nx, ny, nz, 1.0)
        check(self._lib.kcf_lbm_equilibrium(self.handle, C.byref(g), _ptr(rho), _ptr(u),
                                            _ptr(f_out)))
        return f_out

    def lbm_step(self, f_in, f_out, model, nu, c_nu, stats=True):
        """One D3Q27 collide-and-stream step f_in -> f_out ((27, nz, ny, nx) device float32,
        distinct); model is a name of LBM_MODELS or its number. Returns the statistics of the
        state f_in (dict) or None."""
        if f_in is None or f_in.dim() != 4 or f_in.shape[0] != 27:
            raise ValueError("f_in: expected a (27, nz, ny, nx) tensor")
        nz, ny, nx = (int(v) for v in f_in.shape[1:])
        n = nx * ny * nz
        _need((f_out, 27 * n, "f_out"))
        if f_out is None or f_out.data_ptr() == f_in.data_ptr():
            raise ValueError("f_out must be a distinct buffer")
        m = LBM_MODELS[model] if isinstance(model, str) else int(model)
        g = Grid(nx, ny, nz, 1.0)
        p = LbmParams(m, nu, c_nu)
        st = LbmStats() if stats else None
        check(self._lib.kcf_lbm_step(self.handle, C.byref(g), C.byref(p), _ptr(f_in), _ptr(f_out),
                                     C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def input_stats(self, rho, u, h):
        nz, ny, nx = _grid3(rho)
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        _need((rho, n, "rho"), (u, 3 * n, "u"))
        pr, pu = _sized(rho, n, "rho"), _sized(u, 3 * n, "u")
        s = InputSummary()
        check(self._lib.kcf_input_stats(self.handle, C.byref(g), pr, pu, C.byref(s)))
        return dict(mean_rho=s.mean_rho, ek=s.ek, enstrophy=s.enstrophy, n_nonfinite=s.n_nonfinite)

    def stream_probe(self, inp, out):
        """kcf_stream_probe on inp (nin, ...) and out (nout, ...) blocks of equal size."""
        nin, nout = int(inp.shape[0]), int(out.shape[0])
        n = inp[0].numel()
        _need((inp, nin * n, "in"), (out, nout * n, "out"))
        check(self._lib.kcf_stream_probe(self.handle, _ptr(inp), nin, _ptr(out), nout, n))

    def reduce_check(self, a, b=None):
        out = (C.c_double * 3)()
        _need((b, a.numel(), "b"))
        pa, pb = _ptr(a), _ptr(b)
        check(self._lib.kcf_reduce_check(self.handle, pa, pb, a.numel(), out))
        return list(out)


N_PARAMS = 9670
N_NORM = 68


def _rows(x, ncol, name):
    """Row count of an (n, ncol) matrix, checked."""
    if x is None or x.dim() != 2 or x.shape[1] != ncol or x.shape[0] < 1:
        raise ValueError(f"{name}: expected an (n, {ncol}) matrix, got "
                         f"{None if x is None else tuple(x.shape)}")
    return int(x.shape[0])


def _f32(a, n):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32).ravel()
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


class MLP:
    """Learned-closure network state on the GPU (see include/kcf.h)."""

    def __init__(self, ctx: Context):
        import weakref
        self.ctx = ctx
        self._lib = ctx._lib
        h = C.c_void_p()
        check(self._lib.kcf_mlp_create(ctx.handle, C.byref(h)))
        self.handle = h
        ctx._children.append(weakref.ref(self))

    def close(self):
        if self.handle:
            self._lib.kcf_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        a, ptr = _f32(params, N_PARAMS)
        check(self._lib.kcf_mlp_set_params(self.handle, ptr))

    def get_params(self):
        import numpy as np
        a = np.empty(N_PARAMS, dtype=np.float32)
        check(self._lib.kcf_mlp_get_params(self.handle, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def set_norm(self, norm):
        a, ptr = _f32(norm, N_NORM)
        check(self._lib.kcf_mlp_set_norm(self.handle, ptr))

    def get_norm(self):
        import numpy as np
        a = np.empty(N_NORM, dtype=np.float32)
        check(self._lib.kcf_mlp_get_norm(self.handle, a.ctypes.data_as(C.POINTER(C.c_float))))
        return a

    def step_count(self):
        s = C.c_int64()
        check(self._lib.kcf_mlp_step_count(self.handle, C.byref(s)))
        return s.value

    def fit_norm(self, x, y):
        n = _rows(x, 14, "x")
        _need((y, 6 * n, "y"))
        px, py = _ptr(x), _ptr(y)
        check(self._lib.kcf_mlp_fit_norm(self.handle, px, py, n))

    def _batch(self, x, y, idx, batch):
        import torch
        n = _rows(x, 14, "x")
        _need((y, 6 * n, "y"))
        if batch <= 0 or (idx is None and batch > n):
            raise ValueError(f"batch {batch} outside 1..{n}")
        if idx is not None and idx.numel() < batch:
            raise ValueError(f"idx: {idx.numel()} indices for a batch of {batch}")
        return n, _ptr(y), _ptr(idx, torch.int32)

    def train_step(self, x, y, idx, batch, lr, loss_out=None):
        _need((loss_out, 1, "loss_out"))
        n, py, pi = self._batch(x, y, idx, batch)
        px, pl = _ptr(x), _ptr(loss_out)
        check(self._lib.kcf_mlp_train_step(self.handle, px, py, n, pi, batch, lr, pl))

    def grads(self, x, y, idx, batch):
        import numpy as np
        n, py, pi = self._batch(x, y, idx, batch)
        px = _ptr(x)
        g = np.empty(N_PARAMS, dtype=np.float32)
        loss = C.c_double()
        check(self._lib.kcf_mlp_grads(self.handle, px, py, n, pi,
                                      batch, g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)))
        return loss.value, g

    def predict(self, x):
        import torch
        n = _rows(x, 14, "x")
        px = _ptr(x)
        y = torch.empty((n, 6), dtype=torch.float32, device=x.device)
        check(self._lib.kcf_mlp_predict(self.handle, px, n, _ptr(y)))
        return y

    def infer_field(self, rho_bar, ut, h, delta, m2, tau_out=None, mask_out=None, count=True):
        import torch
        nz, ny, nx = _grid3(rho_bar, "rho_bar")
        n = nx * ny * nz
        g = Grid(nx, ny, nz, h)
        _need((rho_bar, n, "rho_bar"), (ut, 3 * n, "ut"), (tau_out, 6 * n, "tau_out"),
              (mask_out, (n + 15) // 16, "mask_out"))
        if tau_out is None:
            tau_out = torch.empty((6, nz, ny, nx), dtype=torch.float32, device=rho_bar.device)
        ptrs = (_sized(rho_bar, n, "rho_bar"), _sized(ut, 3 * n, "ut"))
        pt = _sized(tau_out, 6 * n, "tau_out")
        pm = _sized(mask_out, (n + 15) // 16, "mask_out", torch.int16)
        nfb = C.c_int64()
        check(self._lib.kcf_mlp_infer_field(self.handle, C.byref(g), *ptrs, delta, m2, pt, pm,
                                            C.byref(nfb) if count else None))
        return tau_out, (nfb.value if count else None)

    def save(self, path):
        check(self._lib.kcf_mlp_save(self.handle, os.fsencode(path)))

    def load(self, path):
        check(self._lib.kcf_mlp_load(self.handle, os.fsencode(path)))


def mlp_features(ctx, rho_bar, ut, tau, h, delta, with_targets=True):
    """Network inputs (N, 14) and targets (N, 6) of every grid point (device tensors)."""
    import torch
    nz, ny, nx = _grid3(rho_bar, "rho_bar")
    n = nx * ny * nz
    g = Grid(nx, ny, nz, h)
    _need((rho_bar, n, "rho_bar"), (ut, 3 * n, "ut"), (tau, 6 * n, "tau"))
    pr, pu = _sized(rho_bar, n, "rho_bar"), _sized(ut, 3 * n, "ut")
    pt = _sized(tau, 6 * n, "tau") if with_targets else None
    if with_targets and pt is None:
        raise ValueError("targets need tau")
    x = torch.empty((n, 14), dtype=torch.float32, device=rho_bar.device)
    y = torch.empty((n, 6), dtype=torch.float32, device=rho_bar.device) if with_targets else None
    check(ctx._lib.kcf_mlp_features(ctx.handle, C.byref(g), pr, pu, pt, delta, _ptr(x), _ptr(y)))
    return x, y


def column_stats(ctx, X):
    if X.dim() != 2 or not 1 <= X.shape[1] <= 32:
        raise ValueError(f"X: expected an (n, ncol <= 32) matrix, got {tuple(X.shape)}")
    ncol = X.shape[1]
    arrs = [(C.c_double * ncol)() for _ in range(4)]
    check(ctx._lib.kcf_mlp_column_stats(ctx.handle, _ptr(X), X.shape[0], ncol, *arrs))
    return [list(a) for a in arrs]
