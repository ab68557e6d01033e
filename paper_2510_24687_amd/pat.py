"""Thin ctypes binding of ``libpat.so`` (the C ABI declared in include/pat.h).

Only argument marshalling lives here: every step of A and A* runs in the HIP
kernels of the library.  PyTorch supplies device memory and the current HIP
stream.  If the library is not built, or no GPU is present, calls raise --
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpat.so")
_lib = None

PAT_F32, PAT_F64 = 0, 1


class Geometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("a", ctypes.c_double), ("R", ctypes.c_double),
                ("c", ctypes.c_double), ("m", ctypes.c_int), ("theta0", ctypes.c_double),
                ("arc", ctypes.c_double), ("nt", ctypes.c_int), ("T", ctypes.c_double),
                ("taper_rho", ctypes.c_double), ("mask_radius", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("m", ctypes.c_int), ("nt", ctypes.c_int), ("m_full", ctypes.c_int),
                ("grid", ctypes.c_int), ("stencil", ctypes.c_int), ("rings", ctypes.c_int),
                ("dct_half", ctypes.c_int), ("kmax", ctypes.c_int), ("kpad", ctypes.c_int),
                ("klow", ctypes.c_int), ("lcorr", ctypes.c_int), ("ring_points", ctypes.c_int),
                ("max_ring", ctypes.c_int), ("spread_tiles", ctypes.c_int),
                ("dlam", ctypes.c_double), ("period", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("ws_per_image", ctypes.c_size_t), ("table_bytes", ctypes.c_size_t),
                ("tune_fft_radix_log2", ctypes.c_int), ("tune_cols_per_block", ctypes.c_int),
                ("tune_dct_cols_per_block", ctypes.c_int), ("tune_ring_images", ctypes.c_int),
                ("tune_spread_images", ctypes.c_int), ("tune_twiddle_table", ctypes.c_int),
                ("tune_spread_staged", ctypes.c_int), ("tune_dct_wave", ctypes.c_int),
                ("tune_wave_fft", ctypes.c_int), ("tuned", ctypes.c_int),
                ("tuned_ms", ctypes.c_double)]


EXPORTED = ["pat_plan_create", "pat_plan_query", "pat_plan_destroy", "pat_plan_get_info",
            "pat_workspace_size", "pat_forward", "pat_adjoint", "pat_forward_batched",
            "pat_adjoint_batched", "pat_inverse", "pat_inverse_batched", "pat_adjoint_scale", "pat_status_string", "pat_last_error",
            "pat_debug_bessel", "pat_axpby", "pat_conv_packed_size", "pat_conv_pack_weights", "pat_conv3x3",
            "pat_conv_wgrad_partials", "pat_conv3x3_wgrad", "pat_conv_bwd_partials", "pat_plane_sum", "pat_adam", "pat_opnorm_estimate",
            "pat_group_create", "pat_group_destroy", "pat_group_forward", "pat_group_adjoint",
            "pat_filter_length", "pat_filter_create", "pat_filter_destroy", "pat_filter_apply",
            "pat_gconv_packed_size", "pat_gconv_pack", "pat_gconv", "pat_gconv_wgrad_partials", "pat_gconv_wgrad",
            "pat_bn_partials", "pat_bn_forward", "pat_bn_backward", "pat_maxpool2", "pat_maxpool2_backward",
            "pat_nhwc_pack", "pat_nhwc_unpack_grad", "pat_head_forward", "pat_head_partials", "pat_head_backward",
            "pat_dot_batched", "pat_dot_batched_noalloc", "pat_forward_residual", "pat_forward_cp_dual",
            "pat_adjoint_nnls", "pat_adjoint_cp_primal", "pat_timing_start", "pat_timing_start_stages",
            "pat_timing_stop"]


class ConvDesc(ctypes.Structure):
    """pat_conv_desc: one 3x3 convolution between planar / NHWC FP32 tensors."""
    _fields_ = [("B", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int), ("cin", ctypes.c_int),
                ("cout", ctypes.c_int), ("in_planar", ctypes.c_int), ("out_planar", ctypes.c_int),
                ("inp", ctypes.c_void_p * 4), ("out", ctypes.c_void_p * 4), ("residual", ctypes.c_void_p * 4),
                ("scale", ctypes.c_float * 4), ("weight", ctypes.c_void_p), ("bias", ctypes.c_void_p),
                ("alpha", ctypes.c_void_p), ("pre", ctypes.c_void_p), ("bwd_pre", ctypes.c_void_p),
                ("partials", ctypes.c_void_p), ("grad_bias_alpha", ctypes.c_void_p), ("accumulate", ctypes.c_int)]


class GConvDesc(ctypes.Structure):
    """pat_gconv_desc: one implicit-GEMM convolution between NHWC tensors."""
    _fields_ = [("B", ctypes.c_int), ("H", ctypes.c_int), ("W", ctypes.c_int),
                ("src", ctypes.c_void_p * 2), ("csrc", ctypes.c_int * 2),
                ("Hs", ctypes.c_int), ("Ws", ctypes.c_int), ("in_stride", ctypes.c_int), ("ntaps", ctypes.c_int),
                ("dy", ctypes.c_int * 9), ("dx", ctypes.c_int * 9), ("weight", ctypes.c_void_p),
                ("cout", ctypes.c_int), ("dst", ctypes.c_void_p * 2), ("cdst", ctypes.c_int * 2),
                ("dst_bf16", ctypes.c_int * 2), ("accumulate", ctypes.c_int * 2),
                ("Ho", ctypes.c_int), ("Wo", ctypes.c_int), ("out_stride", ctypes.c_int), ("oy", ctypes.c_int),
                ("ox", ctypes.c_int)]


def load():
    """Load libpat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpat.so is not built (run __graft_entry__.build() or "
                           "python paper_2510_24687_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, L, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_size_t
    gp = ctypes.POINTER(Geometry)
    lib.pat_plan_create.argtypes = [ctypes.POINTER(vp), gp, i, i, ctypes.c_char_p]
    lib.pat_plan_query.argtypes = [gp, i, ctypes.POINTER(PlanInfo)]
    lib.pat_plan_destroy.argtypes = [vp]
    lib.pat_plan_get_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    lib.pat_workspace_size.argtypes = [vp, i, ctypes.POINTER(sz)]
    lib.pat_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.pat_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.pat_forward_batched.argtypes = [vp, i, vp, L, vp, L, vp, vp]
    lib.pat_adjoint_batched.argtypes = [vp, i, vp, L, vp, L, vp, vp]
    lib.pat_inverse.argtypes = [vp, vp, vp, vp, vp]
    lib.pat_inverse_batched.argtypes = [vp, i, vp, L, vp, L, vp, vp]
    lib.pat_filter_length.argtypes = [i, ctypes.POINTER(i)]
    lib.pat_filter_create.argtypes = [ctypes.POINTER(vp), i, ctypes.c_double, i, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double), i, i]
    lib.pat_filter_destroy.argtypes = [vp]
    lib.pat_filter_apply.argtypes = [vp, i, i, vp, L, vp, L, vp]
    lib.pat_adjoint_scale.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.pat_status_string.argtypes = [i]
    lib.pat_status_string.restype = ctypes.c_char_p
    lib.pat_last_error.restype = ctypes.c_char_p
    lib.pat_debug_bessel.argtypes = [ctypes.c_double, i, ctypes.POINTER(ctypes.c_double)]
    D = ctypes.c_double
    lib.pat_axpby.argtypes = [vp, L, D, vp, D, vp, vp, vp]
    cd = ctypes.POINTER(ConvDesc)
    lib.pat_conv_packed_size.argtypes = [i, i, i]
    lib.pat_conv_packed_size.restype = L
    lib.pat_conv_pack_weights.argtypes = [vp, i, i, i, i, vp, vp]
    lib.pat_conv3x3.argtypes = [cd, vp]
    lib.pat_conv_wgrad_partials.argtypes = [cd, i]
    lib.pat_conv_wgrad_partials.restype = L
    lib.pat_conv3x3_wgrad.argtypes = [cd, vp, i, vp, vp, i, vp]
    lib.pat_conv_bwd_partials.argtypes = [cd]
    lib.pat_conv_bwd_partials.restype = L
    lib.pat_plane_sum.argtypes = [L, vp, vp, i, vp, i, vp]
    lib.pat_adam.argtypes = [L, vp, vp, vp, vp, vp, D, D, i, D, D, D, D, vp, vp]
    lib.pat_opnorm_estimate.argtypes = [vp, i, ctypes.POINTER(D), vp, vp]
    lib.pat_group_create.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(vp)]
    lib.pat_group_destroy.argtypes = [vp]
    ip, vpp = ctypes.POINTER(i), ctypes.POINTER(vp)
    lib.pat_group_forward.argtypes = [vp, ip, vpp, vpp, vpp, vp]
    lib.pat_group_adjoint.argtypes = [vp, ip, vpp, vpp, vpp, vp]
    gd = ctypes.POINTER(GConvDesc)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.pat_gconv_packed_size.argtypes = [i, i, i]
    lib.pat_gconv_packed_size.restype = L
    lib.pat_gconv_pack.argtypes = [vp, i, i, i, i, i, L, L, L, L, i, vp, vp]
    lib.pat_gconv.argtypes = [gd, vp]
    lib.pat_gconv_wgrad_partials.argtypes = [gd, i]
    lib.pat_gconv_wgrad_partials.restype = L
    lib.pat_gconv_wgrad.argtypes = [gd, vp, i, vp, vp, i, L, L, L, L, i, vp]
    lib.pat_bn_partials.argtypes = [L, i]
    lib.pat_bn_partials.restype = L
    lib.pat_bn_forward.argtypes = [L, i, vp, vp, vp, vp, vp, vp, vp, D, D, i, vp, vp, vp]
    lib.pat_bn_backward.argtypes = [L, i, vp, vp, vp, vp, vp, vp, vp, vp, vp, i, vp, vp]
    lib.pat_maxpool2.argtypes = [i, i, i, i, vp, vp, vp]
    lib.pat_maxpool2_backward.argtypes = [i, i, i, i, vp, vp, vp, vp]
    lib.pat_nhwc_pack.argtypes = [L, i, i, vpp, fp, vp, vp]
    lib.pat_nhwc_unpack_grad.argtypes = [L, i, i, vp, fp, vpp, vpp, vp]
    lib.pat_head_forward.argtypes = [L, i, vp, vp, vp, vp, vp, vp]
    lib.pat_head_partials.argtypes = [L, i]
    lib.pat_head_partials.restype = L
    lib.pat_head_backward.argtypes = [L, i, vp, vp, vp, vp, vp, i, vp, vp]
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != 0:
        lib = load()
        raise RuntimeError("%s failed: %s (%s)" % (what, lib.pat_status_string(rc).decode(),
                                                    lib.pat_last_error().decode()))


GEOM_DEFAULTS = dict(a=1.0, R=1.0, c=1.0, theta0=0.0, arc=2 * math.pi, T=2.0, rho=0.8, mask_radius=0.0)


def make_geometry(geom: dict) -> Geometry:
    g = dict(GEOM_DEFAULTS)
    g.update(geom)
    return Geometry(int(g["n"]), float(g["a"]), float(g["R"]), float(g["c"]), int(g["m"]),
                    float(g["theta0"]), float(g["arc"]), int(g["nt"]), float(g["T"]),
                    float(g.get("taper_rho", g["rho"])), float(g["mask_radius"]))


def _info_dict(info: PlanInfo) -> dict:
    return {name: getattr(info, name) for name, _ in PlanInfo._fields_}


def plan_query(geom: dict, dtype: str = "f32") -> dict:
    """Parameters the library would choose for this geometry (host only)."""
    lib = load()
    info = PlanInfo()
    _check(lib.pat_plan_query(ctypes.byref(make_geometry(geom)), PAT_F64 if dtype == "f64" else PAT_F32,
                              ctypes.byref(info)), "pat_plan_query")
    return _info_dict(info)


def debug_bessel(x: float, K: int) -> np.ndarray:
    lib = load()
    out = np.zeros(K + 1)
    _check(lib.pat_debug_bessel(float(x), int(K), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "pat_debug_bessel")
    return out


class Plan:
    """A plan for one geometry and precision.  ``forward`` / ``adjoint`` take
    torch tensors on the GPU, shaped (n, n) / (nt, m) or batched (B, n, n) /
    (B, nt, m), and return new tensors (or fill ``out``)."""

    def __init__(self, geom: dict, dtype=None, max_batch: int = 1, device=None, tuning_cache: Optional[str] = None):
        """tuning_cache: path of the autotuner's cache file (None: default launch shapes)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libpat needs a GPU: torch.cuda.is_available() is False")
        self.torch = torch
        self.dtype = torch.float32 if dtype is None else dtype
        if self.dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.geom = dict(GEOM_DEFAULTS)
        self.geom.update(geom)
        self.n, self.m, self.nt = int(self.geom["n"]), int(self.geom["m"]), int(self.geom["nt"])
        self.max_batch = int(max_batch)
        lib = load()
        self._lib = lib
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.pat_plan_create(ctypes.byref(h), ctypes.byref(make_geometry(self.geom)),
                                       PAT_F64 if self.dtype == torch.float64 else PAT_F32,
                                       self.max_batch, tuning_cache.encode() if tuning_cache else None),
                   "pat_plan_create")
        self._h = h
        info = PlanInfo()
        _check(lib.pat_plan_get_info(h, ctypes.byref(info)), "pat_plan_get_info")
        self.info = _info_dict(info)
        s = ctypes.c_double()
        _check(lib.pat_adjoint_scale(h, ctypes.byref(s)), "pat_adjoint_scale")
        self.adjoint_scale = s.value
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and self._lib is not None:
            try:
                self.torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self._lib.pat_plan_destroy(h)
            self._h = None

    def workspace(self, batch: int):
        need = self.info["ws_per_image"] * batch
        if self._ws is None or self._ws.numel() < need:
            cap = self.info["ws_per_image"] * self.max_batch
            self._ws = self.torch.empty(max(need, cap), dtype=self.torch.uint8, device=self.device)
        return self._ws

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _prep(self, x, shape_tail):
        t = self.torch
        if not isinstance(x, t.Tensor) or x.device.type != "cuda":
            raise TypeError("expected a CUDA tensor")
        if x.dtype != self.dtype:
            raise TypeError("tensor dtype %s does not match plan dtype %s" % (x.dtype, self.dtype))
        single = x.dim() == 2
        xb = x.unsqueeze(0) if single else x
        if tuple(xb.shape[1:]) != shape_tail:
            raise ValueError("expected trailing shape %s, got %s" % (shape_tail, tuple(xb.shape[1:])))
        return xb.contiguous(), single

    def _out(self, out, shape):
        """The output tensor: a new one, or ``out`` after checking that the
        library may write ``shape`` into it."""
        t = self.torch
        if out is None:
            return t.empty(shape, dtype=self.dtype, device=self.device)
        if not isinstance(out, t.Tensor) or out.device.type != "cuda" or out.dtype != self.dtype:
            raise TypeError("out must be a CUDA tensor of the plan's dtype")
        if not out.is_contiguous() or out.numel() != int(np.prod(shape)):
            raise ValueError("out must be contiguous with %d elements" % int(np.prod(shape)))
        return out.view(shape)

    def forward(self, f, out=None):
        fb, single = self._prep(f, (self.n, self.n))
        B = fb.shape[0]
        g = self._out(out, (B, self.nt, self.m))
        for s in range(0, B, self.max_batch):
            e = min(B, s + self.max_batch)
            ws = self.workspace(e - s)
            _check(self._lib.pat_forward_batched(self._h, e - s, ctypes.c_void_p(fb[s].data_ptr()), self.n * self.n,
                                                 ctypes.c_void_p(g[s].data_ptr()), self.nt * self.m,
                                                 ctypes.c_void_p(ws.data_ptr()), self._stream()),
                   "pat_forward_batched")
        return g[0] if single and out is None else (out if out is not None else g)

    def adjoint(self, g, out=None):
        return self._traces_to_image(self._lib.pat_adjoint_batched, "pat_adjoint_batched", g, out)

    def inverse(self, g, out=None):
        """Approximate inverse A^-1 of Sec. 3.3 (Alg. 3): the universal
        back-projection with the constant of eq. E:silly_integral, restricted
        to the mask disk (see pat_inverse in pat.h)."""
        return self._traces_to_image(self._lib.pat_inverse_batched, "pat_inverse_batched", g, out)

    def _traces_to_image(self, fn, what, g, out):
        gb, single = self._prep(g, (self.nt, self.m))
        B = gb.shape[0]
        f = self._out(out, (B, self.n, self.n))
        for s in range(0, B, self.max_batch):
            e = min(B, s + self.max_batch)
            ws = self.workspace(e - s)
            _check(fn(self._h, e - s, ctypes.c_void_p(gb[s].data_ptr()), self.nt * self.m,
                      ctypes.c_void_p(f[s].data_ptr()), self.n * self.n, ctypes.c_void_p(ws.data_ptr()),
                      self._stream()), what)
        return f[0] if single and out is None else (out if out is not None else f)

    def opnorm(self, iters: int = 30) -> float:
        """||A|| from the X to the Y inner products (power iteration in the library)."""
        out = ctypes.c_double()
        ws = self.workspace(1)
        _check(self._lib.pat_opnorm_estimate(self._h, int(iters), ctypes.byref(out), ctypes.c_void_p(ws.data_ptr()),
                                             self._stream()), "pat_opnorm_estimate")
        return out.value

    def scale_(self, x, a: float):
        """x *= a in place (library kernel; x contiguous, plan dtype)."""
        if not x.is_contiguous() or x.dtype != self.dtype:
            raise TypeError("expected a contiguous tensor of the plan's dtype")
        _check(self._lib.pat_axpby(self._h, x.numel(), float(a), ctypes.c_void_p(x.data_ptr()), 0.0, None,
                                   ctypes.c_void_p(x.data_ptr()), self._stream()), "pat_axpby")
        return x

    def transpose(self, g, out=None):
        """Euclidean transpose A^T = A*/s."""
        return self.scale_(self.adjoint(g, out=out), 1.0 / self.adjoint_scale)


class Group:
    """Plans of different image sizes (same precision) whose forward / adjoint
    chains run as one grouped launch per stage (pat_group_*)."""

    def __init__(self, plans):
        self.plans = list(plans)
        lib = load()
        self._lib = lib
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib.pat_group_create(ctypes.byref(h), len(self.plans), arr), "pat_group_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and self._lib is not None:
            self._lib.pat_group_destroy(h)
            self._h = None

    def _run(self, fn, ins, outs, tails_in, what):
        n = len(self.plans)
        if len(ins) != n or len(outs) != n:
            raise ValueError("one input and one output per plan")
        batch = (ctypes.c_int * n)()
        pin, pout, pws = (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)(), (ctypes.c_void_p * n)()
        for i, (p, x, y) in enumerate(zip(self.plans, ins, outs)):
            for t in (x, y):
                if not t.is_contiguous() or t.dtype != p.dtype or t.device.type != "cuda":
                    raise TypeError("expected contiguous CUDA tensors of the plan's dtype")
            if tuple(x.shape[1:]) != tails_in(p) or x.shape[0] != y.shape[0]:
                raise ValueError("shape mismatch for plan %d" % i)
            batch[i] = x.shape[0]
            pin[i], pout[i] = x.data_ptr(), y.data_ptr()
            pws[i] = p.workspace(x.shape[0]).data_ptr()
        _check(fn(self._h, batch, pin, pout, pws, self.plans[0]._stream()), what)
        return outs

    def forward(self, fs, outs):
        """outs[i] = A_i fs[i] (fs[i]: (B_i, n_i, n_i), outs[i]: (B_i, nt_i, m_i))."""
        return self._run(self._lib.pat_group_forward, fs, outs, lambda p: (p.n, p.n), "pat_group_forward")

    def adjoint(self, gs, outs):
        """outs[i] = A*_i gs[i]."""
        return self._run(self._lib.pat_group_adjoint, gs, outs, lambda p: (p.nt, p.m), "pat_group_adjoint")


def filter_length(nt: int) -> int:
    """N of the measurement filter: the smallest power of two >= 2 nt."""
    lib = load()
    N = ctypes.c_int()
    _check(lib.pat_filter_length(int(nt), ctypes.byref(N)), "pat_filter_length")
    return N.value


class Filter:
    """Measurement operator B of eq. E:real_meas on time-major traces
    (attenuation e^{-gamma t}, transducer response eta given at the N/2 + 1
    non-negative DFT frequencies of the zero-extended trace; see
    pat_filter_create).  apply(g) = B g, apply(g, adjoint=True) = B* g."""

    def __init__(self, nt: int, T: float, m: int, gamma: float, eta, dtype=None, device=None):
        import torch
        self.torch = torch
        self.dtype = dtype if dtype is not None else torch.float32
        if self.dtype not in (torch.float32, torch.float64):
            raise TypeError("dtype must be float32 or float64")
        self.device = torch.device(device if device is not None else "cuda")
        self.nt, self.m, self.T, self.gamma = int(nt), int(m), float(T), float(gamma)
        eta = np.asarray(eta, dtype=np.complex128).ravel()
        buf = np.ascontiguousarray(np.stack([eta.real, eta.imag], axis=1).ravel())
        self._lib = load()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self._lib.pat_filter_create(ctypes.byref(h), self.nt, self.T, self.m, self.gamma,
                                               buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(eta),
                                               1 if self.dtype == torch.float64 else 0), "pat_filter_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and getattr(self, "_lib", None) is not None:
            self._lib.pat_filter_destroy(h)
            self._h = None

    def apply(self, g, adjoint: bool = False, out=None):
        t = self.torch
        if not isinstance(g, t.Tensor) or g.device.type != "cuda" or g.dtype != self.dtype:
            raise TypeError("expected a CUDA tensor of the filter's dtype")
        single = g.dim() == 2
        gb = (g.unsqueeze(0) if single else g).contiguous()
        if tuple(gb.shape[1:]) != (self.nt, self.m):
            raise ValueError("expected traces of shape (nt, m) = (%d, %d)" % (self.nt, self.m))
        B = gb.shape[0]
        if out is None:
            res = t.empty_like(gb)
        else:
            if (not isinstance(out, t.Tensor) or out.dtype != self.dtype or out.device != gb.device
                    or not out.is_contiguous() or out.numel() != gb.numel()):
                raise ValueError("out must be a contiguous tensor like the input")
            res = out.view(gb.shape)
        stream = ctypes.c_void_p(t.cuda.current_stream(gb.device).cuda_stream)
        img = self.nt * self.m
        _check(self._lib.pat_filter_apply(self._h, 1 if adjoint else 0, B, ctypes.c_void_p(gb.data_ptr()), img,
                                          ctypes.c_void_p(res.data_ptr()), img, stream), "pat_filter_apply")
        if out is not None:
            return out
        return res[0] if single else res
