"""MI355X (gfx950) pulse-profile forward model and Poisson likelihood.

Thin ctypes binding of ``libppm.so`` (C ABI in ``include/ppm.h``).  Every
step of the model runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory and the current HIP
stream.  There is no CPU fallback: importing works without a GPU, but
creating a plan needs the built library and a HIP device, and fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libppm.so")

NPARAM = 16
NGRAD = 12
GRAD_SLOTS = (0, 1, 2, 3, 4, 8, 9, 10, 12, 13, 14, 15)
MODE_SD, MODE_OS = 0, 1
I_BLACKBODY, I_TABLE = 0, 1
F32, F64 = 0, 1
INTERP_MIXED, INTERP_CUBIC, INTERP_CUBIC_CLIP, INTERP_CUBIC_LINMU = 0, 1, 2, 3
# per-instance status codes (include/ppm.h)
(INST_OK, INST_NONFINITE, INST_BAD_STAR, INST_COMPACT, INST_BAD_SPOT, INST_FAST_SPIN,
 INST_BAD_MAP) = range(7)

_lib = None


class PPMError(RuntimeError):
    pass


class _Spec(C.Structure):
    _fields_ = [("mode", C.c_int32), ("intensity", C.c_int32), ("n_spots", C.c_int32),
                ("shape", C.c_int32 * 2), ("n_rings", C.c_int32 * 2), ("n_phi", C.c_int32 * 2),
                ("shape_a", C.c_double * 2), ("shape_b", C.c_double * 2),
                ("n_fp", C.c_int32), ("n_phase", C.c_int32), ("n_energy", C.c_int32), ("n_chan", C.c_int32),
                ("energy_kev", C.POINTER(C.c_double)), ("sigma_cm2", C.POINTER(C.c_double)),
                ("rsp", C.POINTER(C.c_double)), ("t_exp", C.c_double),
                ("nT", C.c_int32), ("ng", C.c_int32), ("nmu", C.c_int32), ("nx", C.c_int32),
                ("ax_T", C.POINTER(C.c_double)), ("ax_g", C.POINTER(C.c_double)),
                ("ax_mu", C.POINTER(C.c_double)), ("ax_x", C.POINTER(C.c_double)),
                ("log_intensity", C.POINTER(C.c_double)),
                ("n_alpha", C.c_int32), ("precision", C.c_int32), ("grad", C.c_int32),
                ("interp", C.c_int32), ("n_side", C.c_int32), ("background", C.POINTER(C.c_double)),
                ("count_negative", C.c_int32)]


class _Tiles(C.Structure):
    _fields_ = [("phase_tile", C.c_int32), ("phase_tile_grad", C.c_int32), ("ring_group", C.c_int32)]


TUNE_MAX = 16


class _TuneReport(C.Structure):
    _fields_ = [("n_fwd", C.c_int32), ("n_grad", C.c_int32), ("n_group", C.c_int32),
                ("fwd_tile", C.c_int32 * TUNE_MAX), ("fwd_ms", C.c_double * TUNE_MAX),
                ("grad_tile", C.c_int32 * TUNE_MAX), ("grad_ms", C.c_double * TUNE_MAX),
                ("group", C.c_int32 * TUNE_MAX), ("group_ms", C.c_double * TUNE_MAX),
                ("chosen", _Tiles)]


class _Diag(C.Structure):
    _fields_ = [("n_visible_pairs", C.c_int64), ("n_clamp_T", C.c_int64), ("n_clamp_g", C.c_int64),
                ("n_x_outside", C.c_int64), ("n_multi_image", C.c_int64), ("n_negative", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


PT_MAX_TEMPS = 64


class _PTConfig(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_temps", C.c_int32), ("n_free", C.c_int32),
                ("free_slot", C.c_int32 * 16), ("lo", C.c_double * 16), ("hi", C.c_double * 16),
                ("step", C.c_double * 16), ("beta", C.c_double * PT_MAX_TEMPS), ("seed", C.c_uint64),
                ("swap_every", C.c_int32)]


_VP = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_DP = C.POINTER(C.c_double)

# name -> (restype, argtypes); mirrors include/ppm.h
SIGNATURES = {
    "ppm_plan_create": (C.c_int, [C.POINTER(_Spec), C.c_int, C.c_int, C.POINTER(_VP)]),
    "ppm_plan_destroy": (None, [_VP]),
    "ppm_forward": (C.c_int, [_VP, _VP, C.c_int, _I32P, _VP, _VP]),
    "ppm_flux": (C.c_int, [_VP, _VP, C.c_int, _I32P, _VP, _VP]),
    "ppm_loglike": (C.c_int, [_VP, _VP, C.c_int, _I32P, _VP, _VP, _VP, _VP]),
    "ppm_loglike_grad": (C.c_int, [_VP, _VP, C.c_int, _I32P, _VP, _VP, _VP, _VP]),
    "ppm_loglike_noalloc": (C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP, _VP]),
    "ppm_forward_map": (C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP]),
    "ppm_flux_map": (C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP]),
    "ppm_loglike_map": (C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP, _VP, _VP]),
    "ppm_instance_status": (C.c_int, [_VP, C.c_int, _VP, _VP]),
    "ppm_validate_params": (C.c_int, [_DP, C.c_int, C.c_int, _I32P]),
    "ppm_debug_ring": (C.c_int, [_VP, C.c_int, C.c_int, _DP, _DP, _DP, _I32P, _VP]),
    "ppm_visible_pairs": (C.c_int, [_VP, C.c_int, C.POINTER(C.c_longlong), _VP]),
    "ppm_get_diagnostics": (C.c_int, [_VP, C.c_int, C.POINTER(_Diag), C.POINTER(_Diag), _VP]),
    "ppm_get_passes": (C.c_int, [_VP, C.POINTER(C.c_int)]),
    "ppm_profile_begin": (C.c_int, [_VP, C.c_int]),
    "ppm_profile_end": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "ppm_get_tiles": (C.c_int, [_VP, C.POINTER(_Tiles)]),
    "ppm_set_tiles": (C.c_int, [_VP, C.POINTER(_Tiles)]),
    "ppm_autotune": (C.c_int, [_VP, _VP, C.c_int, _I32P, C.c_int, _VP, C.POINTER(_TuneReport)]),
    "ppm_autotune_map": (C.c_int, [_VP, _VP, C.c_int, _VP, C.c_int, _VP, C.POINTER(_TuneReport)]),
    "ppm_pt_create": (C.c_int, [C.POINTER(_PTConfig), C.POINTER(_VP)]),
    "ppm_pt_destroy": (None, [_VP]),
    "ppm_pt_set_state": (C.c_int, [_VP, _VP, _VP, C.c_int64, _VP]),
    "ppm_pt_propose": (C.c_int, [_VP, _VP, _VP]),
    "ppm_pt_accept": (C.c_int, [_VP, _VP, _VP, _VP]),
    "ppm_pt_run": (C.c_int, [_VP, _VP, _VP, C.c_int, _VP, _VP, _VP]),
    "ppm_pt_get_state": (C.c_int, [_VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_int64), _VP]),
    "ppm_arf_read": (C.c_int, [C.c_char_p, _I32P, _DP, _DP, _DP]),
    "ppm_rmf_read": (C.c_int, [C.c_char_p, _I32P, _I32P, _DP, _DP, _DP, _DP, _DP]),
    "ppm_response_build": (C.c_int, [C.c_int32, _DP, C.c_int32, _DP, _DP, _DP, C.c_int32, _DP, _DP]),
    "ppm_sigma_from_table": (C.c_int, [C.c_int32, _DP, _DP, C.c_double, C.c_int32, _DP, _DP]),
    "ppm_status_string": (C.c_char_p, [C.c_int]),
    "ppm_last_error": (C.c_char_p, []),
    "ppm_version": (C.c_int, []),
}


def lib():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PPMError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        L = lib()
        raise PPMError(f"{what} failed ({rc}: {L.ppm_status_string(rc).decode()}): "
                       f"{L.ppm_last_error().decode()}")


def validate_params(params: np.ndarray, n_spots: int) -> np.ndarray:
    """Host-side parameter validation (same rules as the device)."""
    p = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    out = np.zeros(p.shape[0], dtype=np.int32)
    _check(lib().ppm_validate_params(p.ctypes.data_as(_DP), p.shape[0], n_spots, out.ctypes.data_as(_I32P)),
           "ppm_validate_params")
    return out


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def read_arf(path):
    """OGIP ARF -> (e_lo, e_hi, area) [keV, keV, cm^2]."""
    n = C.c_int32()
    _check(lib().ppm_arf_read(os.fsencode(path), C.byref(n), None, None, None), "ppm_arf_read")
    lo, hi, a = (np.zeros(n.value) for _ in range(3))
    _check(lib().ppm_arf_read(os.fsencode(path), C.byref(n), lo.ctypes.data_as(_DP), hi.ctypes.data_as(_DP),
                              a.ctypes.data_as(_DP)), "ppm_arf_read")
    return lo, hi, a


def read_rmf(path):
    """OGIP RMF -> (e_lo, e_hi, matrix [n_energy, n_chan], ch_lo, ch_hi)."""
    ne, nc = C.c_int32(), C.c_int32()
    _check(lib().ppm_rmf_read(os.fsencode(path), C.byref(ne), C.byref(nc), None, None, None, None, None),
           "ppm_rmf_read")
    lo, hi = np.zeros(ne.value), np.zeros(ne.value)
    m = np.zeros((ne.value, nc.value))
    cl, ch = np.full(nc.value, np.nan), np.full(nc.value, np.nan)
    _check(lib().ppm_rmf_read(os.fsencode(path), C.byref(ne), C.byref(nc), lo.ctypes.data_as(_DP),
                              hi.ctypes.data_as(_DP), m.ctypes.data_as(_DP), cl.ctypes.data_as(_DP),
                              ch.ctypes.data_as(_DP)), "ppm_rmf_read")
    return lo, hi, m, cl, ch


def build_response(e_model, e_lo, e_hi, area, matrix):
    """RSP [n_model, n_chan] = DS (A R) for ppm_spec.rsp (Sect. 2.8.4)."""
    em, lo, hi, mt = _f64(e_model), _f64(e_lo), _f64(e_hi), _f64(matrix)
    ar = None if area is None else _f64(area)
    out = np.zeros((em.size, mt.shape[1]))
    _check(lib().ppm_response_build(em.size, em.ctypes.data_as(_DP), lo.size, lo.ctypes.data_as(_DP),
                                    hi.ctypes.data_as(_DP), None if ar is None else ar.ctypes.data_as(_DP),
                                    mt.shape[1], mt.ctypes.data_as(_DP), out.ctypes.data_as(_DP)),
           "ppm_response_build")
    return out


def sigma_from_table(e_tab, att_tab, nh_ref, energy):
    """Cross-section per H atom [cm^2] from a transmission table at nh_ref."""
    et, at, e = _f64(e_tab), _f64(att_tab), _f64(energy)
    out = np.zeros(e.size)
    _check(lib().ppm_sigma_from_table(et.size, et.ctypes.data_as(_DP), at.ctypes.data_as(_DP), float(nh_ref),
                                      e.size, e.ctypes.data_as(_DP), out.ctypes.data_as(_DP)),
           "ppm_sigma_from_table")
    return out


def _stream_handle(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


class Plan:
    """A plan for one model spec (a dict as built by ``synthetic.config*``)."""

    def __init__(self, spec: dict, max_batch: int = 1, max_cells: int = 0, n_alpha: int | None = None,
                 grad: bool = False, count_negative: bool = False):
        self.keep = []

        def arr(x):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=np.float64)
            self.keep.append(a)
            return a.ctypes.data_as(_DP)

        s = _Spec()
        s.mode = spec["mode"]
        s.intensity = spec["intensity"]
        s.n_spots = spec["n_spots"]
        for i in range(2):
            s.shape[i] = spec["shape"][i]
            s.n_rings[i] = spec["n_rings"][i]
            s.n_phi[i] = spec["n_phi"][i]
            s.shape_a[i] = spec["shape_a"][i]
            s.shape_b[i] = spec["shape_b"][i]
        s.n_fp = spec["n_fp"]
        s.n_phase = spec["n_phase"]
        e = np.asarray(spec["energy"], dtype=np.float64)
        s.n_energy = len(e)
        s.energy_kev = arr(e)
        s.sigma_cm2 = arr(spec.get("sigma"))
        rsp = np.asarray(spec["rsp"], dtype=np.float64)
        s.n_chan = rsp.shape[1]
        s.rsp = arr(rsp)
        s.t_exp = spec["t_exp"]
        if spec["intensity"] == I_TABLE:
            logi = np.asarray(spec["atmos_logI"], dtype=np.float64)
            s.nT, s.ng, s.nmu, s.nx = logi.shape
            at, ag, am, ax = spec["atmos_axes"]
            s.ax_T, s.ax_g, s.ax_mu, s.ax_x = arr(at), arr(ag), arr(am), arr(ax)
            s.log_intensity = arr(logi)
        s.n_alpha = n_alpha if n_alpha is not None else spec.get("n_alpha", 512)
        s.precision = F64 if spec.get("precision", "f32") == "f64" else F32
        s.grad = 1 if grad else 0
        s.interp = int(spec.get("interp", 0))
        s.n_side = int(spec.get("n_side", 0))
        bg = spec.get("background")
        if bg is not None:
            bg = np.asarray(bg, dtype=np.float64)
            assert bg.shape == (s.n_phase, s.n_chan), bg.shape
        s.background = arr(bg)
        s.count_negative = 1 if count_negative else 0
        self.n_side = s.n_side
        self.n_pix = 12 * s.n_side * s.n_side
        self.spec = spec
        self.n_phase = s.n_phase
        self.n_energy = s.n_energy
        self.n_chan = s.n_chan
        self.n_fp = s.n_fp
        self.n_alpha = s.n_alpha
        self.max_batch = max_batch
        if s.n_side:
            self.r_tot = 4 * s.n_side - 1
        else:
            self.r_tot = sum(max(spec["n_rings"][i], max_cells) for i in range(min(2, spec["n_spots"])))
        h = C.c_void_p()
        _check(lib().ppm_plan_create(C.byref(s), max_batch, max_cells, C.byref(h)), "ppm_plan_create")
        self.handle = h
        self.keep = []

    def close(self):
        if getattr(self, "handle", None):
            lib().ppm_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ncells(n_cells, B):
        if n_cells is None:
            return None, None
        a = np.ascontiguousarray(n_cells, dtype=np.int32)
        assert a.shape == (B,)
        return a, a.ctypes.data_as(_I32P)

    def _params(self, params):
        import torch
        assert params.is_cuda and params.dtype == torch.float64 and params.is_contiguous()
        assert params.dim() == 2 and params.shape[1] == NPARAM
        return params.shape[0]

    def forward(self, params, n_cells=None, out=None, stream=None):
        """counts[B, P, C] (float64, device)."""
        import torch
        B = self._params(params)
        if out is None:
            out = torch.empty((B, self.n_phase, self.n_chan), dtype=torch.float64, device=params.device)
        keep, nc = self._ncells(n_cells, B)
        _check(lib().ppm_forward(self.handle, _dptr(params), B, nc, _dptr(out), _stream_handle(stream)),
               "ppm_forward")
        return out

    def flux(self, params, n_cells=None, out=None, stream=None):
        """Photon flux before absorption and response, [B, P, E] float64."""
        import torch
        B = self._params(params)
        if out is None:
            out = torch.empty((B, self.n_phase, self.n_energy), dtype=torch.float64, device=params.device)
        keep, nc = self._ncells(n_cells, B)
        _check(lib().ppm_flux(self.handle, _dptr(params), B, nc, _dptr(out), _stream_handle(stream)), "ppm_flux")
        return out

    def loglike(self, params, data, n_cells=None, counts=None, out=None, stream=None):
        """logL[B] (float64, device); data: int32 [P, C] on the device."""
        import torch
        B = self._params(params)
        assert data.is_cuda and data.dtype == torch.int32 and data.is_contiguous()
        assert data.numel() == self.n_phase * self.n_chan
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=params.device)
        keep, nc = self._ncells(n_cells, B)
        cptr = _dptr(counts) if counts is not None else None
        _check(lib().ppm_loglike(self.handle, _dptr(params), B, nc, _dptr(data), _dptr(out), cptr,
                                 _stream_handle(stream)), "ppm_loglike")
        return out

    def loglike_noalloc(self, params, data, counts=None, out=None, stream=None):
        """logL[B] through ``ppm_loglike_noalloc`` (the spec's own grids; the
        library allocates nothing in the call; ``out`` given: this binding
        allocates nothing either)."""
        import torch
        B = self._params(params)
        assert data.is_cuda and data.dtype == torch.int32 and data.is_contiguous()
        assert data.numel() == self.n_phase * self.n_chan
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=params.device)
        cptr = _dptr(counts) if counts is not None else None
        _check(lib().ppm_loglike_noalloc(self.handle, _dptr(params), B, _dptr(data), _dptr(out), cptr,
                                         _stream_handle(stream)), "ppm_loglike_noalloc")
        return out

    def loglike_grad(self, params, data, n_cells=None, out=None, grad=None, stream=None):
        """(logL[B], grad[B, 12]) float64 on the device; gradient order M, R_e,
        i, Phi, N_H, theta_1, zeta_1, logT_1, theta_2, zeta_2, logT_2, dphi_2.
        Needs a plan created with grad=True."""
        import torch
        B = self._params(params)
        assert data.is_cuda and data.dtype == torch.int32 and data.is_contiguous()
        assert data.numel() == self.n_phase * self.n_chan
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=params.device)
        if grad is None:
            grad = torch.empty((B, NGRAD), dtype=torch.float64, device=params.device)
        keep, nc = self._ncells(n_cells, B)
        _check(lib().ppm_loglike_grad(self.handle, _dptr(params), B, nc, _dptr(data), _dptr(out), _dptr(grad),
                                      _stream_handle(stream)), "ppm_loglike_grad")
        return out, grad

    def _map(self, logT_map, B):
        import torch
        assert self.n_side > 0, "plan has no temperature map (spec n_side = 0)"
        assert logT_map.is_cuda and logT_map.dtype == torch.float64 and logT_map.is_contiguous()
        assert logT_map.numel() == B * self.n_pix
        return _dptr(logT_map)

    def forward_map(self, params, logT_map, out=None, stream=None):
        """counts[B, P, C] of full-surface temperature maps: logT_map [B, 12
        n_side^2] float64 on the device (log10 T per HEALPix patch, ring
        order; non-finite or non-positive: inactive)."""
        import torch
        B = self._params(params)
        mp = self._map(logT_map, B)
        if out is None:
            out = torch.empty((B, self.n_phase, self.n_chan), dtype=torch.float64, device=params.device)
        _check(lib().ppm_forward_map(self.handle, _dptr(params), B, mp, _dptr(out), _stream_handle(stream)),
               "ppm_forward_map")
        return out

    def flux_map(self, params, logT_map, out=None, stream=None):
        """Flux before absorption and response [B, P, E] of temperature maps."""
        import torch
        B = self._params(params)
        mp = self._map(logT_map, B)
        if out is None:
            out = torch.empty((B, self.n_phase, self.n_energy), dtype=torch.float64, device=params.device)
        _check(lib().ppm_flux_map(self.handle, _dptr(params), B, mp, _dptr(out), _stream_handle(stream)),
               "ppm_flux_map")
        return out

    def loglike_map(self, params, logT_map, data, counts=None, out=None, stream=None):
        """logL[B] of temperature maps; data int32 [P, C] on the device."""
        import torch
        B = self._params(params)
        mp = self._map(logT_map, B)
        assert data.is_cuda and data.dtype == torch.int32 and data.is_contiguous()
        assert data.numel() == self.n_phase * self.n_chan
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=params.device)
        cptr = _dptr(counts) if counts is not None else None
        _check(lib().ppm_loglike_map(self.handle, _dptr(params), B, mp, _dptr(data), _dptr(out), cptr,
                                     _stream_handle(stream)), "ppm_loglike_map")
        return out

    def status(self, B, stream=None):
        import torch
        out = torch.empty(B, dtype=torch.int32, device="cuda")
        _check(lib().ppm_instance_status(self.handle, B, _dptr(out), _stream_handle(stream)), "ppm_instance_status")
        return out

    def debug_ring(self, b, r, stream=None):
        tab = np.zeros((self.n_alpha, 4))
        info = np.zeros(4)
        tr = np.zeros((self.n_fp + 1, 4))
        ti = np.zeros(3, dtype=np.int32)
        _check(lib().ppm_debug_ring(self.handle, b, r, tab.ctypes.data_as(_DP), info.ctypes.data_as(_DP),
                                    tr.ctypes.data_as(_DP), ti.ctypes.data_as(_I32P), _stream_handle(stream)),
               "ppm_debug_ring")
        return dict(table=tab, alpha_max=info[0], psi_top=info[1], u=info[2], R=info[3], trace=tr,
                    visible=bool(ti[0]), inv=(int(ti[1]), int(ti[2])))

    def profile_begin(self, max_calls):
        _check(lib().ppm_profile_begin(self.handle, max_calls), "ppm_profile_begin")

    def profile_end(self):
        """(summed hot-kernel milliseconds, number of timed calls)."""
        ms = C.c_double()
        n = C.c_int()
        _check(lib().ppm_profile_end(self.handle, C.byref(ms), C.byref(n)), "ppm_profile_end")
        return ms.value, n.value

    @property
    def tiles(self):
        """(phase_tile, phase_tile_grad): phases per work-group of the forward
        and of the adjoint accumulation kernels."""
        t = _Tiles()
        _check(lib().ppm_get_tiles(self.handle, C.byref(t)), "ppm_get_tiles")
        return int(t.phase_tile), int(t.phase_tile_grad)

    @property
    def ring_group(self):
        """Rings summed per work-group of the windowed forward kernel."""
        t = _Tiles()
        _check(lib().ppm_get_tiles(self.handle, C.byref(t)), "ppm_get_tiles")
        return int(t.ring_group)

    def set_tiles(self, phase_tile=None, phase_tile_grad=None, ring_group=None):
        t = _Tiles()
        _check(lib().ppm_get_tiles(self.handle, C.byref(t)), "ppm_get_tiles")
        if phase_tile is not None:
            t.phase_tile = int(phase_tile)
        if phase_tile_grad is not None:
            t.phase_tile_grad = int(phase_tile_grad)
        if ring_group is not None:
            t.ring_group = int(ring_group)
        _check(lib().ppm_set_tiles(self.handle, C.byref(t)), "ppm_set_tiles")

    def autotune(self, params, n_cells=None, reps=5, stream=None):
        """Times every candidate phase tile on this batch (``reps`` calls each,
        median) and keeps the fastest on the plan.  Returns
        {"forward": {tile: ms}, "grad": {tile: ms}, "chosen": (fwd, grad)}."""
        B = self._params(params)
        keep, nc = self._ncells(n_cells, B)
        r = _TuneReport()
        _check(lib().ppm_autotune(self.handle, _dptr(params), B, nc, int(reps), _stream_handle(stream),
                                  C.byref(r)), "ppm_autotune")
        return {"forward": {int(r.fwd_tile[i]): float(r.fwd_ms[i]) for i in range(r.n_fwd)},
                "group": {int(r.group[i]): float(r.group_ms[i]) for i in range(r.n_group)},
                "grad": {int(r.grad_tile[i]): float(r.grad_ms[i]) for i in range(r.n_grad)},
                "chosen": (int(r.chosen.phase_tile), int(r.chosen.phase_tile_grad)),
                "ring_group": int(r.chosen.ring_group)}

    def autotune_map(self, params, logT_map, reps=5, stream=None):
        """Autotuner of a temperature-map plan (phase tiles 8, 16, 32);
        returns {"forward": {tile: ms}, "chosen": (fwd, grad)}."""
        B = self._params(params)
        mp = self._map(logT_map, B)
        r = _TuneReport()
        _check(lib().ppm_autotune_map(self.handle, _dptr(params), B, mp, int(reps), _stream_handle(stream),
                                      C.byref(r)), "ppm_autotune_map")
        return {"forward": {int(r.fwd_tile[i]): float(r.fwd_ms[i]) for i in range(r.n_fwd)},
                "chosen": (int(r.chosen.phase_tile), int(r.chosen.phase_tile_grad))}

    def diagnostics(self, B, per_instance=False, stream=None):
        """Counters of the last evaluation (``ppm_get_diagnostics``): a dict
        of totals over its first B instances, or (totals, [per instance])."""
        tot = _Diag()
        per = (_Diag * B)() if per_instance else None
        _check(lib().ppm_get_diagnostics(self.handle, B, C.byref(tot), per, _stream_handle(stream)),
               "ppm_get_diagnostics")
        if per_instance:
            return tot.as_dict(), [per[i].as_dict() for i in range(B)]
        return tot.as_dict()

    @property
    def passes(self):
        """Workspace passes of the last evaluation."""
        n = C.c_int()
        _check(lib().ppm_get_passes(self.handle, C.byref(n)), "ppm_get_passes")
        return n.value

    def visible_pairs(self, B, stream=None):
        out = C.c_longlong()
        _check(lib().ppm_visible_pairs(self.handle, B, C.byref(out), _stream_handle(stream)), "ppm_visible_pairs")
        return out.value


class GraphedLogLike:
    """One likelihood evaluation of B parameter vectors (with the gradient
    when ``grad=True``; the plan must then have been created with
    ``grad=True``) captured as a HIP graph (through torch.cuda.CUDAGraph) and
    replayed per call: the whole launch sequence of the evaluation is
    submitted at once.  ``__call__`` copies the parameters into the captured
    input buffer, replays, and returns the captured output tensor(s)
    (overwritten by the next call): logL[B], or (logL[B], grad[B, 12])."""

    def __init__(self, plan: Plan, data, B: int, n_cells=None, grad: bool = False):
        import torch
        self.plan = plan
        self.with_grad = grad
        dev = data.device
        self.params = torch.zeros((B, NPARAM), dtype=torch.float64, device=dev)
        self.out = torch.empty(B, dtype=torch.float64, device=dev)
        self.grad = torch.empty((B, NGRAD), dtype=torch.float64, device=dev) if grad else None
        self.data = data
        self.n_cells = None if n_cells is None else np.ascontiguousarray(n_cells, dtype=np.int32)
        # a valid parameter set for the warm-up (the graph records launches only)
        from_spec = np.zeros(NPARAM)
        from_spec[[0, 1, 2, 5, 6, 8, 9, 10, 12, 13, 14]] = [1.4, 12.0, 1.0, 100.0, 100.0, 1.0, 0.1, 6.0, 2.0,
                                                           0.1, 6.0]
        self.params.copy_(torch.tensor(np.tile(from_spec, (B, 1)), device=dev))
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._launch()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._launch()

    def _launch(self):
        if self.with_grad:
            self.plan.loglike_grad(self.params, self.data, n_cells=self.n_cells, out=self.out, grad=self.grad)
        else:
            self.plan.loglike(self.params, self.data, n_cells=self.n_cells, out=self.out)

    def __call__(self, params):
        self.params.copy_(params)
        self.graph.replay()
        return (self.out, self.grad) if self.with_grad else self.out


class PTSampler:
    """GPU-resident parallel-tempered Metropolis sampler (``ppm_pt_*``):
    n_chains chains at each inverse temperature of ``betas``, random-walk
    moves on the parameter-record slots ``free_slots`` with standard
    deviations ``steps`` (at beta = 1) inside the prior box [lo, hi]."""

    def __init__(self, n_chains, betas, free_slots, lo, hi, steps, seed=0, swap_every=1):
        c = _PTConfig()
        c.n_chains = int(n_chains)
        c.n_temps = len(betas)
        c.n_free = len(free_slots)
        for j, sl in enumerate(free_slots):
            c.free_slot[j] = int(sl)
            c.lo[j] = float(lo[j])
            c.hi[j] = float(hi[j])
            c.step[j] = float(steps[j])
        for t, b in enumerate(betas):
            c.beta[t] = float(b)
        c.seed = int(seed)
        c.swap_every = int(swap_every)
        self.C, self.T = c.n_chains, c.n_temps
        h = C.c_void_p()
        _check(lib().ppm_pt_create(C.byref(c), C.byref(h)), "ppm_pt_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().ppm_pt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, params, logl=None, step=0, stream=None):
        """params [T, C, 16], logl [T, C] (None: -inf), float64 on the device."""
        import torch
        assert params.is_cuda and params.dtype == torch.float64 and params.is_contiguous()
        assert params.numel() == self.T * self.C * NPARAM
        lp = None
        if logl is not None:
            assert logl.dtype == torch.float64 and logl.is_contiguous() and logl.numel() == self.T * self.C
            lp = _dptr(logl)
        _check(lib().ppm_pt_set_state(self.handle, _dptr(params), lp, int(step), _stream_handle(stream)),
               "ppm_pt_set_state")

    def propose(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((self.T, self.C, NPARAM), dtype=torch.float64, device="cuda")
        _check(lib().ppm_pt_propose(self.handle, _dptr(out), _stream_handle(stream)), "ppm_pt_propose")
        return out

    def accept(self, prop, prop_logl, stream=None):
        _check(lib().ppm_pt_accept(self.handle, _dptr(prop), _dptr(prop_logl), _stream_handle(stream)),
               "ppm_pt_accept")

    def run(self, plan: Plan, data, n_steps, chain=None, chain_logl=None, stream=None):
        """n_steps of propose -> plan.loglike -> accept; returns the cold
        chains [n_steps, C, 16] and their logL [n_steps, C]."""
        import torch
        if chain is None:
            chain = torch.empty((n_steps, self.C, NPARAM), dtype=torch.float64, device="cuda")
        if chain_logl is None:
            chain_logl = torch.empty((n_steps, self.C), dtype=torch.float64, device="cuda")
        _check(lib().ppm_pt_run(self.handle, plan.handle, _dptr(data), int(n_steps), _dptr(chain), _dptr(chain_logl),
                                _stream_handle(stream)), "ppm_pt_run")
        return chain, chain_logl

    def state(self, stream=None):
        """(params [T, C, 16], logl [T, C], accept counts [T, C], swap
        counts [T-1, C], step)."""
        import torch
        p = torch.empty((self.T, self.C, NPARAM), dtype=torch.float64, device="cuda")
        ll = torch.empty((self.T, self.C), dtype=torch.float64, device="cuda")
        na = torch.empty((self.T, self.C), dtype=torch.int32, device="cuda")
        ns = torch.zeros((max(self.T - 1, 1), self.C), dtype=torch.int32, device="cuda")
        st = C.c_int64()
        _check(lib().ppm_pt_get_state(self.handle, _dptr(p), _dptr(ll), _dptr(na),
                                      _dptr(ns) if self.T > 1 else None, C.byref(st), _stream_handle(stream)),
               "ppm_pt_get_state")
        return p, ll, na, ns[: self.T - 1], st.value


def _autograd_function():
    import torch

    class PPMLogLike(torch.autograd.Function):
        """logL[B] of parameter vectors [B, 16] with the library's hand-written
        adjoint as backward: d logL / d params is zero in the slots that are
        not differentiable (nu, D, unused)."""

        @staticmethod
        def forward(ctx, params, plan, data, n_cells=None):
            p = params.detach().contiguous()
            if not ctx.needs_input_grad[0]:
                return plan.loglike(p, data, n_cells=n_cells)
            ll, g = plan.loglike_grad(p, data, n_cells=n_cells)
            full = torch.zeros_like(p)
            full[:, list(GRAD_SLOTS)] = g
            ctx.save_for_backward(full)
            return ll

        @staticmethod
        def backward(ctx, grad_out):
            (full,) = ctx.saved_tensors
            return grad_out[:, None] * full, None, None, None

    return PPMLogLike


def loglike_autograd(params, plan: Plan, data, n_cells=None):
    """Differentiable logL[B]: ``loglike_autograd(p, plan, data).sum().backward()``
    fills ``p.grad`` through the adjoint kernels (one forward+adjoint launch
    sequence per call)."""
    global PPMLogLike
    if PPMLogLike is None:
        PPMLogLike = _autograd_function()
    return PPMLogLike.apply(params, plan, data, n_cells)


PPMLogLike = None
