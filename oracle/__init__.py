"""FP64 CPU oracle of the pulse-profile forward model and Poisson likelihood.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP implementation in ``paper_2510_07764_amd``; the two meet only in
the seeded inputs of ``synthetic``.

The numerical work lives in ``ppm_oracle.c`` (plain double precision, naive
loops, adaptive quadrature, OpenMP over rings); this module marshals numpy
arrays through ctypes and adds the central finite-difference gradient.

Parity notes
------------
Every function is pinned by ``tests/test_oracle_*.py`` against closed forms,
independent quadratures (mpmath, of the original radial integrals Eqs. 12
and 15), vector-geometry derivations, brute-force continuum evaluation on
tiny grids, invariants and library routines.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("PPM_ORACLE_LIB", os.path.join(_HERE, "libppm_oracle.so"))
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    src = os.path.join(_HERE, "ppm_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wno-unknown-pragmas", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Spec(C.Structure):
    _fields_ = [("mode", C.c_int), ("intensity", C.c_int), ("n_spots", C.c_int),
                ("shape", C.c_int * 2), ("n_rings", C.c_int * 2), ("n_phi", C.c_int * 2),
                ("shape_a", C.c_double * 2), ("shape_b", C.c_double * 2),
                ("n_fp", C.c_int), ("n_phase", C.c_int), ("n_energy", C.c_int), ("n_chan", C.c_int),
                ("energy", C.POINTER(C.c_double)), ("sigma", C.POINTER(C.c_double)),
                ("rsp", C.POINTER(C.c_double)), ("t_exp", C.c_double),
                ("nT", C.c_int), ("ng", C.c_int), ("nmu", C.c_int), ("nx", C.c_int),
                ("ax_T", C.POINTER(C.c_double)), ("ax_g", C.POINTER(C.c_double)),
                ("ax_mu", C.POINTER(C.c_double)), ("ax_x", C.POINTER(C.c_double)),
                ("logI", C.POINTER(C.c_double)), ("interp", C.c_int)]


class Diag(C.Structure):
    _fields_ = [("n_clamp_T", C.c_longlong), ("n_clamp_g", C.c_longlong),
                ("n_x_outside", C.c_longlong), ("n_multi_image", C.c_longlong),
                ("n_visible_pairs", C.c_longlong), ("status", C.c_int), ("n_negative", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Star(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("GM", "Rs", "Re", "x", "Obar", "o2", "g0", "D", "nu", "incl", "NH")]


class Ring(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("theta", "dcos", "R", "u", "f", "coseta", "sineta", "logg",
                                          "beta", "gamma", "dphi_out", "dphi_in", "dphi_cell", "w_cell",
                                          "alpha_max", "psi_top")] + [("n_cells", C.c_int)]


_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        for name in ("orc_psi", "orc_dpsi_dalpha", "orc_tp", "orc_rho"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double, C.c_double]
        L.orc_alpha_capture.restype = C.c_double
        L.orc_alpha_capture.argtypes = [C.c_double]
        L.orc_invert.restype = C.c_int
        L.orc_invert.argtypes = [C.c_double, C.c_double, C.c_double, _D]
        L.orc_star_setup.argtypes = [C.POINTER(Spec), _D, C.POINTER(Star)]
        L.orc_rings.argtypes = [C.POINTER(Spec), _D, C.c_int, C.POINTER(Ring)]
        L.orc_rings.restype = C.c_int
        L.orc_cdt_oblate.restype = C.c_double
        L.orc_cdt_oblate.argtypes = [C.POINTER(Star), C.c_double]
        L.orc_total_delay.restype = C.c_double
        L.orc_total_delay.argtypes = [C.POINTER(Star), C.c_double, C.c_double, C.c_double]
        L.orc_trace_ring.restype = C.c_int
        L.orc_trace_ring.argtypes = [C.POINTER(Spec), _D, C.POINTER(Ring), _D, _D, _D, _D,
                                     C.POINTER(C.c_int), C.POINTER(Diag)]
        L.orc_atmo_interp_mode.restype = C.c_double
        L.orc_atmo_interp_mode.argtypes = [C.POINTER(Spec), _D, C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.c_int, C.POINTER(Diag)]
        L.orc_blackbody.restype = C.c_double
        L.orc_blackbody.argtypes = [C.c_double, C.c_double]
        L.orc_forward.restype = C.c_int
        L.orc_forward.argtypes = [C.POINTER(Spec), _D, _D, _D, C.POINTER(Diag)]
        L.orc_forward_map.restype = C.c_int
        L.orc_forward_map.argtypes = [C.POINTER(Spec), _D, C.c_int, _D, _D, _D, C.POINTER(Diag)]
        L.orc_healpix_ring.restype = None
        L.orc_healpix_ring.argtypes = [C.c_int, C.c_int, _D, C.POINTER(C.c_int), _D]
        L.orc_loglike_counts.restype = C.c_double
        L.orc_loglike_counts.argtypes = [_D, C.POINTER(C.c_int), C.c_longlong]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_D) if a is not None else None


class OracleSpec:
    """Holds a ctypes Spec plus the numpy arrays it points to."""

    def __init__(self, spec: dict):
        self.keep = []

        def arr(x):
            if x is None:
                return None
            a = np.ascontiguousarray(x, dtype=np.float64)
            self.keep.append(a)
            return a

        s = Spec()
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
        e = arr(spec["energy"])
        s.n_energy = len(e)
        s.energy = _ptr(e)
        sig = arr(spec.get("sigma"))
        s.sigma = _ptr(sig) if sig is not None else None
        rsp = arr(spec.get("rsp"))
        s.n_chan = rsp.shape[1] if rsp is not None else 0
        s.rsp = _ptr(rsp) if rsp is not None else None
        s.t_exp = spec["t_exp"]
        if spec["intensity"] == 1:
            logi = arr(spec["atmos_logI"])
            axes = [arr(a) for a in spec["atmos_axes"]]
            s.nT, s.ng, s.nmu, s.nx = logi.shape
            s.ax_T, s.ax_g, s.ax_mu, s.ax_x = [_ptr(a) for a in axes]
            s.logI = _ptr(logi)
        s.interp = int(spec.get("interp", 0))
        self.s = s
        self.n_phase = s.n_phase
        self.n_energy = s.n_energy
        self.n_chan = s.n_chan


def forward(spec: dict | OracleSpec, params, want_counts=True):
    """Returns (Ft[P, E], counts[P, C] or None, diag dict)."""
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    p = np.ascontiguousarray(params, dtype=np.float64)
    ft = np.zeros((os_.n_phase, os_.n_energy))
    cnt = np.zeros((os_.n_phase, os_.n_chan)) if (want_counts and os_.n_chan) else None
    d = Diag()
    lib().orc_forward(C.byref(os_.s), _ptr(p), _ptr(ft), _ptr(cnt) if cnt is not None else None, C.byref(d))
    return ft, cnt, d.as_dict()


def forward_map(spec: dict | OracleSpec, params, nside: int, logT_map, want_counts=True):
    """Full-surface temperature map on HEALPix (Sects. 2.6, 2.8.1):
    logT_map[12 nside^2] in ring order, non-finite or non-positive entries
    inactive.  Returns (Ft[P, E], counts[P, C] or None, diag dict)."""
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    p = np.ascontiguousarray(params, dtype=np.float64)
    m = np.ascontiguousarray(logT_map, dtype=np.float64)
    assert m.shape == (12 * nside * nside,)
    ft = np.zeros((os_.n_phase, os_.n_energy))
    cnt = np.zeros((os_.n_phase, os_.n_chan)) if (want_counts and os_.n_chan) else None
    d = Diag()
    rc = lib().orc_forward_map(C.byref(os_.s), _ptr(p), int(nside), _ptr(m), _ptr(ft),
                               _ptr(cnt) if cnt is not None else None, C.byref(d))
    assert rc == 0
    return ft, cnt, d.as_dict()


def healpix_ring(nside: int, i: int):
    """(cos colatitude, pixels, azimuth of the first pixel) of HEALPix ring
    i = 1 .. 4 nside - 1."""
    z = C.c_double()
    n = C.c_int()
    f = C.c_double()
    lib().orc_healpix_ring(int(nside), int(i), C.byref(z), C.byref(n), C.byref(f))
    return z.value, n.value, f.value


def loglike_from_counts(counts, data) -> float:
    m = np.ascontiguousarray(counts, dtype=np.float64).ravel()
    d = np.ascontiguousarray(data, dtype=np.int32).ravel()
    return lib().orc_loglike_counts(_ptr(m), d.ctypes.data_as(C.POINTER(C.c_int)), m.size)


def loglike(spec, params, data) -> float:
    _, cnt, _ = forward(spec, params)
    return loglike_from_counts(cnt, data)


def set_threads(n: int):
    """OpenMP threads of the oracle's ring loop (timing only)."""
    lib().orc_set_threads(int(n))


def fd_gradient(spec, params, data, slots, rel_step=1e-4):
    """Central finite differences of the FP64 log-likelihood, step
    h_i = rel_step * |theta_i| (absolute rel_step for a zero parameter)."""
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    p0 = np.asarray(params, dtype=np.float64)
    g = np.zeros(len(slots))
    for n, s in enumerate(slots):
        h = rel_step * abs(p0[s]) if p0[s] != 0 else rel_step
        pp, pm = p0.copy(), p0.copy()
        pp[s] += h
        pm[s] -= h
        g[n] = (loglike(os_, pp, data) - loglike(os_, pm, data)) / (2 * h)
    return g


def fd_gradient_counts(spec, params, data, slots, rel_step=1e-6, background=None):
    """d logL / d theta by the chain rule through the model counts: central
    finite differences of the oracle's counts m with step
    h_i = rel_step |theta_i| (absolute rel_step for a zero parameter),
    contracted with the closed-form derivative of the Poisson log-likelihood
    at the central point, d logL / d m = d / (m + b) - 1 (-1 where d = 0;
    b = background counts or 0).  Differencing the counts instead of logL
    avoids the cancellation of logL's large constant part (sum ln d!,
    sum d ln m), so that the differences converge to ~1e-9 relative wherever
    the model is smooth over the step."""
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    p0 = np.asarray(params, dtype=np.float64)
    d = np.asarray(data, dtype=np.float64)
    _, m0, _ = forward(os_, p0)
    mb = m0 + (np.asarray(background, dtype=np.float64) if background is not None else 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        gm = np.where(d > 0, d / mb, 0.0) - 1.0
    g = np.zeros(len(slots))
    for n, s in enumerate(slots):
        h = rel_step * abs(p0[s]) if p0[s] != 0 else rel_step
        pp, pm = p0.copy(), p0.copy()
        pp[s] += h
        pm[s] -= h
        g[n] = float(np.sum(gm * (forward(os_, pp)[1] - forward(os_, pm)[1]))) / (2 * h)
    return g


# ------------------------------------------------------------- primitives
def psi(u, alpha):
    return lib().orc_psi(u, alpha)


def dpsi_dalpha(u, alpha):
    return lib().orc_dpsi_dalpha(u, alpha)


def tp(u, alpha):
    return lib().orc_tp(u, alpha)


def rho(u, alpha):
    return lib().orc_rho(u, alpha)


def alpha_capture(u):
    return lib().orc_alpha_capture(u)


def invert(u, alpha_max, psi_val):
    out = np.zeros(4)
    ok = lib().orc_invert(u, alpha_max, psi_val, _ptr(out))
    return (out if ok else None)


def star(spec, params):
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    st = Star()
    p = np.ascontiguousarray(params, dtype=np.float64)
    lib().orc_star_setup(C.byref(os_.s), _ptr(p), C.byref(st))
    return st


def rings(spec, params, spot):
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    n = os_.s.n_rings[spot]
    arr = (Ring * n)()
    p = np.ascontiguousarray(params, dtype=np.float64)
    lib().orc_rings(C.byref(os_.s), _ptr(p), spot, arr)
    return [arr[i] for i in range(n)]


def total_delay(spec, params, R, u, alpha):
    st = star(spec, params)
    return lib().orc_total_delay(C.byref(st), R, u, alpha)


def cdt_oblate(spec, params, R):
    st = star(spec, params)
    return lib().orc_cdt_oblate(C.byref(st), R)


def trace_ring(spec, params, ring):
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    n = os_.s.n_fp + 1
    F, z, phio, mu = (np.zeros(n) for _ in range(4))
    inv = (C.c_int * 2)()
    d = Diag()
    p = np.ascontiguousarray(params, dtype=np.float64)
    vis = lib().orc_trace_ring(C.byref(os_.s), _ptr(p), C.byref(ring), _ptr(F), _ptr(z), _ptr(phio),
                               _ptr(mu), inv, C.byref(d))
    return dict(visible=bool(vis), F=F, z=z, phio=phio, mu=mu, inv=(inv[0], inv[1]), diag=d.as_dict())


def atmo(spec, linI, logT, logg, mu, x, mode=0):
    os_ = spec if isinstance(spec, OracleSpec) else OracleSpec(spec)
    li = np.ascontiguousarray(linI, dtype=np.float64)
    d = Diag()
    return lib().orc_atmo_interp_mode(C.byref(os_.s), _ptr(li), logT, logg, mu, x, mode, C.byref(d))


def blackbody(E, T):
    return lib().orc_blackbody(E, T)
