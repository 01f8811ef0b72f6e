"""ctypes binding of libdmwf (include/dmwf.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Host calls take NumPy arrays (maps float64 [nrhs, 3, npix] in RING
order with fields I, Q, U; alm complex128 [nrhs, 3, nalm] packed m-major with
fields T, E, B).  Device calls take torch tensors on the GPU (float64, and
alm as float64 [..., 2] or complex128) plus an optional torch stream.

The library must have been built (``python -m paper_1801_05358_amd.build``);
importing this module without it raises, so that no caller silently falls
back to anything else.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmwf.so")
# the DMWF_ABI_VERSION of include/dmwf.h these signatures follow
ABI_VERSION = 11

DM_OK, DM_EINVAL, DM_ENOMEM, DM_EDEVICE, DM_ENONFINITE, DM_ESTATE, DM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "DM_OK", -1: "DM_EINVAL", -2: "DM_ENOMEM", -3: "DM_EDEVICE", -4: "DM_ENONFINITE",
                -5: "DM_ESTATE", -6: "DM_EUNSUPPORTED"}
GRID_HEALPIX, GRID_GL = 0, 1
FP64, MIXED = 0, 1
NCOV_DIAG3, NCOV_SYM6 = 0, 1
KERNEL_CLASSES = ("legendre_analysis", "legendre_synthesis", "ring_fft_pointwise", "combine_filter",
                  "pixel_update_3x3")


class DmGrid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nside", ctypes.c_int), ("ntheta", ctypes.c_int), ("nphi", ctypes.c_int)]


class DmSchedule(ctypes.Structure):
    _fields_ = [("lambda_start", ctypes.c_double), ("nsteps", ctypes.c_int), ("iters_per_step", ctypes.c_int),
                ("beta", ctypes.c_double), ("eps_start", ctypes.c_double), ("eps_end", ctypes.c_double),
                ("eps_eta", ctypes.c_double), ("max_iters", ctypes.c_int)]


class DmStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("residual", ctypes.c_double), ("cauchy", ctypes.c_double),
                ("chi2", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DmwfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def hip_runtimes():
    """Distinct HIP runtime files (libamdhip64) mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln and "/" in ln})
    except OSError:
        return []


def lib():
    """Load libdmwf.so (once).  Raises if it has not been built.

    PyTorch ships its own HIP runtime (torch/lib/libamdhip64.so, soname
    libamdhip64.so.7).  Loaded after the library, torch would bring a second
    runtime into the process, and the device calls would hand torch's
    streams and allocations to the other one.  So torch, when it is
    installed, is imported first: the library's libamdhip64.so.7 then
    resolves to the runtime already loaded.  The load is refused if two
    runtimes are mapped all the same (e.g. the library was loaded through
    another path before torch)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1801_05358_amd.build`")
    try:
        import torch  # noqa: F401  (loads torch's HIP runtime before the library's)
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    rts = hip_runtimes()
    if len(rts) > 1:
        raise RuntimeError("two HIP runtimes are mapped into this process (" + ", ".join(rts) +
                           "): import torch before anything loads libdmwf.so")
    sig = {
        "dm_abi_version": (ctypes.c_int, []),
        "dm_device_count": (ctypes.c_int, []),
        "dm_plan_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(DmGrid), ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int]),
        "dm_plan_destroy": (ctypes.c_int, [_P]),
        "dm_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int)]),
        "dm_set_spectra": (ctypes.c_int, [_P, _D]),
        "dm_set_noise": (ctypes.c_int, [_P, _D, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]),
        "dm_set_schedule": (ctypes.c_int, [_P, ctypes.POINTER(DmSchedule)]),
        "dm_schedule_trace": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                              ctypes.POINTER(ctypes.c_int)]),
        "dm_set_refinement": (ctypes.c_int, [_P, ctypes.c_int]),
        "dm_refinement_trace": (ctypes.c_int, [_P, _D, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                ctypes.POINTER(ctypes.c_int)]),
        "dm_set_refinement_select": (ctypes.c_int, [_P, ctypes.c_int]),
        "dm_set_adaptive_resolution": (ctypes.c_int, [_P, ctypes.c_double]),
        "dm_step_band_limits": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                                ctypes.POINTER(ctypes.c_int)]),
        "dm_set_diagnostics": (ctypes.c_int, [_P, ctypes.c_int]),
        "dm_diagnostics_trace": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), _D, _D, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "dm_refinement_selected": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                                   ctypes.POINTER(ctypes.c_int)]),
        "dm_wiener_filter": (ctypes.c_int, [_P, ctypes.c_int, _D, _D, _D, ctypes.POINTER(DmStats)]),
        "dm_wiener_filter_device": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, ctypes.POINTER(DmStats)]),
        "dm_wiener_filter_device_f32": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P, ctypes.POINTER(DmStats)]),
        "dm_constrained_realizations": (ctypes.c_int, [_P, ctypes.c_int, _D, _D, _D, _D, _D]),
        "dm_alm2map": (ctypes.c_int, [_P, ctypes.c_int, _D, _D]),
        "dm_map2alm": (ctypes.c_int, [_P, ctypes.c_int, _D, _D]),
        "dm_alm2map_adjoint": (ctypes.c_int, [_P, ctypes.c_int, _D, _D]),
        "dm_alm2map_device": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
        "dm_map2alm_device": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
        "dm_map2alm_device_noalloc": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P]),
        "dm_set_noise_masks": (ctypes.c_int, [_P, _D, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8),
                                              ctypes.POINTER(ctypes.c_uint8)]),
        "dm_autotune": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D]),
        "dm_checkpoint_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
        "dm_checkpoint_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
        "dm_iterate": (ctypes.c_int, [_P, ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_int, _D, _D]),
        "dm_transform_work": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "dm_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
        "dm_kernel_times": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]),
        "dm_last_error": (ctypes.c_char_p, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.dm_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{LIB_PATH} has ABI version {L.dm_abi_version()}, the binding needs {ABI_VERSION}: rebuild it")
    _lib = L
    return L


def exported_symbols():
    """Names declared in include/dmwf.h that the binding expects."""
    return ["dm_abi_version", "dm_device_count", "dm_plan_create", "dm_plan_destroy", "dm_plan_info",
            "dm_set_spectra", "dm_set_noise", "dm_set_noise_masks", "dm_set_schedule", "dm_schedule_trace", "dm_set_refinement",
            "dm_refinement_trace", "dm_set_refinement_select", "dm_refinement_selected",
            "dm_set_diagnostics", "dm_diagnostics_trace", "dm_set_adaptive_resolution", "dm_step_band_limits", "dm_wiener_filter",
            "dm_wiener_filter_device", "dm_wiener_filter_device_f32",
            "dm_constrained_realizations", "dm_alm2map", "dm_map2alm", "dm_alm2map_adjoint", "dm_alm2map_device",
            "dm_map2alm_device", "dm_map2alm_device_noalloc", "dm_autotune", "dm_checkpoint_save", "dm_checkpoint_load", "dm_iterate", "dm_transform_work", "dm_profile_enable", "dm_kernel_times", "dm_last_error"]


def device_count():
    return lib().dm_device_count()


def _dptr(a):
    return a.ctypes.data_as(_D)


def _c64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a.reshape(shape)


def _f64(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape)


def _dev(t, count, name, dtype="torch.float64"):
    """Pointer of a device tensor the library will read or write: of dtype,
    on a GPU, contiguous, with exactly `count` elements (else ValueError, so
    that no kernel sees a buffer of the wrong size)."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a GPU tensor")
    if str(t.dtype) != dtype:
        raise ValueError(f"{name} must be {dtype[6:]}, not {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != count:
        raise ValueError(f"{name} has {t.numel()} elements, expected {count}")
    return _P(t.data_ptr())


class Plan:
    """A solver plan: grid, band limit, batch capacity, precision, device."""

    def __init__(self, lmax, nside=None, ntheta=None, nphi=None, max_rhs=1, precision=FP64, device=0):
        L = lib()
        g = DmGrid()
        if nside is not None:
            g.kind, g.nside = GRID_HEALPIX, int(nside)
        else:
            g.kind, g.ntheta, g.nphi = GRID_GL, int(ntheta), int(nphi)
        h = _P()
        st = L.dm_plan_create(ctypes.byref(h), ctypes.byref(g), int(lmax), int(max_rhs), int(precision), int(device))
        if st != DM_OK:
            raise DmwfError(st, L.dm_last_error(None).decode())
        self._h = h
        self.lmax = int(lmax)
        self.max_rhs = int(max_rhs)
        npix, nalm, nr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        L.dm_plan_info(h, ctypes.byref(npix), ctypes.byref(nalm), ctypes.byref(nr))
        self.npix, self.nalm, self.nrings = npix.value, nalm.value, nr.value

    def close(self):
        if getattr(self, "_h", None):
            lib().dm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != DM_OK:
            raise DmwfError(st, lib().dm_last_error(self._h).decode())

    # -- setup -------------------------------------------------------------
    def set_spectra(self, cl):
        cl = _f64(cl, (4, self.lmax + 1))
        self._check(lib().dm_set_spectra(self._h, _dptr(cl)))

    def _mask(self, m):
        if m is None:
            return None, None
        m = np.ascontiguousarray(np.asarray(m).astype(np.uint8).reshape(self.npix))
        return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))

    def set_noise(self, ncov, obs=None):
        """ncov [3, npix] (II, QQ, UU) or [6, npix] (II, IQ, IU, QQ, QU, UU);
        obs None, a common mask [npix], or a pair (obs_t, obs_p) of a
        temperature and a polarization mask (nonzero = observed)."""
        ncov = np.asarray(ncov)
        rows = ncov.shape[0] if ncov.ndim == 2 else 0
        if rows not in (3, 6):
            raise ValueError(f"ncov must be [3, npix] or [6, npix], got {ncov.shape}")
        layout = NCOV_SYM6 if rows == 6 else NCOV_DIAG3
        ncov = _f64(ncov, (rows, self.npix))
        if isinstance(obs, (tuple, list)):
            ot, pt = self._mask(obs[0])
            op, pp = self._mask(obs[1])
            self._check(lib().dm_set_noise_masks(self._h, _dptr(ncov), layout, pt, pp))
        else:
            o, ptr = self._mask(obs)
            self._check(lib().dm_set_noise(self._h, _dptr(ncov), layout, ptr))

    def set_schedule(self, lambda_start=1e3, nsteps=20, iters_per_step=10, max_iters=0):
        """Fixed mode: nsteps cooling steps lambda_start -> 1, iters_per_step
        each; max_iters > 0 stops a solve after that many iterations in
        total (it can be resumed from a checkpoint)."""
        s = DmSchedule(float(lambda_start), int(nsteps), int(iters_per_step), 0.0, 0.0, 0.0, 0.0, int(max_iters))
        self._check(lib().dm_set_schedule(self._h, ctypes.byref(s)))

    def set_schedule_eps(self, lambda_start=1e3, beta=0.75, eps_start=1e-4, eps_end=1e-6, eta=1.1,
                         max_iters=100000):
        """Epsilon mode (Algorithm 1's stopping rule with the cooled threshold)."""
        s = DmSchedule(float(lambda_start), 0, 0, float(beta), float(eps_start), float(eps_end), float(eta),
                       int(max_iters))
        self._check(lib().dm_set_schedule(self._h, ctypes.byref(s)))

    def autotune(self, nrhs):
        """Pick the launch shapes for nrhs RHS; returns dict(syn_mchunk,
        ana_mchunk, syn_waves, ring_big_threads, ring_small_threads, syn_ms,
        ana_ms, ring_ms)."""
        ch = (ctypes.c_int * 5)()
        ms = (ctypes.c_double * 3)()
        self._check(lib().dm_autotune(self._h, int(nrhs), ch, ms))
        return dict(syn_mchunk=ch[0], ana_mchunk=ch[1], syn_waves=ch[2], ring_big_threads=ch[3],
                    ring_small_threads=ch[4], syn_ms=ms[0], ana_ms=ms[1], ring_ms=ms[2])

    def checkpoint_save(self, path):
        """Write where the last Wiener filter solve stopped to path."""
        self._check(lib().dm_checkpoint_save(self._h, os.fsencode(path)))

    def checkpoint_load(self, path):
        """Load a checkpoint; the next Wiener filter call continues from it."""
        self._check(lib().dm_checkpoint_load(self._h, os.fsencode(path)))

    def set_refinement(self, ncorrections):
        """Appendix A's corrections after every later solve (0 = off)."""
        self._check(lib().dm_set_refinement(self._h, int(ncorrections)))

    def set_refinement_select(self, keep_best):
        """Return the last iterate (False, Appendix A) or the iterate of
        smallest residual (True) from a refined solve."""
        self._check(lib().dm_set_refinement_select(self._h, 1 if keep_best else 0))

    def refinement_selected(self):
        """Per RHS of the last refined solve, the index (into
        refinement_trace()'s rows) of the iterate it returned."""
        n = ctypes.c_int(0)
        self._check(lib().dm_refinement_selected(self._h, None, 0, ctypes.byref(n)))
        idx = np.zeros(n.value, dtype=np.int32)
        self._check(lib().dm_refinement_selected(self._h, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                                 n.value, ctypes.byref(n)))
        return idx

    def refinement_trace(self):
        """Relative residual norms of the last refined solve, [ncorr + 1, nrhs]
        (before each correction and after the last)."""
        n, b = ctypes.c_int(0), ctypes.c_int(0)
        self._check(lib().dm_refinement_trace(self._h, None, 0, ctypes.byref(n), ctypes.byref(b)))
        h = np.zeros(n.value)
        self._check(lib().dm_refinement_trace(self._h, h.ctypes.data_as(_D), n.value, ctypes.byref(n),
                                              ctypes.byref(b)))
        return h.reshape(-1, b.value) if n.value else h.reshape(0, 0)

    def set_adaptive_resolution(self, factor):
        """Per cooling step band limit min(lmax, ceil(factor ell_iter(mu)))
        (0 = off, else >= 1)."""
        self._check(lib().dm_set_adaptive_resolution(self._h, float(factor)))

    def step_band_limits(self):
        """Band limit of each cooling step of the last solve."""
        n = ctypes.c_int(0)
        self._check(lib().dm_step_band_limits(self._h, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int32)
        self._check(lib().dm_step_band_limits(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n.value,
                                              ctypes.byref(n)))
        return out

    def set_diagnostics(self, every):
        """Record chi^2 (eq 3) and the Appendix C residual of the iterate
        after every `every`-th iteration and the last (0 = off)."""
        self._check(lib().dm_set_diagnostics(self._h, int(every)))

    def diagnostics_trace(self):
        """(iteration [n], chi2 [n, nrhs], residual [n, nrhs]) of the last solve."""
        n, b = ctypes.c_int(0), ctypes.c_int(0)
        self._check(lib().dm_diagnostics_trace(self._h, None, None, None, 0, ctypes.byref(n), ctypes.byref(b)))
        it = np.zeros(n.value, dtype=np.int32)
        w = max(b.value, 1)
        c2 = np.zeros(n.value * w)
        rs = np.zeros(n.value * w)
        self._check(lib().dm_diagnostics_trace(self._h, it.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                               c2.ctypes.data_as(_D), rs.ctypes.data_as(_D), n.value,
                                               ctypes.byref(n), ctypes.byref(b)))
        return it, c2.reshape(n.value, w), rs.reshape(n.value, w)

    def schedule_trace(self):
        """(cauchy [n], step [n]) of the last epsilon-mode solve."""
        n = ctypes.c_int(0)
        self._check(lib().dm_schedule_trace(self._h, None, None, 0, ctypes.byref(n)))
        c = np.zeros(n.value)
        st = np.zeros(n.value, dtype=np.int32)
        self._check(lib().dm_schedule_trace(self._h, c.ctypes.data_as(_D),
                                            st.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), n.value,
                                            ctypes.byref(n)))
        return c, st

    # -- solves ------------------------------------------------------------
    def wiener_filter(self, d, want_map=False, want_stats=False):
        d = np.asarray(d, dtype=np.float64)
        nrhs = 1 if d.ndim == 2 else d.shape[0]
        d = _f64(d, (nrhs, 3, self.npix))
        alm = np.empty((nrhs, 3, self.nalm), dtype=np.complex128)
        mp = np.empty((nrhs, 3, self.npix)) if want_map else None
        stats = (DmStats * nrhs)() if want_stats else None
        self._check(lib().dm_wiener_filter(self._h, nrhs, _dptr(d), alm.ctypes.data_as(_D),
                                           _dptr(mp) if mp is not None else None, stats))
        out = {"alm": alm}
        if mp is not None:
            out["map"] = mp
        if stats is not None:
            out["stats"] = [s.as_dict() for s in stats]
        return out

    def wiener_filter_device(self, d, alm, map=None, stream=None, want_stats=False):
        """d: torch [nrhs, 3, npix] on the GPU; alm: torch tensor of nrhs*3*nalm
        complex values as (re, im) pairs; map: optional torch [nrhs, 3, npix].
        All float64, or all float32 (dm_wiener_filter_device_f32)."""
        nrhs = d.shape[0]
        stats = (DmStats * nrhs)() if want_stats else None
        sp = _P(stream.cuda_stream) if stream is not None else None
        nm, na = nrhs * 3 * self.npix, nrhs * 3 * self.nalm * 2
        dt = str(d.dtype)
        if dt not in ("torch.float64", "torch.float32"):
            raise ValueError(f"d must be float64 or float32, not {d.dtype}")
        fn = lib().dm_wiener_filter_device if dt == "torch.float64" else lib().dm_wiener_filter_device_f32
        self._check(fn(self._h, nrhs, _dev(d, nm, "d", dt), _dev(alm, na, "alm", dt),
                       _dev(map, nm, "map", dt) if map is not None else None, sp, stats))
        return [s.as_dict() for s in stats] if stats is not None else None

    def constrained_realizations(self, d, shat, dhat, want_f=False):
        nreal = shat.shape[0]
        d = _f64(d, (3, self.npix))
        shat = _c64(shat, (nreal, 3, self.nalm))
        dhat = _f64(dhat, (nreal, 3, self.npix))
        scr = np.empty((nreal, 3, self.nalm), dtype=np.complex128)
        f = np.empty_like(scr) if want_f else None
        self._check(lib().dm_constrained_realizations(self._h, nreal, _dptr(d), shat.ctypes.data_as(_D), _dptr(dhat),
                                                      scr.ctypes.data_as(_D),
                                                      f.ctypes.data_as(_D) if f is not None else None))
        return (scr, f) if want_f else scr

    # -- single transforms -------------------------------------------------
    def alm2map(self, alm):
        alm = np.asarray(alm)
        nrhs = 1 if alm.ndim == 2 else alm.shape[0]
        a = _c64(alm, (nrhs, 3, self.nalm))
        out = np.empty((nrhs, 3, self.npix))
        self._check(lib().dm_alm2map(self._h, nrhs, a.ctypes.data_as(_D), _dptr(out)))
        return out if alm.ndim == 3 else out[0]

    def _m2a(self, fn, m):
        m = np.asarray(m, dtype=np.float64)
        nrhs = 1 if m.ndim == 2 else m.shape[0]
        mm = _f64(m, (nrhs, 3, self.npix))
        out = np.empty((nrhs, 3, self.nalm), dtype=np.complex128)
        self._check(fn(self._h, nrhs, _dptr(mm), out.ctypes.data_as(_D)))
        return out if m.ndim == 3 else out[0]

    def map2alm(self, m):
        return self._m2a(lib().dm_map2alm, m)

    def adjoint(self, m):
        return self._m2a(lib().dm_alm2map_adjoint, m)

    def alm2map_device(self, alm, map, stream=None):
        """alm: torch float64 [nrhs, 3, 2 nalm] on the GPU; map: [nrhs, 3, npix]."""
        nrhs = alm.shape[0]
        sp = _P(stream.cuda_stream) if stream is not None else None
        self._check(lib().dm_alm2map_device(self._h, nrhs, _dev(alm, nrhs * 3 * self.nalm * 2, "alm"),
                                            _dev(map, nrhs * 3 * self.npix, "map"), sp))

    def map2alm_device(self, map, alm, stream=None):
        """map: torch float64 [nrhs, 3, npix] on the GPU; alm: [nrhs, 3, 2 nalm]."""
        nrhs = map.shape[0]
        sp = _P(stream.cuda_stream) if stream is not None else None
        self._check(lib().dm_map2alm_device(self._h, nrhs, _dev(map, nrhs * 3 * self.npix, "map"),
                                            _dev(alm, nrhs * 3 * self.nalm * 2, "alm"), sp))

    def map2alm_device_noalloc(self, map, alm, stream=None):
        """map2alm_device with its work memory in the library's fixed
        device array (no allocation; calls overlapping on one GPU race)."""
        nrhs = map.shape[0]
        sp = _P(stream.cuda_stream) if stream is not None else None
        self._check(lib().dm_map2alm_device_noalloc(self._h, nrhs, _dev(map, nrhs * 3 * self.npix, "map"),
                                                    _dev(alm, nrhs * 3 * self.nalm * 2, "alm"), sp))

    def iterate(self, d, t, lam, niter):
        d = np.asarray(d, dtype=np.float64)
        nrhs = 1 if d.ndim == 2 else d.shape[0]
        dd = _f64(d, (nrhs, 3, self.npix))
        tt = _f64(t, (nrhs, 3, self.npix))
        alm = np.empty((nrhs, 3, self.nalm), dtype=np.complex128)
        tout = np.empty((nrhs, 3, self.npix))
        self._check(lib().dm_iterate(self._h, nrhs, _dptr(dd), _dptr(tt), float(lam), int(niter),
                                     alm.ctypes.data_as(_D), _dptr(tout)))
        if d.ndim == 2:
            return alm[0], tout[0]
        return alm, tout

    def transform_work(self):
        """(points, executed) of one Legendre transform per RHS: ring pairs x
        nalm, and the points at or above their start degrees."""
        a, b = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(lib().dm_transform_work(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # -- profiling ---------------------------------------------------------
    def profile(self, enable=True):
        self._check(lib().dm_profile_enable(self._h, 1 if enable else 0))

    def kernel_times(self):
        ms = (ctypes.c_double * 8)()
        n = (ctypes.c_int64 * 8)()
        cnt = ctypes.c_int(8)
        self._check(lib().dm_kernel_times(self._h, ms, n, ctypes.byref(cnt)))
        return {KERNEL_CLASSES[k]: (ms[k], n[k]) for k in range(min(cnt.value, len(KERNEL_CLASSES)))}
