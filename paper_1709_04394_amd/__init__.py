"""libmcspin: MI355X (gfx950) Monte Carlo engine for Ising-type spin models.

This module is the Python binding of the C ABI in ``include/mcspin.h``.  It
only marshals arguments: PyTorch provides device memory and the current HIP
stream, and every step of the method runs in the library's HIP kernels.  If
``libmcspin.so`` has not been built the import fails loudly; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmcspin.so")

INT8, MSC64 = 0, 1
METROPOLIS, HEATBATH = 0, 1
COLD, HOT = 0, 1
MUCA_HOT, MUCA_STRATIFIED = 0, 1

MC_OK, MC_E_INVAL, MC_E_SHAPE, MC_E_RANGE, MC_E_LAYOUT, MC_E_WORKSPACE, MC_E_DEVICE, MC_E_NOTCONV, MC_E_IO = \
    0, -1, -2, -3, -4, -5, -6, -7, -8


class MCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libmcspin error %d: %s" % (code, msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("libmcspin.so is not built (expected at %s); run "
                      "`python -m paper_1709_04394_amd.build` or __graft_entry__.build()" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p


class Geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32), ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("Lz", ctypes.c_int32), ("layout", ctypes.c_int32), ("count", ctypes.c_int32)]

    @property
    def N(self):
        return self.Lx * self.Ly * (self.Lz if self.dims == 3 else 1)

    @property
    def lanes(self):
        return 64 if self.layout == MSC64 else 1


class PAArgs(ctypes.Structure):
    _fields_ = [("npop", ctypes.c_int32), ("L", ctypes.POINTER(ctypes.c_int32)), ("R", ctypes.c_int32),
                ("theta", ctypes.c_int32), ("seed", ctypes.c_uint64), ("step_first", ctypes.c_int32),
                ("nsteps", ctypes.c_int32), ("beta", ctypes.POINTER(ctypes.c_double))]


class PTArgs(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("n_temps", ctypes.c_int32), ("n_sets", ctypes.c_int32),
                ("beta", ctypes.POINTER(ctypes.c_double)), ("theta", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("round0", ctypes.c_uint64), ("rounds", ctypes.c_int32)]


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int64)


class MucaArgs(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("walkers", ctypes.c_int32), ("eq_sweeps", ctypes.c_int32),
                ("rec_sweeps", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("prod_sweeps", ctypes.c_int32),
                ("flat", ctypes.c_double), ("seed", ctypes.c_uint64), ("start", ctypes.c_int32),
                ("rec_max", ctypes.c_int32), ("eq_scale", ctypes.c_int32), ("prep_sweeps", ctypes.c_int32),
                ("rec_rule", ctypes.c_int32), ("progress", PROGRESS_FN), ("progress_user", ctypes.c_void_p)]


class MucaStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("sweeps_per_walker", ctypes.c_int64),
                ("min_over_max", ctypes.c_double)]


WL_PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64)


class WlArgs(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("nwin", ctypes.c_int32), ("lo", ctypes.POINTER(ctypes.c_int32)),
                ("hi", ctypes.POINTER(ctypes.c_int32)), ("walkers", ctypes.c_int32), ("check_sweeps", ctypes.c_int32),
                ("flat", ctypes.c_double), ("lnf_final", ctypes.c_double), ("max_sweeps", ctypes.c_int64),
                ("max_pass", ctypes.c_int32), ("seed", ctypes.c_uint64), ("progress", WL_PROGRESS_FN),
                ("progress_user", ctypes.c_void_p)]


class WlWindowStats(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("converged", ctypes.c_int32), ("sweeps", ctypes.c_int64)]


class MucaWinArgs(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("nwin", ctypes.c_int32), ("lo", ctypes.POINTER(ctypes.c_int32)),
                ("hi", ctypes.POINTER(ctypes.c_int32)), ("walkers", ctypes.c_int32), ("eq_sweeps", ctypes.c_int32),
                ("rec_sweeps", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("flat", ctypes.c_double),
                ("max_pass", ctypes.c_int32), ("seed", ctypes.c_uint64), ("progress", WL_PROGRESS_FN),
                ("progress_user", ctypes.c_void_p)]


class MucaWinStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32)]


class MlpArgs(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class SweepArgs(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("beta", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("replica0", ctypes.c_uint32), ("sweep0", ctypes.c_uint64), ("nsweeps", ctypes.c_int32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_c = ctypes
_lib_fns = dict(
    mc_abi_version=_sig("mc_abi_version", _c.c_int, []),
    mc_strerror=_sig("mc_strerror", _c.c_char_p, [_c.c_int]),
    mc_ctx_create=_sig("mc_ctx_create", _c.c_int, [_c.POINTER(_vp), _c.c_int]),
    mc_ctx_destroy=_sig("mc_ctx_destroy", None, [_vp]),
    mc_ctx_last_error=_sig("mc_ctx_last_error", _c.c_char_p, [_vp]),
    mc_init=_sig("mc_init", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _c.c_int32, _c.c_uint64, _c.c_uint32, _vp]),
    mc_couplings=_sig("mc_couplings", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _c.c_uint64, _vp]),
    mc_sweep_workspace_bytes=_sig("mc_sweep_workspace_bytes", _c.c_size_t, [_c.POINTER(Geom)]),
    mc_sweep=_sig("mc_sweep", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _vp, _c.POINTER(SweepArgs), _vp, _vp,
                                         _c.c_size_t, _vp]),
    mc_measure=_sig("mc_measure", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _vp, _vp, _vp]),
    mc_static_scratch_bytes=_sig("mc_static_scratch_bytes", _c.c_size_t, []),
    mc_sweep_noalloc=_sig("mc_sweep_noalloc", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _vp, _c.POINTER(SweepArgs), _vp,
                                                         _vp]),
    mc_couplings_msc64=_sig("mc_couplings_msc64", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _c.c_uint64, _c.c_uint32,
                                                             _vp]),
    mc_sweep_sg_msc64=_sig("mc_sweep_sg_msc64", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _vp, _c.POINTER(SweepArgs),
                                                           _vp, _vp]),
    mc_dcb_workspace_bytes=_sig("mc_dcb_workspace_bytes", _c.c_size_t, [_c.POINTER(Geom)]),
    mc_sweep_dcb=_sig("mc_sweep_dcb", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _c.POINTER(SweepArgs), _c.c_int32,
                                                 _c.c_int32, _vp, _vp, _c.c_size_t, _vp]),
    mc_sweep_betas=_sig("mc_sweep_betas", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _vp, _c.POINTER(SweepArgs),
                                                     _c.POINTER(_c.c_double), _vp, _vp, _c.c_size_t, _vp]),
    mc_set_tile_plan=_sig("mc_set_tile_plan", _c.c_int, [_vp, _c.POINTER(Geom), _c.c_int32, _c.c_int32,
                                                         _c.c_int32]),
    mc_get_tile_plan=_sig("mc_get_tile_plan", _c.c_int, [_vp, _c.POINTER(Geom), _c.POINTER(_c.c_int32),
                                                         _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32)]),
    mc_tune_sweep=_sig("mc_tune_sweep", _c.c_int, [_vp, _c.POINTER(Geom), _vp, _vp, _c.c_double, _c.c_int32,
                                                   _vp]),
    mc_tune_sweep_rule=_sig("mc_tune_sweep_rule", _c.c_int, [_vp, _c.POINTER(Geom), _c.c_int32, _vp, _vp,
                                                             _c.c_double, _c.c_int32, _vp]),
    mc_mlp_param_count=_sig("mc_mlp_param_count", _c.c_int32, []),
    mc_mlp_workspace_bytes=_sig("mc_mlp_workspace_bytes", _c.c_size_t, [_c.c_int32]),
    mc_mlp_training_set=_sig("mc_mlp_training_set", _c.c_int,
                             [_vp, _c.c_int32, _c.POINTER(_c.c_int32), _c.POINTER(_c.POINTER(_c.c_double)),
                              _c.POINTER(_c.c_float), _c.POINTER(_c.c_float), _c.c_int32, _c.POINTER(_c.c_int32)]),
    mc_mlp_lnw_workspace_bytes=_sig("mc_mlp_lnw_workspace_bytes", _c.c_size_t, [_c.c_int32]),
    mc_mlp_lnw_init=_sig("mc_mlp_lnw_init", _c.c_int, [_vp, _vp, _c.c_int32, _c.POINTER(_c.c_double),
                                                         _c.POINTER(_c.c_int32), _vp, _c.c_size_t, _vp]),
    mc_mlp_init=_sig("mc_mlp_init", _c.c_int, [_vp, _vp, _c.c_uint64, _vp]),
    mc_mlp_grad=_sig("mc_mlp_grad", _c.c_int, [_vp, _vp, _vp, _vp, _c.c_int32, _vp, _vp, _vp, _c.c_size_t, _vp]),
    mc_mlp_train=_sig("mc_mlp_train", _c.c_int, [_vp, _c.POINTER(MlpArgs), _vp, _vp, _c.c_int32, _vp, _vp, _vp,
                                                 _c.c_size_t, _vp]),
    mc_mlp_predict=_sig("mc_mlp_predict", _c.c_int, [_vp, _vp, _vp, _c.c_int32, _vp, _vp]),
    mc_muca_workspace_bytes=_sig("mc_muca_workspace_bytes", _c.c_size_t, [_c.c_int32, _c.c_int32]),
    mc_muca_start=_sig("mc_muca_start", _c.c_int, [_vp, _c.c_int32, _c.c_int32, _c.c_uint64, _c.c_int32, _vp, _vp,
                                                   _vp]),
    mc_muca_sweeps=_sig("mc_muca_sweeps", _c.c_int, [_vp, _c.c_int32, _c.c_int32, _vp, _vp, _c.POINTER(_c.c_double),
                                                     _c.c_uint64, _c.c_uint64, _c.c_int32, _c.c_int32, _vp, _vp,
                                                     _c.c_size_t, _vp]),
    mc_muca_run=_sig("mc_muca_run", _c.c_int, [_vp, _c.POINTER(MucaArgs), _c.POINTER(_c.c_double), _vp,
                                               _c.POINTER(_c.c_double), _c.POINTER(_c.c_int64),
                                               _c.POINTER(_c.c_double), _c.POINTER(_c.c_double),
                                               _c.POINTER(MucaStats), _vp, _c.c_size_t, _vp]),
    mc_pa_workspace_bytes=_sig("mc_pa_workspace_bytes", _c.c_size_t, [_c.POINTER(PAArgs)]),
    mc_pa_anneal=_sig("mc_pa_anneal", _c.c_int, [_vp, _c.POINTER(PAArgs), _c.POINTER(_vp), _c.POINTER(_c.c_double),
                                                 _c.POINTER(_c.c_double), _c.POINTER(_c.c_double),
                                                 _c.POINTER(_c.c_int64), _vp, _c.c_size_t, _vp]),
    mc_set_pa_group=_sig("mc_set_pa_group", _c.c_int, [_vp, _c.c_int32, _c.c_int32]),
    mc_wl_workspace_bytes=_sig("mc_wl_workspace_bytes", _c.c_size_t, [_c.POINTER(WlArgs)]),
    mc_win_drive=_sig("mc_win_drive", _c.c_int, [_vp, _c.c_int32, _c.c_int32, _vp, _vp, _c.c_int32, _c.c_uint64,
                                                 _c.c_int32, _vp, _vp, _vp, _c.c_size_t, _vp]),
    mc_wl_sweeps=_sig("mc_wl_sweeps", _c.c_int, [_vp, _c.c_int32, _c.c_int32, _vp, _vp, _c.c_int32, _vp, _vp,
                                                 _c.c_double, _c.c_uint64, _c.c_uint64, _c.c_int32, _vp, _vp, _vp,
                                                 _vp, _vp, _vp, _c.c_size_t, _vp]),
    mc_wl_run=_sig("mc_wl_run", _c.c_int, [_vp, _c.POINTER(WlArgs), _vp, _vp, _c.POINTER(_c.c_double),
                                           _c.POINTER(_c.c_double), _c.POINTER(WlWindowStats), _vp, _c.c_size_t,
                                           _vp]),
    mc_muca_windows_workspace_bytes=_sig("mc_muca_windows_workspace_bytes", _c.c_size_t, [_c.POINTER(MucaWinArgs)]),
    mc_muca_windows_run=_sig("mc_muca_windows_run", _c.c_int, [_vp, _c.POINTER(MucaWinArgs), _vp, _vp,
                                                               _c.POINTER(_c.c_double), _c.POINTER(_c.c_double),
                                                               _c.POINTER(MucaWinStats), _vp, _c.c_size_t, _vp]),
    mc_muca_update=_sig("mc_muca_update", _c.c_int, [_vp, _c.c_int32, _c.POINTER(_c.c_double),
                                                     _c.POINTER(_c.c_int64), _c.POINTER(_c.c_double),
                                                     _c.POINTER(_c.c_double)]),
    mc_sweep_path=_sig("mc_sweep_path", _c.c_int, [_vp, _c.POINTER(Geom), _c.c_int32, _c.c_int32, _c.c_int32,
                                                   _c.c_size_t, _c.POINTER(_c.c_int32)]),
    mc_pt_exchange=_sig("mc_pt_exchange", _c.c_int, [_vp, _c.c_int32, _c.POINTER(_c.c_double),
                                                     _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int32),
                                                     _c.POINTER(_c.c_int32), _c.c_uint64, _c.c_uint64,
                                                     _c.POINTER(_c.c_int64)]),
    mc_pt_workspace_bytes=_sig("mc_pt_workspace_bytes", _c.c_size_t, [_c.POINTER(PTArgs)]),
    mc_pt_run=_sig("mc_pt_run", _c.c_int, [_vp, _c.POINTER(PTArgs), _vp, _c.POINTER(_c.c_int32),
                                           _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64),
                                           _vp, _c.c_size_t, _vp]),
    mc_tuning_save=_sig("mc_tuning_save", _c.c_int, [_vp, _c.c_char_p]),
    mc_tuning_load=_sig("mc_tuning_load", _c.c_int, [_vp, _c.c_char_p]),
    mc_get_pa_group=_sig("mc_get_pa_group", _c.c_int, [_vp, _c.c_int32, _c.POINTER(_c.c_int32)]),
    mc_tune_pa=_sig("mc_tune_pa", _c.c_int, [_vp, _c.POINTER(PAArgs), _c.POINTER(_vp), _vp, _c.c_size_t,
                                             _c.POINTER(_c.c_int32), _vp]),
)


def exported_symbols():
    return sorted(_lib_fns)


def abi_version():
    return _lib.mc_abi_version()


def strerror(code):
    return _lib.mc_strerror(code).decode()


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return _vp(t.data_ptr())


def _stream(device):
    return _vp(torch.cuda.current_stream(device).cuda_stream)


def make_geom(dims, L, layout=INT8, count=1):
    if isinstance(L, int):
        L = (L,) * dims
    Lz = L[2] if dims == 3 else 1
    return Geom(dims, L[0], L[1], Lz, layout, count)


def lattice_tensor(geom, device="cuda"):
    """Uninitialised lattice buffer of the geometry: int8 [count, N] or the
    MSC64 words as int64 [count, N] (bit-identical to uint64)."""
    dt = torch.int8 if geom.layout == INT8 else torch.int64
    return torch.empty((geom.count, geom.N), dtype=dt, device=device)


class Context:
    """A libmcspin context bound to one HIP device (host state only)."""

    def __init__(self, device=0):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        h = _vp()
        rc = _lib.mc_ctx_create(ctypes.byref(h), self.device.index or 0)
        if rc != MC_OK:
            raise MCError(rc, "mc_ctx_create(device=%s): %s" % (device, strerror(rc)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.mc_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != MC_OK:
            detail = _lib.mc_ctx_last_error(self._h)
            raise MCError(rc, "%s: %s (%s)" % (what, strerror(rc), detail.decode() if detail else ""))
        return rc

    # -------------------------------------------------------------- lattices
    def init(self, geom, spins, start, seed, replica0=0):
        return self._check(_lib.mc_init(self._h, ctypes.byref(geom), _ptr(spins), start, seed, replica0,
                                        _stream(self.device)), "mc_init")

    def couplings(self, geom, J, seed):
        return self._check(_lib.mc_couplings(self._h, ctypes.byref(geom), _ptr(J), seed, _stream(self.device)),
                           "mc_couplings")

    def sweep_workspace_bytes(self, geom):
        return int(_lib.mc_sweep_workspace_bytes(ctypes.byref(geom)))

    def sweep(self, geom, spins, beta, seed, nsweeps, sweep0=0, replica0=0, rule=METROPOLIS, J=None, EM=None,
              ws=None):
        a = SweepArgs(rule, float(beta), seed, replica0, sweep0, nsweeps)
        wsb = 0 if ws is None else ws.numel() * ws.element_size()
        return self._check(_lib.mc_sweep(self._h, ctypes.byref(geom), _ptr(spins), _ptr(J), ctypes.byref(a),
                                         _ptr(EM), _ptr(ws), wsb, _stream(self.device)), "mc_sweep")

    def sweep_noalloc(self, geom, spins, beta, seed, nsweeps, sweep0=0, replica0=0, rule=METROPOLIS, J=None,
                      EM=None):
        """mc_sweep_noalloc: the sweep with the library's fixed device scratch
        instead of a workspace (allocates nothing)."""
        a = SweepArgs(rule, float(beta), seed, replica0, sweep0, nsweeps)
        return self._check(_lib.mc_sweep_noalloc(self._h, ctypes.byref(geom), _ptr(spins), _ptr(J), ctypes.byref(a),
                                                 _ptr(EM), _stream(self.device)), "mc_sweep_noalloc")

    def couplings_msc64(self, geom, J, seed, realisation0=0):
        """Couplings of 64 realisations per word (mc_couplings_msc64) into J,
        an int64 tensor [count, dims * N] (bit-identical to uint64)."""
        return self._check(_lib.mc_couplings_msc64(self._h, ctypes.byref(geom), _ptr(J), seed, realisation0,
                                                   _stream(self.device)), "mc_couplings_msc64")

    def sweep_sg_msc64(self, geom, spins, J, beta, seed, nsweeps, sweep0=0, replica0=0, rule=METROPOLIS, EM=None):
        """Sweeps of spin glasses coded across realisations, one shared random
        number per site (mc_sweep_sg_msc64)."""
        a = SweepArgs(rule, float(beta), seed, replica0, sweep0, nsweeps)
        return self._check(_lib.mc_sweep_sg_msc64(self._h, ctypes.byref(geom), _ptr(spins), _ptr(J), ctypes.byref(a),
                                                  _ptr(EM), _stream(self.device)), "mc_sweep_sg_msc64")

    def dcb_workspace_bytes(self, geom):
        return int(_lib.mc_dcb_workspace_bytes(ctypes.byref(geom)))

    def sweep_dcb(self, geom, spins, beta, seed, nsweeps, tile, hits, sweep0=0, replica0=0, EM=None, ws=None):
        """Double-checkerboard Metropolis sweeps with `hits` updates per tile
        (mc_sweep_dcb); ws defaults to a fresh workspace."""
        if ws is None:
            ws = torch.empty(max(1, self.dcb_workspace_bytes(geom)), dtype=torch.uint8, device=self.device)
        a = SweepArgs(METROPOLIS, float(beta), seed, replica0, sweep0, nsweeps)
        return self._check(_lib.mc_sweep_dcb(self._h, ctypes.byref(geom), _ptr(spins), ctypes.byref(a), tile, hits,
                                             _ptr(EM), _ptr(ws), ws.numel() * ws.element_size(),
                                             _stream(self.device)), "mc_sweep_dcb")

    def sweep_betas(self, geom, spins, betas, seed, nsweeps, sweep0=0, replica0=0, rule=METROPOLIS, J=None,
                    EM=None, ws=None):
        if len(betas) != geom.count:
            raise ValueError("need one beta per lattice")
        b = (ctypes.c_double * geom.count)(*[float(x) for x in betas])
        a = SweepArgs(rule, float(betas[0]), seed, replica0, sweep0, nsweeps)
        wsb = 0 if ws is None else ws.numel() * ws.element_size()
        return self._check(_lib.mc_sweep_betas(self._h, ctypes.byref(geom), _ptr(spins), _ptr(J), ctypes.byref(a), b,
                                               _ptr(EM), _ptr(ws), wsb, _stream(self.device)), "mc_sweep_betas")

    def measure(self, geom, spins, EM, J=None):
        return self._check(_lib.mc_measure(self._h, ctypes.byref(geom), _ptr(spins), _ptr(J), _ptr(EM),
                                           _stream(self.device)), "mc_measure")

    # --------------------------------------------------------- population annealing
    @staticmethod
    def _pa_args(Ls, R, theta, seed, beta, step_first, nsteps):
        import numpy as np

        Larr = (ctypes.c_int32 * len(Ls))(*[int(x) for x in Ls])
        barr = np.ascontiguousarray(beta, dtype=np.float64)
        a = PAArgs(len(Ls), Larr, R, theta, seed, step_first, nsteps,
                   barr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        return a, (Larr, barr)

    def pa_workspace_bytes(self, Ls, R, theta, beta, step_first=1, nsteps=None):
        nsteps = len(beta) - step_first if nsteps is None else nsteps
        a, keep = self._pa_args(Ls, R, theta, 0, beta, step_first, nsteps)
        return int(_lib.mc_pa_workspace_bytes(ctypes.byref(a)))

    def pa_population_tensors(self, Ls, R):
        """One device buffer of 2 R L^2 int8 per population (current population
        in the first half)."""
        return [torch.empty(2 * R * L * L, dtype=torch.int8, device=self.device) for L in Ls]

    def pa_anneal(self, Ls, R, theta, seed, beta, pops, step_first=1, nsteps=None, lnZ0=None, ws=None):
        """Run annealing steps step_first .. step_first + nsteps - 1; returns a dict
        with Ctot, lnQ ([npop][nsteps]), lnZ ([npop][nsteps+1]) and hist (list of
        [nsteps+1][L^2+1] int64 arrays)."""
        import numpy as np

        nsteps = len(beta) - step_first if nsteps is None else nsteps
        a, keep = self._pa_args(Ls, R, theta, seed, beta, step_first, nsteps)
        need = int(_lib.mc_pa_workspace_bytes(ctypes.byref(a)))
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
        npop = len(Ls)
        ptrs = (_vp * npop)(*[_vp(t.data_ptr()) for t in pops])
        Ctot = np.zeros((npop, max(nsteps, 1)), dtype=np.float64)
        lnQ = np.zeros((npop, max(nsteps, 1)), dtype=np.float64)
        lnZ = np.zeros((npop, nsteps + 1), dtype=np.float64)
        if lnZ0 is not None:
            lnZ[:, 0] = lnZ0
        hist = np.zeros(sum((nsteps + 1) * (L * L + 1) for L in Ls), dtype=np.int64)
        dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._check(_lib.mc_pa_anneal(self._h, ctypes.byref(a), ptrs, dp(Ctot), dp(lnQ), dp(lnZ),
                                      hist.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(ws),
                                      ws.numel() * ws.element_size(), _stream(self.device)), "mc_pa_anneal")
        out, off = [], 0
        for L in Ls:
            n = (nsteps + 1) * (L * L + 1)
            out.append(hist[off:off + n].reshape(nsteps + 1, L * L + 1))
            off += n
        return dict(Ctot=Ctot[:, :nsteps], lnQ=lnQ[:, :nsteps], lnZ=lnZ, hist=out)

    def set_pa_group(self, L, G):
        """Replicas per workgroup for populations of extent L (0: built-in rule)."""
        return self._check(_lib.mc_set_pa_group(self._h, L, G), "mc_set_pa_group")

    def muca_update(self, L, lnW, H):
        """One step of the weight recursion (mc_muca_update): returns the new
        ln W (float64 [N/2 + 1]) and the flatness min/max of H."""
        import numpy as np

        K = L * L // 2
        lnW = np.ascontiguousarray(lnW, dtype=np.float64)
        H = np.ascontiguousarray(H, dtype=np.int64)
        if lnW.size != K + 1 or H.size != K + 1:
            raise ValueError("lnW and H need L^2 / 2 + 1 entries")
        out = np.empty(K + 1, dtype=np.float64)
        flat = ctypes.c_double()
        p = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
        self._check(_lib.mc_muca_update(self._h, L, p(lnW, ctypes.c_double), p(H, ctypes.c_int64),
                                        p(out, ctypes.c_double), ctypes.byref(flat)), "mc_muca_update")
        return out, flat.value

    def pt_exchange(self, beta, E, temp_of, replica_at, seed, round, accepted):
        """One round of replica exchanges (mc_pt_exchange) on numpy arrays:
        beta float64 [n], E int64 [n] by replica, temp_of / replica_at int32 [n]
        and accepted int64 [n-1], the last three updated in place."""
        import numpy as np

        beta = np.ascontiguousarray(beta, dtype=np.float64)
        E = np.ascontiguousarray(E, dtype=np.int64)
        for a, dt in ((temp_of, np.int32), (replica_at, np.int32), (accepted, np.int64)):
            if not (isinstance(a, np.ndarray) and a.dtype == dt and a.flags.c_contiguous):
                raise TypeError("temp_of, replica_at: contiguous int32 arrays; accepted: contiguous int64")
        n = beta.size
        if E.size != n or temp_of.size != n or replica_at.size != n or accepted.size != max(n - 1, 0):
            raise ValueError("beta, E, temp_of, replica_at need n entries and accepted n - 1")
        p = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
        return self._check(_lib.mc_pt_exchange(self._h, n, p(beta, ctypes.c_double), p(E, ctypes.c_int64),
                                               p(temp_of, ctypes.c_int32), p(replica_at, ctypes.c_int32), seed,
                                               round, p(accepted, ctypes.c_int64)), "mc_pt_exchange")

    @staticmethod
    def _pt_args(L, beta, n_sets, theta, seed, round0, rounds):
        import numpy as np

        b = np.ascontiguousarray(beta, dtype=np.float64)
        a = PTArgs(L, b.size, n_sets, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), theta, seed, round0, rounds)
        return a, b

    def pt_workspace_bytes(self, L, beta, n_sets, theta, rounds):
        a, keep = self._pt_args(L, beta, n_sets, theta, 0, 0, rounds)
        return int(_lib.mc_pt_workspace_bytes(ctypes.byref(a)))

    def pt_state(self, L, n_temps, n_sets, seed, start=HOT):
        """A fresh tempering run: lattices of replica ids 0 .. n_sets n_temps - 1
        (device int8 [n_sets n_temps, L^2]), identity maps and zero counts."""
        import numpy as np

        g = make_geom(2, L, count=n_sets * n_temps)
        spins = lattice_tensor(g, self.device)
        self.init(g, spins, start, seed, 0)
        ident = np.tile(np.arange(n_temps, dtype=np.int32), (n_sets, 1))
        return dict(spins=spins, temp_of=ident.copy(), replica_at=ident.copy(),
                    accepted=np.zeros((n_sets, n_temps - 1), dtype=np.int64))

    def pt_run(self, L, beta, theta, seed, state, round0, rounds, record=True, ws=None):
        """Rounds of parallel tempering (mc_pt_run) on state (from pt_state:
        device spins, host maps and counts, updated in place); returns E_at
        ([rounds][n_sets][n_temps] int64) or None."""
        import numpy as np

        n_sets, n_temps = state["temp_of"].shape
        a, keep = self._pt_args(L, beta, n_sets, theta, seed, round0, rounds)
        need = int(_lib.mc_pt_workspace_bytes(ctypes.byref(a)))
        if ws is None:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
        E_at = np.zeros((max(rounds, 1), n_sets, n_temps), dtype=np.int64) if record else None
        p = lambda x, t: None if x is None else x.ctypes.data_as(ctypes.POINTER(t))
        for k, dt in (("temp_of", np.int32), ("replica_at", np.int32), ("accepted", np.int64)):
            x = state[k]
            if not (isinstance(x, np.ndarray) and x.dtype == dt and x.flags.c_contiguous):
                raise TypeError("state[%r] must be a contiguous %s array" % (k, dt.__name__))
        self._check(_lib.mc_pt_run(self._h, ctypes.byref(a), _ptr(state["spins"]), p(state["temp_of"], ctypes.c_int32),
                                   p(state["replica_at"], ctypes.c_int32), p(state["accepted"], ctypes.c_int64),
                                   p(E_at, ctypes.c_int64), _ptr(ws), ws.numel() * ws.element_size(),
                                   _stream(self.device)), "mc_pt_run")
        return None if E_at is None else E_at[:rounds]

    def save_launch_shapes(self, path):
        """Write the context's tile plans and PA groups to a text file."""
        return self._check(_lib.mc_tuning_save(self._h, os.fsencode(path)), "mc_tuning_save")

    def load_launch_shapes(self, path):
        """Read launch shapes written by save_launch_shapes (all or none)."""
        return self._check(_lib.mc_tuning_load(self._h, os.fsencode(path)), "mc_tuning_load")

    def get_pa_group(self, L):
        G = ctypes.c_int32()
        self._check(_lib.mc_get_pa_group(self._h, L, ctypes.byref(G)), "mc_get_pa_group")
        return G.value

    def tune_pa(self, Ls, R, theta, seed, beta, pops, step_first=1, nsteps=None, ws=None):
        """Time replicas per workgroup for each extent in Ls and keep the fastest;
        pops and ws are overwritten.  Returns the chosen G per population."""
        import numpy as np

        nsteps = len(beta) - step_first if nsteps is None else nsteps
        a, keep = self._pa_args(Ls, R, theta, seed, beta, step_first, nsteps)
        if ws is None:
            need = max(self.pa_workspace_bytes([L], R, theta, beta, 1, min(step_first - 1 + nsteps, 20))
                       for L in Ls)
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
        ptrs = (_vp * len(Ls))(*[_vp(t.data_ptr()) for t in pops])
        G = np.zeros(len(Ls), dtype=np.int32)
        self._check(_lib.mc_tune_pa(self._h, ctypes.byref(a), ptrs, _ptr(ws), ws.numel() * ws.element_size(),
                                    G.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _stream(self.device)),
                    "mc_tune_pa")
        return [int(g) for g in G]

    # ---------------------------------------------------------------------- MLP
    def mlp_init(self, seed):
        p = torch.empty(int(_lib.mc_mlp_param_count()), dtype=torch.float32, device=self.device)
        self._check(_lib.mc_mlp_init(self._h, _ptr(p), seed, _stream(self.device)), "mc_mlp_init")
        return p

    def _mlp_ws(self, n):
        return torch.empty(int(_lib.mc_mlp_workspace_bytes(n)), dtype=torch.uint8, device=self.device)

    def mlp_grad(self, params, X, Y):
        n = Y.numel()
        g = torch.empty_like(params)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        ws = self._mlp_ws(n)
        self._check(_lib.mc_mlp_grad(self._h, _ptr(params), _ptr(X), _ptr(Y), n, _ptr(g), _ptr(loss), _ptr(ws),
                                     ws.numel(), _stream(self.device)), "mc_mlp_grad")
        return g, loss

    def mlp_train(self, params, X, Y, epochs, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        n = Y.numel()
        log = torch.empty(max(1, epochs), dtype=torch.float32, device=self.device)
        ws = self._mlp_ws(n)
        a = MlpArgs(epochs, lr, beta1, beta2, eps)
        self._check(_lib.mc_mlp_train(self._h, ctypes.byref(a), _ptr(X), _ptr(Y), n, _ptr(params), _ptr(log),
                                      _ptr(ws), ws.numel(), _stream(self.device)), "mc_mlp_train")
        return log[:epochs]

    def mlp_predict(self, params, X):
        n = X.shape[0]
        Y = torch.empty(n, dtype=torch.float32, device=self.device)
        self._check(_lib.mc_mlp_predict(self._h, _ptr(params), _ptr(X), n, _ptr(Y), _stream(self.device)),
                    "mc_mlp_predict")
        return Y

    def mlp_training_set(self, lnW_by_L):
        """(X, Y) host float32 arrays from converged ln W per L (dict L -> array
        of N/2 + 1 doubles), as mc_mlp_training_set builds them."""
        import numpy as np

        Ls = sorted(lnW_by_L)
        arrs = [np.ascontiguousarray(lnW_by_L[L], dtype=np.float64) for L in Ls]
        cap = sum(L * L // 2 for L in Ls)
        X = np.zeros((max(cap, 1), 2), dtype=np.float32)
        Y = np.zeros(max(cap, 1), dtype=np.float32)
        n = ctypes.c_int32()
        Larr = (ctypes.c_int32 * len(Ls))(*Ls)
        parr = (ctypes.POINTER(ctypes.c_double) * len(Ls))(
            *[a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) for a in arrs])
        fp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._check(_lib.mc_mlp_training_set(self._h, len(Ls), Larr, parr, fp(X), fp(Y), cap, ctypes.byref(n)),
                    "mc_mlp_training_set")
        return X[:n.value], Y[:n.value]

    def mlp_lnw_init(self, params, L):
        """Initial ln W (host float64, N/2 + 1 levels) of an L x L lattice from
        a trained network, and whether the flat fallback was used."""
        import numpy as np

        out = np.zeros(L * L // 2 + 1, dtype=np.float64)
        fb = ctypes.c_int32()
        nb = int(_lib.mc_mlp_lnw_workspace_bytes(L))
        if nb == 0:
            raise MCError(MC_E_SHAPE, "unsupported L=%d" % L)
        ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        self._check(_lib.mc_mlp_lnw_init(self._h, _ptr(params), L,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(fb),
                                         _ptr(ws), ws.numel(), _stream(self.device)), "mc_mlp_lnw_init")
        return out, bool(fb.value)

    # ----------------------------------------------------------- multicanonical
    def muca_workspace(self, L, walkers):
        n = int(_lib.mc_muca_workspace_bytes(L, walkers))
        if n == 0:
            raise MCError(MC_E_SHAPE, "unsupported L=%d or walkers=%d" % (L, walkers))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def muca_start(self, L, walkers, seed, spins=None, E=None, start=0):
        spins = torch.empty((walkers, L * L), dtype=torch.int8, device=self.device) if spins is None else spins
        E = torch.empty(walkers, dtype=torch.int64, device=self.device) if E is None else E
        self._check(_lib.mc_muca_start(self._h, L, walkers, seed, start, _ptr(spins), _ptr(E),
                                       _stream(self.device)), "mc_muca_start")
        return spins, E

    def muca_sweeps(self, L, spins, E, lnW, seed, sweep0, nsweeps, record, H=None, ws=None):
        import numpy as np

        walkers = E.numel()
        ws = self.muca_workspace(L, walkers) if ws is None else ws
        lw = np.ascontiguousarray(lnW, dtype=np.float64)
        self._check(_lib.mc_muca_sweeps(self._h, L, walkers, _ptr(spins), _ptr(E),
                                        lw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), seed, sweep0, nsweeps,
                                        1 if record else 0, _ptr(H), _ptr(ws), ws.numel(), _stream(self.device)),
                    "mc_muca_sweeps")

    def muca_run(self, L, walkers, seed, eq_sweeps, rec_sweeps, max_iter, prod_sweeps, flat=0.8, lnW_init=None,
                 spins=None, ws=None, start=0, rec_max=0, eq_scale=0, prep_sweeps=0, rec_rule=0, progress=None):
        """Full multicanonical run; returns a dict like oracle.muca_run."""
        import numpy as np

        K1 = L * L // 2 + 1
        spins = torch.empty((walkers, L * L), dtype=torch.int8, device=self.device) if spins is None else spins
        ws = self.muca_workspace(L, walkers) if ws is None else ws
        cb = PROGRESS_FN(progress) if progress is not None else PROGRESS_FN()
        a = MucaArgs(L, walkers, eq_sweeps, rec_sweeps, max_iter, prod_sweeps, float(flat), seed, start, rec_max,
                     eq_scale, prep_sweeps, rec_rule, cb, None)
        init = None
        if lnW_init is not None:
            init = np.ascontiguousarray(lnW_init, dtype=np.float64)
        lnW = np.zeros(K1)
        H = np.zeros(K1, dtype=np.int64)
        lng = np.zeros(K1)
        hist = np.zeros(max(1, max_iter))
        st = MucaStats()
        dp = lambda x: None if x is None else x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rc = _lib.mc_muca_run(self._h, ctypes.byref(a), dp(init), _ptr(spins), dp(lnW),
                              H.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), dp(lng), dp(hist), ctypes.byref(st),
                              _ptr(ws), ws.numel(), _stream(self.device))
        if rc not in (MC_OK, MC_E_NOTCONV):
            self._check(rc, "mc_muca_run")
        return dict(lnW=lnW, iterations=st.iterations, converged=bool(st.converged),
                    min_over_max=st.min_over_max, sweeps_per_walker=st.sweeps_per_walker,
                    H_prod=H if prod_sweeps > 0 else None, lng=lng if prod_sweeps > 0 else None,
                    history=list(hist[:st.iterations]), spins=spins)

    # ------------------------------------------------------- Wang-Landau windows
    @staticmethod
    def _wl_args(L, lo, hi, walkers, seed=0, check_sweeps=1, flat=0.8, lnf_final=1e-6, max_sweeps=1 << 40,
                 max_pass=1000, progress=None):
        import numpy as np

        lo = np.ascontiguousarray(lo, dtype=np.int32)
        hi = np.ascontiguousarray(hi, dtype=np.int32)
        cb = WL_PROGRESS_FN(progress) if progress is not None else WL_PROGRESS_FN()
        i32p = ctypes.POINTER(ctypes.c_int32)
        a = WlArgs(L, lo.size, lo.ctypes.data_as(i32p), hi.ctypes.data_as(i32p), walkers, check_sweeps, float(flat),
                   float(lnf_final), max_sweeps, max_pass, seed, cb, None)
        return a, (lo, hi, cb)  # the arrays and callback must outlive the call

    def wl_workspace(self, L, lo, hi, walkers):
        a, keep = self._wl_args(L, lo, hi, walkers)
        n = int(_lib.mc_wl_workspace_bytes(ctypes.byref(a)))
        if n == 0:
            raise MCError(MC_E_RANGE, "invalid windows or walkers")
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def win_drive(self, L, lo, hi, walkers, seed, max_pass=1000, ws=None):
        """Walkers driven into their windows (mc_win_drive); returns (spins
        [nwin walkers][N] int8, E int64) on the device."""
        import numpy as np

        lo = np.ascontiguousarray(lo, dtype=np.int32)
        hi = np.ascontiguousarray(hi, dtype=np.int32)
        W = lo.size * walkers
        spins = torch.empty((W, L * L), dtype=torch.int8, device=self.device)
        E = torch.empty(W, dtype=torch.int64, device=self.device)
        ws = self.wl_workspace(L, lo, hi, walkers) if ws is None else ws
        self._check(_lib.mc_win_drive(self._h, L, lo.size, lo.ctypes.data, hi.ctypes.data, walkers, seed, max_pass,
                                      _ptr(spins), _ptr(E), _ptr(ws), ws.numel(), _stream(self.device)),
                    "mc_win_drive")
        return spins, E

    def wl_sweeps(self, L, lo, hi, walkers, inc, active, seed, sweep0, nsweeps, spins, E, G, H, flags, flat=0.8,
                  ws=None):
        """nsweeps Wang-Landau sweeps (mc_wl_sweeps) in place on the device
        tensors spins, E, G [W][wmax] int64, H [W][wmax] int32 (bit-identical
        to uint32), flags [W] int32."""
        import numpy as np

        lo = np.ascontiguousarray(lo, dtype=np.int32)
        hi = np.ascontiguousarray(hi, dtype=np.int32)
        inc = np.ascontiguousarray(inc, dtype=np.int64)
        act = np.ascontiguousarray(active, dtype=np.uint8)
        ws = self.wl_workspace(L, lo, hi, walkers) if ws is None else ws
        return self._check(_lib.mc_wl_sweeps(self._h, L, lo.size, lo.ctypes.data, hi.ctypes.data, walkers,
                                             inc.ctypes.data, act.ctypes.data, float(flat), seed, sweep0, nsweeps,
                                             _ptr(spins), _ptr(E), _ptr(G), _ptr(H), _ptr(flags), _ptr(ws),
                                             ws.numel(), _stream(self.device)), "mc_wl_sweeps")

    def wl_run(self, L, lo, hi, walkers, seed, lnf_final, flat=0.8, check_sweeps=1, max_sweeps=1 << 40,
               max_pass=1000, progress=None, ws=None):
        """Wang-Landau sampling in windows (mc_wl_run); returns a dict like
        oracle.wl_run (pieces, lng, stages, sweeps, converged, spins, E)."""
        import numpy as np

        a, keep = self._wl_args(L, lo, hi, walkers, seed, check_sweeps, flat, lnf_final, max_sweeps, max_pass,
                                progress)
        lo_a, hi_a = keep[0], keep[1]
        nwin = lo_a.size
        wmax = int((hi_a - lo_a).max()) + 1
        W = nwin * walkers
        spins = torch.empty((W, L * L), dtype=torch.int8, device=self.device)
        E = torch.empty(W, dtype=torch.int64, device=self.device)
        ws = self.wl_workspace(L, lo_a, hi_a, walkers) if ws is None else ws
        pieces = np.zeros((nwin, wmax))
        lng = np.zeros(L * L // 2 + 1)
        st = (WlWindowStats * nwin)()
        dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rc = _lib.mc_wl_run(self._h, ctypes.byref(a), _ptr(spins), _ptr(E), dp(pieces), dp(lng), st, _ptr(ws),
                            ws.numel(), _stream(self.device))
        if rc not in (MC_OK, MC_E_NOTCONV):
            self._check(rc, "mc_wl_run")
        return dict(pieces=[pieces[i, :hi_a[i] - lo_a[i] + 1].copy() for i in range(nwin)], lng=lng,
                    stages=[st[i].stages for i in range(nwin)], sweeps=[st[i].sweeps for i in range(nwin)],
                    converged=[bool(st[i].converged) for i in range(nwin)], spins=spins, E=E)

    def muca_windows_run(self, L, lo, hi, walkers, seed, rec_sweeps, max_iter, flat=0.8, eq_sweeps=2,
                         max_pass=1000, progress=None, ws=None):
        """The multicanonical recursion in windows (mc_muca_windows_run);
        returns a dict like oracle.muca_windows_run."""
        import numpy as np

        lo_a = np.ascontiguousarray(lo, dtype=np.int32)
        hi_a = np.ascontiguousarray(hi, dtype=np.int32)
        cb = WL_PROGRESS_FN(progress) if progress is not None else WL_PROGRESS_FN()
        i32p = ctypes.POINTER(ctypes.c_int32)
        a = MucaWinArgs(L, lo_a.size, lo_a.ctypes.data_as(i32p), hi_a.ctypes.data_as(i32p), walkers, eq_sweeps,
                        rec_sweeps, max_iter, float(flat), max_pass, seed, cb, None)
        nwin = lo_a.size
        wmax = int((hi_a - lo_a).max()) + 1
        W = nwin * walkers
        if ws is None:
            n = int(_lib.mc_muca_windows_workspace_bytes(ctypes.byref(a)))
            if n == 0:
                raise MCError(MC_E_RANGE, "invalid windows or walkers")
            ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        spins = torch.empty((W, L * L), dtype=torch.int8, device=self.device)
        E = torch.empty(W, dtype=torch.int64, device=self.device)
        pieces = np.zeros((nwin, wmax))
        lng = np.zeros(L * L // 2 + 1)
        st = (MucaWinStats * nwin)()
        dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        rc = _lib.mc_muca_windows_run(self._h, ctypes.byref(a), _ptr(spins), _ptr(E), dp(pieces), dp(lng), st,
                                      _ptr(ws), ws.numel(), _stream(self.device))
        if rc not in (MC_OK, MC_E_NOTCONV):
            self._check(rc, "mc_muca_windows_run")
        return dict(pieces=[pieces[i, :hi_a[i] - lo_a[i] + 1].copy() for i in range(nwin)], lng=lng,
                    iterations=[st[i].iterations for i in range(nwin)],
                    converged=[bool(st[i].converged) for i in range(nwin)], spins=spins, E=E)

    def set_tile_plan(self, geom, H, K, threads):
        return self._check(_lib.mc_set_tile_plan(self._h, ctypes.byref(geom), H, K, threads), "mc_set_tile_plan")

    def get_tile_plan(self, geom):
        H, K, T = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(_lib.mc_get_tile_plan(self._h, ctypes.byref(geom), ctypes.byref(H), ctypes.byref(K),
                                          ctypes.byref(T)), "mc_get_tile_plan")
        return H.value, K.value, T.value

    def tune_sweep(self, geom, scratch_a, scratch_b, beta, sweeps=20, rule=METROPOLIS):
        self._check(_lib.mc_tune_sweep_rule(self._h, ctypes.byref(geom), rule, _ptr(scratch_a), _ptr(scratch_b),
                                            float(beta), sweeps, _stream(self.device)), "mc_tune_sweep_rule")
        return self.get_tile_plan(geom)
