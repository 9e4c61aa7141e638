"""ctypes binding of libmfr (include/mfr.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor
devices, dtypes, shapes and contiguity, passes raw device pointers and the
current HIP stream, and converts status codes into exceptions.  Device
memory (workspaces, outputs) is allocated through torch.  There is no CPU
fallback: if the library is missing, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmfr.so")

MFR_OK = 0
STATUS = {0: "MFR_OK", -1: "MFR_EINVAL", -2: "MFR_ENOMEM", -3: "MFR_EHIP", -4: "MFR_ENONFINITE",
          -5: "MFR_ELINESEARCH", -6: "MFR_EBREAKDOWN", -7: "MFR_ENOTCONV"}


class MfrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class CGrid(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3), ("my", ctypes.c_int32 * 3),
                ("mT", ctypes.c_int32 * 3), ("hT", ctypes.c_double * 3),
                ("tau", ctypes.c_double), ("rho", ctypes.c_double), ("alpha", ctypes.c_double),
                ("distance", ctypes.c_int32), ("regulariser", ctypes.c_int32),
                ("lame_mu", ctypes.c_double), ("lame_lambda", ctypes.c_double)]


class CPcgOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double), ("precond", ctypes.c_int32),
                ("fallback_iters", ctypes.c_int32), ("require_converged", ctypes.c_int32)]


class CPcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("relres", ctypes.c_double), ("flag", ctypes.c_int32),
                ("used_fallback", ctypes.c_int32)]


class CGnOpts(ctypes.Structure):
    _fields_ = [("pcg_max", ctypes.c_int32), ("pcg_rtol", ctypes.c_double), ("precond", ctypes.c_int32),
                ("armijo_c1", ctypes.c_double), ("armijo_max", ctypes.c_int32), ("fallback_iters", ctypes.c_int32)]


class CGnInfo(ctypes.Structure):
    _fields_ = [("J_before", ctypes.c_double), ("J_after", ctypes.c_double), ("eta", ctypes.c_double),
                ("slope", ctypes.c_double), ("pcg_iters", ctypes.c_int32), ("pcg_relres", ctypes.c_double),
                ("pcg_flag", ctypes.c_int32), ("accepted", ctypes.c_int32), ("ls_trials", ctypes.c_int32)]


class CMlOpts(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("gn_iters", ctypes.c_int32), ("pcg_max", ctypes.c_int32),
                ("pcg_rtol", ctypes.c_double), ("armijo_c1", ctypes.c_double), ("armijo_max", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("u_init", ctypes.c_void_p), ("pc", ctypes.c_void_p),
                ("fallback_iters", ctypes.c_int32)]


class CMlReport(ctypes.Structure):
    _fields_ = [("J_final", ctypes.c_double), ("gn_done", ctypes.c_int32 * 8), ("pcg_total", ctypes.c_int32 * 8),
                ("status", ctypes.c_int32 * 8), ("seconds", ctypes.c_double), ("J_start", ctypes.c_double * 8),
                ("J_level", ctypes.c_double * 8)]


class CProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int32 * 6), ("ms", ctypes.c_double * 6)]


class CTileConfig(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int32), ("by", ctypes.c_int32), ("chunk_len", ctypes.c_int32),
                ("target_groups", ctypes.c_int32)]


MAX_BATCH = 12


class CBatchReport(ctypes.Structure):
    _fields_ = [("J_final", ctypes.c_double * MAX_BATCH), ("gn_done", ctypes.c_int32 * MAX_BATCH),
                ("pcg_total", ctypes.c_int32 * MAX_BATCH), ("status", ctypes.c_int32 * MAX_BATCH),
                ("graph_launches", ctypes.c_int32), ("seconds", ctypes.c_double)]


PC_PARAMS = 4 * (27 * 16 * 16 + 16)


class CPcTrainOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("pcg_iters", ctypes.c_int32), ("sample_every", ctypes.c_int32)]


class CPcTrainInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("loss_mean", ctypes.c_double)]


class CLbfgsOpts(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("mem", ctypes.c_int32), ("gamma", ctypes.c_double),
                ("armijo_c1", ctypes.c_double), ("armijo_max", ctypes.c_int32)]


class CLbfgsReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("pairs_skipped", ctypes.c_int32), ("evals", ctypes.c_int32), ("J_initial", ctypes.c_double),
                ("J_final", ctypes.c_double), ("seconds", ctypes.c_double)]


PROFILE_KERNELS = ("tile_obj", "tile_grad", "tile_hv", "jacobi_diag", "node_pass", "pc_network")

_lib = None

# exported function -> (restype, argtypes)
_VP, _SZ, _D, _I = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double, ctypes.c_int32
SIGNATURES = {
    "mfr_abi_version": (ctypes.c_int, []),
    "mfr_last_error": (ctypes.c_char_p, []),
    "mfr_workspace_size": (ctypes.c_int, [ctypes.POINTER(CGrid), ctypes.POINTER(_SZ)]),
    "mfr_create": (ctypes.c_int, [ctypes.POINTER(CGrid), _VP, _VP, _SZ, ctypes.POINTER(_VP)]),
    "mfr_destroy": (None, [_VP]),
    "mfr_set_images": (ctypes.c_int, [_VP, _VP, _VP]),
    "mfr_objective": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "mfr_gradient": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_D), _VP]),
    "mfr_hess_vec": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mfr_objective_async": (ctypes.c_int, [_VP, _VP, _VP]),
    "mfr_gradient_async": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mfr_hess_vec_noalloc": (ctypes.c_int, [ctypes.POINTER(CGrid), _VP, _VP, _VP, _VP, _VP, _VP]),
    "mfr_jacobi_diag": (ctypes.c_int, [_VP, _VP, _VP]),
    "mfr_pcg_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(CPcgOpts), ctypes.POINTER(CPcgInfo)]),
    "mfr_pcg_solve_async": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.POINTER(CPcgOpts), _VP]),
    "mfr_gn_step": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(CGnOpts), ctypes.POINTER(CGnInfo)]),
    "mfr_gn_step_async": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(CGnOpts), _VP]),
    "mfr_ml_workspace_size": (ctypes.c_int, [ctypes.POINTER(CGrid), _I, ctypes.POINTER(_SZ)]),
    "mfr_register_multilevel": (ctypes.c_int, [ctypes.POINTER(CGrid), ctypes.POINTER(CMlOpts), _VP, _VP, _SZ,
                                               _VP, _VP, _VP, ctypes.POINTER(CMlReport)]),
    "mfr_ml_level_grid": (ctypes.c_int, [ctypes.POINTER(CGrid), _I, _I, ctypes.POINTER(CGrid)]),
    "mfr_restrict_image": (ctypes.c_int, [ctypes.POINTER(_I), _VP, _VP, _VP]),
    "mfr_prolong_workspace_size": (ctypes.c_int, [ctypes.POINTER(CGrid), ctypes.POINTER(_SZ)]),
    "mfr_prolong": (ctypes.c_int, [ctypes.POINTER(CGrid), ctypes.POINTER(CGrid), _VP, _VP, _VP, _SZ, _VP]),
    "mfr_batch_workspace_size": (ctypes.c_int, [_I, ctypes.POINTER(CGrid), _I, ctypes.POINTER(_SZ)]),
    "mfr_batch_create": (ctypes.c_int, [_I, ctypes.POINTER(CGrid), _I, _VP, _VP, _SZ, ctypes.POINTER(_VP)]),
    "mfr_batch_destroy": (None, [_VP]),
    "mfr_batch_set_images": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP)]),
    "mfr_batch_hess_vec": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP)]),
    "mfr_batch_register": (ctypes.c_int, [_VP, ctypes.POINTER(CMlOpts), _I, ctypes.POINTER(_VP),
                                          ctypes.POINTER(CBatchReport)]),
    "mfr_pc_workspace_size": (ctypes.c_int, [ctypes.POINTER(CGrid), _I, ctypes.POINTER(_SZ)]),
    "mfr_pc_create": (ctypes.c_int, [_VP, _I, _VP, _SZ, ctypes.POINTER(_VP)]),
    "mfr_pc_destroy": (None, [_VP]),
    "mfr_pc_bind": (ctypes.c_int, [_VP, _VP]),
    "mfr_pc_set_params": (ctypes.c_int, [_VP, _VP]),
    "mfr_pc_get_params": (ctypes.c_int, [_VP, _VP]),
    "mfr_pc_apply": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "mfr_pc_train_system": (ctypes.c_int, [_VP, _VP, _VP, ctypes.POINTER(CPcTrainOpts), ctypes.POINTER(CPcTrainInfo)]),
    "mfr_attach_pc": (ctypes.c_int, [_VP, _VP]),
    "mfr_cnn_conv": (ctypes.c_int, [_I, _I, _I, _VP, _VP, _VP, _I, _VP, _VP, _VP]),
    "mfr_cnn_conv_bwd_data": (ctypes.c_int, [_I, _I, _I, _VP, _VP, _VP, _VP, _VP, _VP]),
    "mfr_cnn_wgrad_workspace_size": (ctypes.c_int, [_I, _I, _I, ctypes.POINTER(_SZ)]),
    "mfr_cnn_conv_bwd_weight": (ctypes.c_int, [_I, _I, _I, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "mfr_set_tile_config": (ctypes.c_int, [ctypes.POINTER(CTileConfig)]),
    "mfr_get_tile_config": (ctypes.c_int, [ctypes.POINTER(CTileConfig)]),
    "mfr_profile_enable": (ctypes.c_int, [_VP, _I]),
    "mfr_profile_read": (ctypes.c_int, [_VP, ctypes.POINTER(CProfile), _I]),
    "mfr_lbfgs_workspace_size": (ctypes.c_int, [ctypes.POINTER(CGrid), _I, ctypes.POINTER(_SZ)]),
    "mfr_h0_solve": (ctypes.c_int, [_VP, _D, _VP, _VP, _VP, _SZ]),
    "mfr_lbfgs": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(CLbfgsOpts), _VP, _SZ, ctypes.POINTER(CLbfgsReport)]),
}


def load():
    """Load libmfr.so and bind every exported entry point (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libmfr.so not found at {LIB_PATH}; build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != MFR_OK:
        raise MfrError(status, _lib.mfr_last_error().decode())


DISTANCES = {"ngf": 0, "ssd": 1}   # mfr_grid.distance
REGULARISERS = {"curvature": 0, "diffusive": 1, "elastic": 2}   # mfr_grid.regulariser


def is_plane(m, my):
    """A two-dimensional problem: one image cell and one node along z."""
    return int(m[2]) == 1 and int(my[2]) == 1


def node_shape_of(m, my):
    """Shape of a node vector: (3, n_z, n_y, n_x), or (2, n_y, n_x) in 2D."""
    if is_plane(m, my):
        return (2, int(my[1]), int(my[0]))
    return (3, int(my[2]), int(my[1]), int(my[0]))


def node_count(m, my):
    return int(np.prod(node_shape_of(m, my)))


def make_grid(spec):
    """CGrid from any object with m, h, my, tau, rho, alpha (optional mT, hT,
    distance "ngf" or "ssd", regulariser "curvature", "diffusive" or "elastic" with
    lame_mu, lame_lambda)."""
    g = CGrid()
    for k in range(3):
        g.m[k] = int(spec.m[k])
        g.h[k] = float(spec.h[k])
        g.my[k] = int(spec.my[k])
        mT = getattr(spec, "mT", None)
        hT = getattr(spec, "hT", None)
        g.mT[k] = int(mT[k]) if mT is not None else 0
        g.hT[k] = float(hT[k]) if hT is not None else 0.0
    g.tau, g.rho, g.alpha = float(spec.tau), float(spec.rho), float(spec.alpha)
    dist = getattr(spec, "distance", "ngf")
    if dist not in DISTANCES:
        raise ValueError(f"distance must be one of {sorted(DISTANCES)}, got {dist!r}")
    g.distance = DISTANCES[dist]
    reg = getattr(spec, "regulariser", "curvature")
    if reg not in REGULARISERS:
        raise ValueError(f"regulariser must be one of {sorted(REGULARISERS)}, got {reg!r}")
    g.regulariser = REGULARISERS[reg]
    g.lame_mu = float(getattr(spec, "lame_mu", 1.0))
    g.lame_lambda = float(getattr(spec, "lame_lambda", 0.0))
    return g


def _dev_tensor(x, numel, name, device):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.device.type != "cuda" or (device is not None and x.device != device):
        raise ValueError(f"{name} must live on {device}")
    if x.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if x.numel() != numel:
        raise ValueError(f"{name} has {x.numel()} elements, expected {numel}")
    return ctypes.c_void_p(x.data_ptr())


def _f64_tensor(x, numel, name, device):
    """A contiguous float64 device tensor of numel elements (scalars the device writes)."""
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 torch tensor")
    if x.device != device or not x.is_contiguous() or x.numel() != numel:
        raise ValueError(f"{name}: expected a contiguous tensor of {numel} elements on {device}")
    return ctypes.c_void_p(x.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_size(spec):
    lib = load()
    g = make_grid(spec)
    n = ctypes.c_size_t()
    _check(lib.mfr_workspace_size(ctypes.byref(g), ctypes.byref(n)))
    return n.value


def hess_vec_noalloc(spec, R, T, u, p, out):
    """q = (H + alpha nabla^2 S) p through mfr_hess_vec_noalloc: no context, no
    workspace; the library's fixed scratch array of the current device serves
    as workspace.  Every tensor is caller-provided (out included)."""
    lib = load()
    g = make_grid(spec)
    m, my = tuple(int(k) for k in spec.m), tuple(int(k) for k in spec.my)
    mT = getattr(spec, "mT", None)
    mT = tuple(int(k) for k in (mT if mT is not None else m))
    dev = u.device
    nv = node_count(m, my)
    args = (_dev_tensor(R, m[0] * m[1] * m[2], "R", dev), _dev_tensor(T, mT[0] * mT[1] * mT[2], "T", dev),
            _dev_tensor(u, nv, "u", dev), _dev_tensor(p, nv, "p", dev), _dev_tensor(out, nv, "q", dev))
    _check(lib.mfr_hess_vec_noalloc(ctypes.byref(g), _stream(dev), *args))
    return out


def _alloc_workspace(nbytes, device):
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws, ws.data_ptr() + off


class Context:
    """One registration problem bound to a device, a stream and a workspace."""

    def __init__(self, spec, device="cuda:0"):
        self.lib = load()
        self.device = torch.device(device)
        self.spec = spec
        self.grid = make_grid(spec)
        self.m = tuple(int(k) for k in spec.m)
        self.my = tuple(int(k) for k in spec.my)
        mT = getattr(spec, "mT", None)
        self.mT = tuple(int(k) for k in (mT if mT is not None else spec.m))
        self.nbar = self.my[0] * self.my[1] * self.my[2]
        self.mbar = self.m[0] * self.m[1] * self.m[2]
        self.nc = 2 if is_plane(self.m, self.my) else 3   # node vector components
        self.ws_bytes = workspace_size(spec)
        self._ws, ptr = _alloc_workspace(self.ws_bytes, self.device)
        h = ctypes.c_void_p()
        _check(self.lib.mfr_create(ctypes.byref(self.grid), _stream(self.device), ctypes.c_void_p(ptr),
                                   self.ws_bytes, ctypes.byref(h)))
        self._h = h
        self._images = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.mfr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_shape(self):
        return node_shape_of(self.m, self.my)

    def set_images(self, R, T):
        r = _dev_tensor(R, self.mbar, "R", self.device)
        t = _dev_tensor(T, self.mT[0] * self.mT[1] * self.mT[2], "T", self.device)
        _check(self.lib.mfr_set_images(self._h, r, t))
        self._images = (R, T)   # keep the borrowed buffers alive

    def objective(self, u):
        J, D, S = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self.lib.mfr_objective(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                      ctypes.byref(J), ctypes.byref(D), ctypes.byref(S)))
        return J.value, D.value, S.value

    def gradient(self, u, out=None, want_J=True):
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        J = ctypes.c_double()
        _check(self.lib.mfr_gradient(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                     ctypes.byref(J) if want_J else None,
                                     _dev_tensor(out, self.nc * self.nbar, "g", self.device)))
        return out, (J.value if want_J else None)

    def objective_async(self, u, out=None):
        """(J, D, S) written by the device into `out` (float64 [3] on the device);
        no synchronisation, so the call can be captured in a HIP graph."""
        out = torch.empty(3, dtype=torch.float64, device=self.device) if out is None else out
        _check(self.lib.mfr_objective_async(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                            _f64_tensor(out, 3, "out", self.device)))
        return out

    def gradient_async(self, u, out=None, J=None):
        """The gradient into `out` and, if `J` (float64 [1] on the device) is
        given, J(u) written by the device there; no synchronisation."""
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        _check(self.lib.mfr_gradient_async(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                           None if J is None else _f64_tensor(J, 1, "J", self.device),
                                           _dev_tensor(out, self.nc * self.nbar, "g", self.device)))
        return out

    def hess_vec(self, u, p, out=None):
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        _check(self.lib.mfr_hess_vec(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                     _dev_tensor(p, self.nc * self.nbar, "p", self.device),
                                     _dev_tensor(out, self.nc * self.nbar, "q", self.device)))
        return out

    def jacobi_diag(self, u, out=None):
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        _check(self.lib.mfr_jacobi_diag(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                        _dev_tensor(out, self.nc * self.nbar, "diag", self.device)))
        return out

    def _lbfgs_work(self, mem):
        n = ctypes.c_size_t()
        _check(self.lib.mfr_lbfgs_workspace_size(ctypes.byref(self.grid), int(mem), ctypes.byref(n)))
        cache = getattr(self, "_lb_work", None)
        if cache is None or cache[2] < n.value:
            buf, ptr = _alloc_workspace(n.value, self.device)
            self._lb_work = (buf, ptr, n.value)
        return self._lb_work[1], self._lb_work[2]

    def h0_solve(self, v, gamma, out=None):
        """x = (alpha nabla^2 S + gamma I)^{-1} v, the L-BFGS initial matrix solve."""
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        ptr, nbytes = self._lbfgs_work(1)
        _check(self.lib.mfr_h0_solve(self._h, float(gamma), _dev_tensor(v, self.nc * self.nbar, "v", self.device),
                                     _dev_tensor(out, self.nc * self.nbar, "x", self.device), ctypes.c_void_p(ptr),
                                     nbytes))
        return out

    def lbfgs(self, u, iters=10, mem=5, gamma=1.0, armijo_c1=1e-4, armijo_max=10):
        """L-BFGS iterations; u (device, float32) is updated in place.  Returns the report."""
        ptr, nbytes = self._lbfgs_work(mem)
        opts = CLbfgsOpts(int(iters), int(mem), float(gamma), float(armijo_c1), int(armijo_max))
        rep = CLbfgsReport()
        _check(self.lib.mfr_lbfgs(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device), ctypes.byref(opts),
                                  ctypes.c_void_p(ptr), nbytes, ctypes.byref(rep)))
        return {f[0]: getattr(rep, f[0]) for f in CLbfgsReport._fields_}

    def gn_step(self, u, pcg_max=50, pcg_rtol=1e-3, precond=1, armijo_c1=1e-4, armijo_max=10, fallback_iters=0):
        """One Gauss-Newton step; u (device, float32) is updated in place."""
        opts = CGnOpts(int(pcg_max), float(pcg_rtol), int(precond), float(armijo_c1), int(armijo_max),
                       int(fallback_iters))
        info = CGnInfo()
        _check(self.lib.mfr_gn_step(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device), ctypes.byref(opts),
                                    ctypes.byref(info)))
        return {f[0]: getattr(info, f[0]) for f in CGnInfo._fields_}

    def gn_step_async(self, u, pcg_max=50, pcg_rtol=1e-3, precond=1, armijo_c1=1e-4, armijo_max=10, info=None):
        """One Gauss-Newton step as a fixed launch sequence (capturable in a HIP
        graph): u updated in place on the device; the fields of gn_step's result
        written by the device into `info` (float64 [9] on the device)."""
        info = torch.empty(9, dtype=torch.float64, device=self.device) if info is None else info
        opts = CGnOpts(int(pcg_max), float(pcg_rtol), int(precond), float(armijo_c1), int(armijo_max), 0)
        _check(self.lib.mfr_gn_step_async(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                          ctypes.byref(opts), _f64_tensor(info, 9, "info", self.device)))
        return info

    def profile(self, enable=True):
        """Turn kernel timing (HIP events on this context's stream) on or off."""
        _check(self.lib.mfr_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self, reset=True):
        """{kernel: (launches, total ms)} accumulated since the last reset."""
        st = CProfile()
        _check(self.lib.mfr_profile_read(self._h, ctypes.byref(st), 1 if reset else 0))
        return {k: (st.launches[i], st.ms[i]) for i, k in enumerate(PROFILE_KERNELS)}

    def pcg_solve(self, u, b, max_iter=50, rtol=1e-3, precond=1, fallback_iters=0, out=None,
                  require_converged=False):
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        opts = CPcgOpts(int(max_iter), float(rtol), int(precond), int(fallback_iters), 1 if require_converged else 0)
        info = CPcgInfo()
        _check(self.lib.mfr_pcg_solve(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                      _dev_tensor(b, self.nc * self.nbar, "b", self.device),
                                      _dev_tensor(out, self.nc * self.nbar, "s", self.device),
                                      ctypes.byref(opts), ctypes.byref(info)))
        return out, dict(iters=info.iters, relres=info.relres, flag=info.flag, used_fallback=info.used_fallback)

    def pcg_solve_async(self, u, b, max_iter=50, rtol=1e-3, precond=1, out=None, info=None):
        """The solve as one fixed launch sequence (capturable in a HIP graph): s into
        `out`, (iterations, relative residual, flag) written by the device into
        `info` (float64 [3] on the device); no synchronisation."""
        out = torch.empty(self.node_shape(), dtype=torch.float32, device=self.device) if out is None else out
        info = torch.empty(3, dtype=torch.float64, device=self.device) if info is None else info
        opts = CPcgOpts(int(max_iter), float(rtol), int(precond), 0, 0)
        _check(self.lib.mfr_pcg_solve_async(self._h, _dev_tensor(u, self.nc * self.nbar, "u", self.device),
                                            _dev_tensor(b, self.nc * self.nbar, "b", self.device),
                                            _dev_tensor(out, self.nc * self.nbar, "s", self.device),
                                            ctypes.byref(opts), _f64_tensor(info, 3, "info", self.device)))
        return out, info

    def attach_pc(self, pc):
        """Use a LearnedPC of this context for precond = 2 (None detaches)."""
        _check(self.lib.mfr_attach_pc(self._h, None if pc is None else pc._h))
        self._pc = pc


def ml_level_grid(spec, levels, level):
    """CGrid of pyramid level ``level`` (0 = coarsest) of a ``levels``-level registration."""
    lib = load()
    g = make_grid(spec)
    out = CGrid()
    _check(lib.mfr_ml_level_grid(ctypes.byref(g), int(levels), int(level), ctypes.byref(out)))
    return out


def register_multilevel(spec, R, T, levels=3, gn_iters=10, pcg_max=50, pcg_rtol=1e-3, armijo_c1=1e-4,
                        armijo_max=10, precond=1, u0=None, device="cuda:0", pc=None, fallback_iters=0):
    """Coarse-to-fine Gauss-Newton registration; returns (u_finest, report dict).
    ``u0``: initial displacement on the COARSEST deformation grid (None: 0).
    ``pc`` (precond 2): a LearnedPC whose workspace fits the finest grid; the
    library binds it to each level in turn and leaves it unbound (``pc.bind``
    before its next use)."""
    lib = load()
    device = torch.device(device)
    g = make_grid(spec)
    n = ctypes.c_size_t()
    _check(lib.mfr_ml_workspace_size(ctypes.byref(g), int(levels), ctypes.byref(n)))
    ws, ptr = _alloc_workspace(n.value, device)
    my = tuple(int(k) for k in spec.my)
    nv = node_count(spec.m, my)
    u = torch.empty(node_shape_of(spec.m, my), dtype=torch.float32, device=device)
    mbar = int(spec.m[0]) * int(spec.m[1]) * int(spec.m[2])
    mT = getattr(spec, "mT", None) or spec.m
    init = None
    if u0 is not None:
        gc = ml_level_grid(spec, levels, 0)
        init = _dev_tensor(u0, node_count(gc.m, gc.my), "u0", device)
    if int(precond) == 2 and pc is None:
        raise ValueError("precond 2 needs a LearnedPC (pc=...)")
    opts = CMlOpts(int(levels), int(gn_iters), int(pcg_max), float(pcg_rtol), float(armijo_c1), int(armijo_max),
                   int(precond), init, None if pc is None else pc._h, int(fallback_iters))
    if pc is not None and int(precond) == 2:
        pc._unbind()   # the library moves it through the levels' contexts
    rep = CMlReport()
    _check(lib.mfr_register_multilevel(ctypes.byref(g), ctypes.byref(opts), _stream(device), ctypes.c_void_p(ptr),
                                       n.value, _dev_tensor(R, mbar, "R", device),
                                       _dev_tensor(T, int(mT[0]) * int(mT[1]) * int(mT[2]), "T", device),
                                       _dev_tensor(u, nv, "u", device), ctypes.byref(rep)))
    del ws
    return u, dict(J_final=rep.J_final, gn_done=list(rep.gn_done)[:levels], pcg_total=list(rep.pcg_total)[:levels],
                   status=list(rep.status)[:levels], seconds=rep.seconds, J_start=list(rep.J_start)[:levels],
                   J_level=list(rep.J_level)[:levels])


def restrict_image(img):
    """One pyramid level of a device float32 image [m_z, m_y, m_x] (2x2x2 means)."""
    lib = load()
    if img.dim() != 3:
        raise ValueError("image must be 3-D [m_z, m_y, m_x]")
    mz, my_, mx = (int(k) for k in img.shape)
    m = (ctypes.c_int32 * 3)(mx, my_, mz)
    out = torch.empty(((mz + 1) // 2, (my_ + 1) // 2, (mx + 1) // 2), dtype=torch.float32, device=img.device)
    _check(lib.mfr_restrict_image(m, _dev_tensor(img, mx * my_ * mz, "fine", img.device),
                                  _dev_tensor(out, out.numel(), "coarse", img.device), _stream(img.device)))
    return out


def prolong(uc, coarse_spec, fine_spec):
    """Displacement on the coarse deformation grid -> fine grid (linear, per dimension).
    The specs may be grid specs or CGrid structures."""
    lib = load()
    gc = coarse_spec if isinstance(coarse_spec, CGrid) else make_grid(coarse_spec)
    gf = fine_spec if isinstance(fine_spec, CGrid) else make_grid(fine_spec)
    dev = uc.device
    n = ctypes.c_size_t()
    _check(lib.mfr_prolong_workspace_size(ctypes.byref(gf), ctypes.byref(n)))
    work, ptr = _alloc_workspace(n.value, dev)
    out = torch.empty(node_shape_of(gf.m, gf.my), dtype=torch.float32, device=dev)
    _check(lib.mfr_prolong(ctypes.byref(gc), ctypes.byref(gf),
                           _dev_tensor(uc, node_count(gc.m, gc.my), "uc", dev),
                           _dev_tensor(out, out.numel(), "uf", dev), ctypes.c_void_p(ptr), n.value, _stream(dev)))
    del work
    return out


def set_tile_config(bx, by, chunk_len=0, target_groups=0):
    """Tile shape (bx x by threads), z planes per work-group (0: derived) and
    the work-group count the derived split aims for (0: library default), for
    contexts and batches created afterwards in this process."""
    lib = load()
    c = CTileConfig(int(bx), int(by), int(chunk_len), int(target_groups))
    _check(lib.mfr_set_tile_config(ctypes.byref(c)))


def get_tile_config():
    lib = load()
    c = CTileConfig()
    _check(lib.mfr_get_tile_config(ctypes.byref(c)))
    return dict(bx=c.bx, by=c.by, chunk_len=c.chunk_len, target_groups=c.target_groups)


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))()
    for i, p in enumerate(ptrs):
        arr[i] = p.value if isinstance(p, ctypes.c_void_p) else p
    return arr


class Batch:
    """Independent registration problems (up to MAX_BATCH, sizes may differ)
    advanced together by the batched library path on a stream of its own."""

    def __init__(self, specs, levels=1, device="cuda:0"):
        self.lib = load()
        self.device = torch.device(device)
        self.specs = list(specs)
        self.n = len(self.specs)
        if not 1 <= self.n <= MAX_BATCH:
            raise ValueError(f"batch size must be in 1..{MAX_BATCH}")
        self.levels = int(levels)
        self.grids = (CGrid * self.n)(*[make_grid(s) for s in self.specs])
        self.my = [tuple(int(k) for k in s.my) for s in self.specs]
        self.m = [tuple(int(k) for k in s.m) for s in self.specs]
        self.mT = [tuple(int(k) for k in (getattr(s, "mT", None) or s.m)) for s in self.specs]
        nbytes = ctypes.c_size_t()
        _check(self.lib.mfr_batch_workspace_size(self.n, self.grids, self.levels, ctypes.byref(nbytes)))
        self.ws_bytes = nbytes.value
        self._ws, ptr = _alloc_workspace(self.ws_bytes, self.device)
        self.stream = torch.cuda.Stream(self.device)   # default priority; graphs need a non-null stream
        h = ctypes.c_void_p()
        _check(self.lib.mfr_batch_create(self.n, self.grids, self.levels, ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.c_void_p(ptr), self.ws_bytes, ctypes.byref(h)))
        self._h = h
        self._images = None

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.stream.synchronize()
            self.lib.mfr_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def node_shape(self, k):
        my = self.my[k]
        return (3, my[2], my[1], my[0])

    def _nodes(self, k):
        my = self.my[k]
        return 3 * my[0] * my[1] * my[2]

    def _enter(self):
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def _leave(self):
        torch.cuda.current_stream(self.device).wait_stream(self.stream)

    def set_images(self, Rs, Ts):
        if len(Rs) != self.n or len(Ts) != self.n:
            raise ValueError("one reference and one template image per pair")
        r = [_dev_tensor(Rs[k], self.m[k][0] * self.m[k][1] * self.m[k][2], f"R[{k}]", self.device)
             for k in range(self.n)]
        t = [_dev_tensor(Ts[k], self.mT[k][0] * self.mT[k][1] * self.mT[k][2], f"T[{k}]", self.device)
             for k in range(self.n)]
        self._enter()
        _check(self.lib.mfr_batch_set_images(self._h, _ptr_array(r), _ptr_array(t)))
        self._leave()
        self._images = (list(Rs), list(Ts))

    def hess_vec(self, us, ps, outs=None):
        """q_k = H_k p_k at u_k on the finest grids, all pairs in one pass."""
        if outs is None:
            outs = [torch.empty(self.node_shape(k), dtype=torch.float32, device=self.device) for k in range(self.n)]
        u = [_dev_tensor(us[k], self._nodes(k), f"u[{k}]", self.device) for k in range(self.n)]
        p = [_dev_tensor(ps[k], self._nodes(k), f"p[{k}]", self.device) for k in range(self.n)]
        q = [_dev_tensor(outs[k], self._nodes(k), f"q[{k}]", self.device) for k in range(self.n)]
        self._enter()
        _check(self.lib.mfr_batch_hess_vec(self._h, _ptr_array(u), _ptr_array(p), _ptr_array(q)))
        self._leave()
        return outs

    def register(self, gn_iters=10, pcg_max=50, pcg_rtol=1e-3, armijo_c1=1e-4, armijo_max=10, precond=1,
                 use_graph=True, u0=None):
        """Coarse-to-fine Gauss-Newton registration of every pair; returns
        (list of finest displacements, report dict)."""
        us = [torch.zeros(self.node_shape(k), dtype=torch.float32, device=self.device) if u0 is None
              else u0[k].clone() for k in range(self.n)]
        ptr = [_dev_tensor(us[k], self._nodes(k), f"u[{k}]", self.device) for k in range(self.n)]
        opts = CMlOpts(self.levels, int(gn_iters), int(pcg_max), float(pcg_rtol), float(armijo_c1),
                       int(armijo_max), int(precond))
        rep = CBatchReport()
        self._enter()
        _check(self.lib.mfr_batch_register(self._h, ctypes.byref(opts), 1 if use_graph else 0, _ptr_array(ptr),
                                           ctypes.byref(rep)))
        self._leave()
        n = self.n
        return us, dict(J_final=list(rep.J_final)[:n], gn_done=list(rep.gn_done)[:n],
                        pcg_total=list(rep.pcg_total)[:n], status=list(rep.status)[:n],
                        graph_launches=rep.graph_launches, seconds=rep.seconds)


class LearnedPC:
    """The learned preconditioner of one context (see include/mfr.h)."""

    def __init__(self, ctx, train=False, capacity=()):
        """capacity: further grid specs the preconditioner may later be bound to
        (the workspace is sized for the largest)."""
        self.lib = load()
        self.ctx = ctx
        self.train = bool(train)
        sizes = []
        for g in [ctx.grid] + [make_grid(sp) for sp in capacity]:
            n = ctypes.c_size_t()
            _check(self.lib.mfr_pc_workspace_size(ctypes.byref(g), 1 if train else 0, ctypes.byref(n)))
            sizes.append(n.value)
        self.ws_bytes = max(sizes)
        self._ws, ptr = _alloc_workspace(self.ws_bytes, ctx.device)
        h = ctypes.c_void_p()
        _check(self.lib.mfr_pc_create(ctx._h, 1 if train else 0, ctypes.c_void_p(ptr), self.ws_bytes,
                                      ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            if getattr(self.ctx, "_pc", None) is self:
                self.ctx.attach_pc(None)
            self.lib.mfr_pc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bind(self, ctx):
        """Move to another context (parameters and optimiser state are kept)."""
        if self.ctx is not None and getattr(self.ctx, "_pc", None) is self:
            self.ctx.attach_pc(None)
        _check(self.lib.mfr_pc_bind(self._h, ctx._h))
        self.ctx = ctx

    def _bound_ctx(self):
        if self.ctx is None:
            raise MfrError(-1, "the preconditioner is not bound to a context; call bind(ctx) first")
        return self.ctx

    def _unbind(self):
        # the library takes the preconditioner off its context (multilevel runs)
        if self.ctx is not None and getattr(self.ctx, "_pc", None) is self:
            self.ctx._pc = None
        self.ctx = None

    def set_params(self, params):
        import numpy as np

        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        if a.size != PC_PARAMS:
            raise ValueError(f"expected {PC_PARAMS} parameters, got {a.size}")
        _check(self.lib.mfr_pc_set_params(self._h, a.ctypes.data_as(ctypes.c_void_p)))

    def get_params(self):
        import numpy as np

        a = np.empty(PC_PARAMS, dtype=np.float32)
        _check(self.lib.mfr_pc_get_params(self._h, a.ctypes.data_as(ctypes.c_void_p)))
        return a

    def apply(self, u, r, out=None):
        c = self._bound_ctx()
        out = torch.empty(c.node_shape(), dtype=torch.float32, device=c.device) if out is None else out
        _check(self.lib.mfr_pc_apply(self._h, _dev_tensor(u, 3 * c.nbar, "u", c.device),
                                     _dev_tensor(r, 3 * c.nbar, "r", c.device),
                                     _dev_tensor(out, 3 * c.nbar, "z", c.device)))
        return out

    def train_system(self, u, b, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, pcg_iters=20, sample_every=4):
        c = self._bound_ctx()
        opts = CPcTrainOpts(float(lr), float(beta1), float(beta2), float(eps), int(pcg_iters), int(sample_every))
        info = CPcTrainInfo()
        _check(self.lib.mfr_pc_train_system(self._h, _dev_tensor(u, 3 * c.nbar, "u", c.device),
                                            _dev_tensor(b, 3 * c.nbar, "b", c.device), ctypes.byref(opts),
                                            ctypes.byref(info)))
        return {f[0]: getattr(info, f[0]) for f in CPcTrainInfo._fields_}


def _bf16_tensor(x, numel, name, device):
    if not isinstance(x, torch.Tensor) or x.dtype not in (torch.bfloat16, torch.int16):
        raise TypeError(f"{name} must be a bfloat16 tensor")
    if x.device != device or not x.is_contiguous() or x.numel() != numel:
        raise ValueError(f"{name}: expected a contiguous tensor of {numel} elements on {device}")
    return ctypes.c_void_p(x.data_ptr())


def cnn_conv(x, w, bias=None, relu=False, out32=True, out16=False):
    """One 3x3x3 convolution on the device: x [nz, ny, nx, 16] bf16, w [27, 16, 16]
    bf16, bias [16] float32.  Returns (y32 or None, y16 or None)."""
    lib = load()
    nz, ny, nx = (int(k) for k in x.shape[:3])
    dev = x.device
    n = nx * ny * nz
    y32 = torch.empty((nz, ny, nx, 16), dtype=torch.float32, device=dev) if out32 else None
    y16 = torch.empty((nz, ny, nx, 16), dtype=torch.bfloat16, device=dev) if out16 else None
    b = None if bias is None else _dev_tensor(bias, 16, "bias", dev)
    _check(lib.mfr_cnn_conv(nx, ny, nz, _bf16_tensor(x, 16 * n, "x", dev), _bf16_tensor(w, 27 * 256, "w", dev), b,
                            1 if relu else 0, None if y32 is None else _dev_tensor(y32, 16 * n, "y32", dev),
                            None if y16 is None else ctypes.c_void_p(y16.data_ptr()), _stream(dev)))
    return y32, y16


def cnn_conv_bwd_data(g, w, mask=None, out32=True, out16=False):
    """Gradient with respect to the input of a convolution, zeroed where mask <= 0."""
    lib = load()
    nz, ny, nx = (int(k) for k in g.shape[:3])
    dev = g.device
    n = nx * ny * nz
    d32 = torch.empty((nz, ny, nx, 16), dtype=torch.float32, device=dev) if out32 else None
    d16 = torch.empty((nz, ny, nx, 16), dtype=torch.bfloat16, device=dev) if out16 else None
    m = None if mask is None else _bf16_tensor(mask, 16 * n, "mask", dev)
    _check(lib.mfr_cnn_conv_bwd_data(nx, ny, nz, _bf16_tensor(g, 16 * n, "g", dev), _bf16_tensor(w, 27 * 256, "w", dev),
                                     m, None if d32 is None else _dev_tensor(d32, 16 * n, "dx32", dev),
                                     None if d16 is None else ctypes.c_void_p(d16.data_ptr()), _stream(dev)))
    return d32, d16


def cnn_conv_bwd_weight(x, g):
    """(dW [27, 16, 16], db [16]) float32 of sum(g * conv(x))."""
    lib = load()
    nz, ny, nx = (int(k) for k in x.shape[:3])
    dev = x.device
    n = nx * ny * nz
    nb = ctypes.c_size_t()
    _check(lib.mfr_cnn_wgrad_workspace_size(nx, ny, nz, ctypes.byref(nb)))
    ws = torch.empty(max(nb.value // 4, 1), dtype=torch.float32, device=dev)
    out = torch.empty(27 * 256 + 16, dtype=torch.float32, device=dev)
    _check(lib.mfr_cnn_conv_bwd_weight(nx, ny, nz, _bf16_tensor(x, 16 * n, "x", dev), _bf16_tensor(g, 16 * n, "g", dev),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nb.value,
                                       _stream(dev)))
    torch.cuda.current_stream(dev).synchronize()
    return out[:27 * 256].view(27, 16, 16), out[27 * 256:]
