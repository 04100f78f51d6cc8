"""ctypes binding of libfvim.so (argument marshalling only).

Every function below checks the torch tensors it is given (device, dtype,
contiguity, shape) and forwards raw device pointers to the C ABI declared in
``include/fvim.h``; all arithmetic happens in the HIP kernels.  There is no
fallback: if the library is missing or the tensors are not on a HIP device,
the call raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfvim.so")

FVIM_OK, FVIM_EINVAL, FVIM_ENOMEM, FVIM_EHIP, FVIM_ENOCONV, FVIM_ENODEV = 0, -1, -2, -3, -4, -5
PRECISION = {"fp64": 0, "fp32_refined": 1}
K0 = {"include": 0, "exclude": 1}


class FvimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fvim error %d: %s" % (code, msg))
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double)]


class _Material(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("nu", ctypes.c_double),
                ("sigma_y0", ctypes.c_double), ("E_h", ctypes.c_double)]


class _ContactInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_change", ctypes.c_double),
                ("kkt_residual", ctypes.c_double), ("contact_fraction", ctypes.c_double),
                ("mean_gap", ctypes.c_double)]


class _TangentialInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_change", ctypes.c_double),
                ("stick_fraction", ctypes.c_double), ("shift", ctypes.c_double * 2)]


class _FrictionalInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("contact_iters", ctypes.c_int), ("tangential_iters", ctypes.c_int),
                ("rel_change", ctypes.c_double), ("kkt_residual", ctypes.c_double),
                ("stick_fraction", ctypes.c_double), ("shift", ctypes.c_double * 2)]


class _AdhesiveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("contact_iters", ctypes.c_int), ("cohesive_fraction", ctypes.c_double),
                ("contact_fraction", ctypes.c_double), ("adhesive_force", ctypes.c_double),
                ("kkt_residual", ctypes.c_double)]


class _State(ctypes.Structure):
    _fields_ = [("eps_p", ctypes.c_void_p), ("ep", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("traction", ctypes.c_void_p), ("u3p", ctypes.c_void_p)]


class EPOptions(ctypes.Structure):
    _fields_ = [("tol_outer", ctypes.c_double), ("relax", ctypes.c_double),
                ("tol_plastic", ctypes.c_double), ("tol_contact", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("max_plastic", ctypes.c_int),
                ("max_contact", ctypes.c_int), ("solver", ctypes.c_int),
                ("literal_alg1", ctypes.c_int), ("anderson_m", ctypes.c_int),
                ("warm_start", ctypes.c_int), ("inner_rel", ctypes.c_double),
                ("krylov_dim", ctypes.c_int), ("mu_f", ctypes.c_double),
                ("q_ratio", ctypes.c_double * 2), ("coupling", ctypes.c_int), ("coupling_krylov", ctypes.c_int),
                ("cerruti", ctypes.c_int), ("adh_sigma0", ctypes.c_double), ("adh_h0", ctypes.c_double)]

    def __init__(self, tol_outer=1e-9, relax=0.3, tol_plastic=1e-12, tol_contact=1e-14,
                 max_outer=400, max_plastic=2000, max_contact=20000, solver=0, literal_alg1=0,
                 anderson_m=0, warm_start=0, inner_rel=0.0, krylov_dim=0, mu_f=0.0, q_ratio=(0.0, 0.0),
                 coupling=0, coupling_krylov=0, cerruti=0, adhesion=None):
        super().__init__(tol_outer, relax, tol_plastic, tol_contact, max_outer, max_plastic,
                         max_contact, solver, literal_alg1, anderson_m, warm_start, inner_rel,
                         krylov_dim, mu_f, (ctypes.c_double * 2)(*q_ratio), coupling, coupling_krylov,
                         cerruti, *(adhesion if adhesion is not None else (0.0, 0.0)))


class _EPInfo(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("plastic_iters", ctypes.c_int),
                ("contact_iters", ctypes.c_int), ("r_evals", ctypes.c_int),
                ("outer_err", ctypes.c_double), ("plastic_res", ctypes.c_double),
                ("kkt", ctypes.c_double), ("committed", ctypes.c_int)]


MAX_STEPS = 16


class _Request(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("mat", _Material), ("precision", ctypes.c_int),
                ("n_steps", ctypes.c_int), ("W_steps", ctypes.c_double * MAX_STEPS),
                ("opts", EPOptions), ("h", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("info", _EPInfo), ("contact_fraction", ctypes.c_double),
                ("p", ctypes.c_void_p), ("u3p", ctypes.c_void_p), ("error", ctypes.c_char * 160)]


class _ServerStats(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int), ("running", ctypes.c_int), ("completed", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("budget", ctypes.c_size_t)]


_LIB = None
_P = ctypes.c_void_p


def load_library(path=None):
    """Load libfvim.so once and declare the signatures."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise FvimError(FVIM_ENODEV, "%s is not built; run python -m paper_1811_11558_amd.build" % path)
    lib = ctypes.CDLL(path)
    lib.fvim_create.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Material), ctypes.c_int,
                                ctypes.c_int, _P, ctypes.POINTER(_P)]
    lib.fvim_destroy.argtypes = [_P]
    lib.fvim_destroy.restype = None
    lib.fvim_set_stream.argtypes = [_P, _P]
    lib.fvim_set_depth_nodes.argtypes = [_P, _P]
    lib.fvim_footprint_bytes.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int, ctypes.c_int]
    lib.fvim_footprint_bytes.restype = ctypes.c_size_t
    lib.fvim_last_error.restype = ctypes.c_char_p
    lib.fvim_version.restype = ctypes.c_char_p
    lib.fvim_set_timing.argtypes = [_P, ctypes.c_int]
    lib.fvim_set_option.argtypes = [_P, ctypes.c_int, ctypes.c_int]
    lib.fvim_get_option.argtypes = [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.fvim_stage_times.argtypes = [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.mindlin_apply.argtypes = [_P, _P, _P, _P, _P, _P]
    lib.boussinesq_apply.argtypes = [_P, _P, _P, _P, _P, _P]
    lib.fvim_operator_apply.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    lib.fvim_operator_apply_noalloc.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    lib.fvim_operator_apply_batch.argtypes = [_P, ctypes.c_int, _P, _P, _P, _P, _P, _P]
    lib.return_map.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    lib.contact_solve.argtypes = [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, _P,
                                  ctypes.POINTER(_ContactInfo)]
    lib.tangential_solve.argtypes = [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, _P, ctypes.POINTER(_TangentialInfo)]
    lib.frictional_contact_solve.argtypes = [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, _P, ctypes.POINTER(_FrictionalInfo)]
    lib.adhesive_contact_solve.argtypes = [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, _P, _P, ctypes.POINTER(_AdhesiveInfo)]
    lib.elastoplastic_solve.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                        ctypes.POINTER(EPOptions), ctypes.POINTER(_State),
                                        ctypes.POINTER(_EPInfo)]
    lib.fvim_admit_index.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.c_int, ctypes.c_size_t,
                                     ctypes.c_size_t]
    lib.fvim_request_bytes.argtypes = [ctypes.POINTER(_Request)]
    lib.fvim_request_bytes.restype = ctypes.c_size_t
    lib.fvim_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.POINTER(_P)]
    lib.fvim_server_submit.argtypes = [_P, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.fvim_server_poll.argtypes = [_P, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_Result)]
    lib.fvim_server_release.argtypes = [_P, ctypes.c_uint64]
    lib.fvim_server_get_stats.argtypes = [_P, ctypes.POINTER(_ServerStats)]
    lib.fvim_server_destroy.argtypes = [_P]
    lib.fvim_server_destroy.restype = None
    _LIB = lib
    return lib


def _check(rc):
    if rc != FVIM_OK:
        msg = _LIB.fvim_last_error().decode()
        raise FvimError(rc, msg)


def _ptr(t, shape, name):
    """Device pointer of a contiguous float64 tensor of the given shape."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise FvimError(FVIM_EINVAL, "%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise FvimError(FVIM_EINVAL, "%s must live on the GPU" % name)
    if t.dtype != torch.float64:
        raise FvimError(FVIM_EINVAL, "%s must be float64" % name)
    if not t.is_contiguous():
        raise FvimError(FVIM_EINVAL, "%s must be contiguous" % name)
    if tuple(t.shape) != tuple(shape):
        raise FvimError(FVIM_EINVAL, "%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """One grid + material + precision; owns the device workspace.

    grid: dict(nx, ny, nz, lx, ly, lz).  Tensors passed to the methods must be
    float64, contiguous and on the context's device.
    """

    def __init__(self, grid, E, nu, sigma_y0=0.0, E_h=0.0, precision="fp64", k0="include",
                 stream=None):
        lib = load_library()
        self.grid = dict(grid)
        self.nx, self.ny, self.nz = int(grid["nx"]), int(grid["ny"]), int(grid["nz"])
        self.E, self.nu, self.sigma_y0, self.E_h = float(E), float(nu), float(sigma_y0), float(E_h)
        self._g = _Grid(self.nx, self.ny, self.nz, float(grid["lx"]), float(grid["ly"]), float(grid["lz"]))
        self._m = _Material(self.E, self.nu, self.sigma_y0, self.E_h)
        self._h = _P()
        _check(lib.fvim_create(ctypes.byref(self._g), ctypes.byref(self._m), PRECISION[precision],
                               K0[k0], _stream_handle(stream), ctypes.byref(self._h)))
        self.precision = precision

    def close(self):
        if self._h:
            _LIB.fvim_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    STAGES = ("x_fwd", "y_fwd", "x_fwd_t", "y_fwd_t", "depth", "y_inv", "x_inv", "depth_nyq")

    OPT_DEPTH_CONFIG, OPT_TUNE, OPT_GRAPHS, OPT_SIDE_STREAM, OPT_STREAMING, OPT_FFT_CONFIG, OPT_PERSISTENT = 1, 2, 3, 4, 5, 6, 7

    def fft_config(self):
        """[(tile, radix)] of the forward row, forward column, inverse column
        and inverse row transforms (the operator's precision)."""
        return unpack_fft_config(self.get_option(self.OPT_FFT_CONFIG))

    def set_fft_config(self, cfg):
        self.set_option(self.OPT_FFT_CONFIG, pack_fft_config(cfg))

    def set_option(self, key, value):
        _check(_LIB.fvim_set_option(self._h, int(key), int(value)))

    def get_option(self, key):
        v = ctypes.c_int()
        _check(_LIB.fvim_get_option(self._h, int(key), ctypes.byref(v)))
        return v.value

    def tune(self):
        """Time every depth-pass layout on the next operator call, keep the fastest."""
        self.set_option(self.OPT_TUNE, 1)

    def set_timing(self, on=True):
        _check(_LIB.fvim_set_timing(self._h, 1 if on else 0))

    def stage_times(self):
        """{stage: (total ms, launches)} since the last call (synchronises)."""
        n = len(self.STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(_LIB.fvim_stage_times(self._h, ms, cnt))
        return {s: (ms[i], cnt[i]) for i, s in enumerate(self.STAGES)}

    def set_stream(self, stream):
        _check(_LIB.fvim_set_stream(self._h, _stream_handle(stream)))

    def set_depth_nodes(self, z=None):
        """Non-uniform depth nodes (nz values, 0 ... lz, increasing); None
        restores the uniform ones."""
        if z is None:
            _check(_LIB.fvim_set_depth_nodes(self._h, None))
            return
        import numpy as np
        z = np.ascontiguousarray(z, dtype=np.float64)
        if z.shape != (self.nz,):
            raise FvimError(FVIM_EINVAL, "depth nodes: need %d values" % self.nz)
        _check(_LIB.fvim_set_depth_nodes(self._h, z.ctypes.data))

    # shapes
    @property
    def tensor_shape(self):
        return (6, self.nz, self.ny, self.nx)

    @property
    def vector_shape(self):
        return (3, self.nz, self.ny, self.nx)

    @property
    def scalar_shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def surface_shape(self):
        return (self.ny, self.nx)

    def _outputs(self, want, out, device):
        shapes = {"strain": self.tensor_shape, "stress": self.tensor_shape,
                  "disp": self.vector_shape, "surf_u3": self.surface_shape}
        res = dict(out or {})
        for k in want:
            if k not in shapes:
                raise FvimError(FVIM_EINVAL, "unknown output %r" % k)
            if k not in res:
                res[k] = torch.empty(shapes[k], dtype=torch.float64, device=device)
        ptrs = [_ptr(res.get(k), shapes[k], k) for k in ("strain", "stress", "disp", "surf_u3")]
        return res, ptrs

    def operator_apply(self, eps_p=None, traction=None, want=("strain",), out=None):
        """strain/stress/disp/surf_u3 of u = M[traction] + N[C:eps_p]."""
        dev = (eps_p if eps_p is not None else traction).device
        pe = _ptr(eps_p, self.tensor_shape, "eps_p")
        pt = _ptr(traction, (3, self.ny, self.nx), "traction")
        res, ptrs = self._outputs(want, out, dev)
        _check(_LIB.fvim_operator_apply(self._h, pe, pt, *ptrs))
        return res

    def operator_apply_noalloc(self, eps_p=None, traction=None, out=None):
        """operator_apply through the entry point that allocates nothing: the
        library's fixed per-device scratch holds the workspace.  out: dict of
        preallocated output tensors (strain, stress, disp, surf_u3), at least
        one."""
        if not out:
            raise FvimError(FVIM_EINVAL, "operator_apply_noalloc: pass preallocated outputs")
        pe = _ptr(eps_p, self.tensor_shape, "eps_p")
        pt = _ptr(traction, (3, self.ny, self.nx), "traction")
        res, ptrs = self._outputs((), out, None)
        _check(_LIB.fvim_operator_apply_noalloc(self._h, pe, pt, *ptrs))
        return res

    def mindlin_apply(self, eps_p, want=("strain",), out=None):
        pe = _ptr(eps_p, self.tensor_shape, "eps_p")
        res, ptrs = self._outputs(want, out, eps_p.device)
        _check(_LIB.mindlin_apply(self._h, pe, *ptrs))
        return res

    def boussinesq_apply(self, traction, want=("strain",), out=None):
        pt = _ptr(traction, (3, self.ny, self.nx), "traction")
        res, ptrs = self._outputs(want, out, traction.device)
        _check(_LIB.boussinesq_apply(self._h, pt, *ptrs))
        return res

    def return_map(self, d_eps, sigma_n, ep_n, d_eps_p=None, d_ep=None, sigma_np1=None):
        ts, ss = self.tensor_shape, self.scalar_shape
        dev = d_eps.device
        if d_eps_p is None:
            d_eps_p = torch.empty(ts, dtype=torch.float64, device=dev)
        if d_ep is None:
            d_ep = torch.empty(ss, dtype=torch.float64, device=dev)
        if sigma_np1 is None:
            sigma_np1 = torch.empty(ts, dtype=torch.float64, device=dev)
        _check(_LIB.return_map(self._h, _ptr(d_eps, ts, "d_eps"), _ptr(sigma_n, ts, "sigma_n"),
                               _ptr(ep_n, ss, "ep_n"), _ptr(d_eps_p, ts, "d_eps_p"),
                               _ptr(d_ep, ss, "d_ep"), _ptr(sigma_np1, ts, "sigma_np1")))
        return d_eps_p, d_ep, sigma_np1

    def contact_solve(self, h, W, tol=1e-14, max_iter=2000, p=None, want_gap=False):
        sh = self.surface_shape
        if p is None:
            p = torch.zeros(sh, dtype=torch.float64, device=h.device)
        gap = torch.empty(sh, dtype=torch.float64, device=h.device) if want_gap else None
        info = _ContactInfo()
        _check(_LIB.contact_solve(self._h, _ptr(h, sh, "h"), float(W), float(tol), int(max_iter),
                                  _ptr(p, sh, "p"), _ptr(gap, sh, "gap"), ctypes.byref(info)))
        return p, gap, contact_info_dict(info)

    def tangential_solve(self, p, mu_f, Q, tol=1e-12, max_iter=100000, q=None):
        """Partial-slip tangential traction (2, ny, nx) under the normal
        pressure p for the total tangential force Q = (Qx, Qy)."""
        sh = self.surface_shape
        if q is None:
            q = torch.empty((2,) + sh, dtype=torch.float64, device=p.device)
        info = _TangentialInfo()
        _check(_LIB.tangential_solve(self._h, _ptr(p, sh, "p"), float(mu_f), float(Q[0]), float(Q[1]),
                                     float(tol), int(max_iter), _ptr(q, (2,) + sh, "q"), ctypes.byref(info)))
        return q, {"iters": info.iters, "rel_change": info.rel_change, "stick_fraction": info.stick_fraction,
                   "shift": (info.shift[0], info.shift[1])}

    def frictional_contact_solve(self, h, W, mu_f, Q, coupled=True, tol=1e-13, max_iter=200, traction=None,
                                 warm=False):
        """Normal contact with Coulomb friction: the surface traction
        (3, ny, nx) = (q1, q2, p) for the load W and tangential force Q,
        coupled through the Cerruti cross terms or (coupled=False) in
        Goodman's sequence.  traction: warm start when warm, else its
        pressure plane is contact_solve's warm start (zeros: uniform)."""
        sh = self.surface_shape
        if traction is None:
            traction = torch.zeros((3,) + sh, dtype=torch.float64, device=h.device)
        info = _FrictionalInfo()
        _check(_LIB.frictional_contact_solve(self._h, _ptr(h, sh, "h"), float(W), float(mu_f), float(Q[0]),
                                             float(Q[1]), int(bool(coupled)), float(tol), int(max_iter),
                                             int(bool(warm)), _ptr(traction, (3,) + sh, "traction"),
                                             ctypes.byref(info)))
        out = {f: getattr(info, f) for f, _ in _FrictionalInfo._fields_ if f != "shift"}
        out["shift"] = (info.shift[0], info.shift[1])
        return traction, out

    def adhesive_contact_solve(self, h, W, sigma0, h0, tol=1e-14, max_iter=200, want_gap=False):
        """Adhesive contact (Dugdale cohesive zone): the total traction p
        (ny, nx) = p_c - sigma0 1[gap <= h0] for the load W."""
        sh = self.surface_shape
        p = torch.empty(sh, dtype=torch.float64, device=h.device)
        gap = torch.empty(sh, dtype=torch.float64, device=h.device) if want_gap else None
        info = _AdhesiveInfo()
        _check(_LIB.adhesive_contact_solve(self._h, _ptr(h, sh, "h"), float(W), float(sigma0), float(h0), float(tol),
                                           int(max_iter), _ptr(p, sh, "p"), _ptr(gap, sh, "gap"), ctypes.byref(info)))
        return p, gap, {f: getattr(info, f) for f, _ in _AdhesiveInfo._fields_}

    def new_state(self, device="cuda"):
        z = lambda s: torch.zeros(s, dtype=torch.float64, device=device)
        return {"eps_p": z(self.tensor_shape), "ep": z(self.scalar_shape), "sigma": z(self.tensor_shape),
                "traction": z((3, self.ny, self.nx)), "u3p": z(self.surface_shape)}

    def elastoplastic_solve(self, h, W_steps, state, opts=None):
        """Algorithm 1 over the cumulative loads W_steps; state updated in place."""
        opts = opts or EPOptions()
        ts, ss, sf = self.tensor_shape, self.scalar_shape, self.surface_shape
        st = _State(_ptr(state["eps_p"], ts, "eps_p"), _ptr(state["ep"], ss, "ep"),
                    _ptr(state["sigma"], ts, "sigma"), _ptr(state["traction"], (3,) + sf, "traction"),
                    _ptr(state["u3p"], sf, "u3p"))
        n = len(W_steps)
        ws = (ctypes.c_double * n)(*[float(w) for w in W_steps])
        infos = (_EPInfo * n)()
        rc = _LIB.elastoplastic_solve(self._h, _ptr(h, sf, "h"), ws, n, ctypes.byref(opts),
                                      ctypes.byref(st), infos)
        out = [{f: getattr(i, f) for f, _ in _EPInfo._fields_} for i in infos]
        if rc != FVIM_OK:
            # the steps before the failing one are committed to the state;
            # the records say which (committed == 1)
            err = FvimError(rc, _LIB.fvim_last_error().decode())
            err.infos = out
            raise err
        return out


def pack_fft_config(cfg):
    """FVIM_OPT_FFT_CONFIG value of four (tile, radix) choices."""
    v = 0
    for k, (tile, radix) in enumerate(cfg):
        v |= ((tile & 3) | (4 if radix == 8 else 0)) << (3 * k)
    return v


def unpack_fft_config(v):
    return [((v >> (3 * k)) & 3, 8 if (v >> (3 * k)) & 4 else 4) for k in range(4)]


def contact_info_dict(info):
    return {f: getattr(info, f) for f, _ in _ContactInfo._fields_}


# module-level functions with the C names
def mindlin_apply(ctx, eps_p, **kw):
    return ctx.mindlin_apply(eps_p, **kw)


def boussinesq_apply(ctx, traction, **kw):
    return ctx.boussinesq_apply(traction, **kw)


def operator_apply(ctx, eps_p=None, traction=None, **kw):
    return ctx.operator_apply(eps_p, traction, **kw)


def operator_apply_noalloc(ctx, eps_p=None, traction=None, out=None):
    return ctx.operator_apply_noalloc(eps_p, traction, out)


NOALLOC_BYTES = 128 << 20


def operator_apply_batch(ctxs, eps_p=None, traction=None, want=("strain",)):
    """The fused operator for several contexts (grids may differ) with the
    depth pass of up to 8 of them in one launch; ordered on ctxs[0]'s stream.
    eps_p / traction: lists of tensors (one per context) or None.  Returns a
    list of output dicts."""
    n = len(ctxs)
    if n == 0:
        raise FvimError(FVIM_EINVAL, "batch: no context")
    outs, cols = [], {k: [] for k in ("strain", "stress", "disp", "surf_u3")}
    ins = {"eps": [], "t": []}
    for i, c in enumerate(ctxs):
        e = eps_p[i] if eps_p is not None else None
        t = traction[i] if traction is not None else None
        ins["eps"].append(_ptr(e, c.tensor_shape, "eps_p"))
        ins["t"].append(_ptr(t, (3, c.ny, c.nx), "traction"))
        res, ptrs = c._outputs(want, None, (e if e is not None else t).device)
        outs.append(res)
        for k, p in zip(("strain", "stress", "disp", "surf_u3"), ptrs):
            cols[k].append(p)

    def arr(v, used):
        return (ctypes.c_void_p * n)(*v) if used else None

    keep = [arr(ins["eps"], eps_p is not None), arr(ins["t"], traction is not None)]
    keep += [arr(cols[k], k in want) for k in ("strain", "stress", "disp", "surf_u3")]
    hs = (ctypes.c_void_p * n)(*[c._h.value for c in ctxs])
    _check(_LIB.fvim_operator_apply_batch(hs, n, *keep))
    return outs


def return_map(ctx, d_eps, sigma_n, ep_n, **kw):
    return ctx.return_map(d_eps, sigma_n, ep_n, **kw)


def contact_solve(ctx, h, W, **kw):
    return ctx.contact_solve(h, W, **kw)


def tangential_solve(ctx, p, mu_f, Q, **kw):
    return ctx.tangential_solve(p, mu_f, Q, **kw)


def frictional_contact_solve(ctx, h, W, mu_f, Q, **kw):
    return ctx.frictional_contact_solve(h, W, mu_f, Q, **kw)


def adhesive_contact_solve(ctx, h, W, sigma0, h0, **kw):
    return ctx.adhesive_contact_solve(h, W, sigma0, h0, **kw)


def elastoplastic_solve(ctx, h, W_steps, state, opts=None):
    return ctx.elastoplastic_solve(h, W_steps, state, opts)


def admit_index(pending_bytes, budget, in_use):
    """The server's admission rule (pure): index of the first pending request
    whose footprint fits in budget - in_use, or -1."""
    lib = load_library()
    arr = (ctypes.c_size_t * max(1, len(pending_bytes)))(*pending_bytes)
    return lib.fvim_admit_index(arr, len(pending_bytes), int(budget), int(in_use))


def make_request(grid, h, W_steps, E=1.0, nu=0.3, sigma_y0=0.01, E_h=0.1, precision="fp64", opts=None,
                 z=None):
    import numpy as np
    h = np.ascontiguousarray(h, dtype=np.float64)
    if h.shape != (grid["ny"], grid["nx"]):
        raise FvimError(FVIM_EINVAL, "h must have shape (ny, nx)")
    if not 1 <= len(W_steps) <= MAX_STEPS:
        raise FvimError(FVIM_EINVAL, "between 1 and %d load steps" % MAX_STEPS)
    r = _Request()
    r.grid = _Grid(int(grid["nx"]), int(grid["ny"]), int(grid["nz"]), float(grid["lx"]), float(grid["ly"]),
                   float(grid["lz"]))
    r.mat = _Material(float(E), float(nu), float(sigma_y0), float(E_h))
    r.precision = PRECISION[precision]
    r.n_steps = len(W_steps)
    for i, w in enumerate(W_steps):
        r.W_steps[i] = float(w)
    r.opts = opts or EPOptions()
    r.h = h.ctypes.data
    if z is not None:
        z = np.ascontiguousarray(z, dtype=np.float64)
        if z.shape != (grid["nz"],):
            raise FvimError(FVIM_EINVAL, "depth nodes: need %d values" % grid["nz"])
        r.z = z.ctypes.data
    return r, (h, z)


def request_bytes(grid, precision="fp64", opts=None):
    import numpy as np
    lib = load_library()
    r, _ = make_request(grid, np.zeros((grid["ny"], grid["nx"])), [1.0], precision=precision, opts=opts)
    return lib.fvim_request_bytes(ctypes.byref(r))


class Server:
    """Continuous-batching solve server (see fvim.h): requests are admitted by
    free slot and HBM footprint and run concurrently on their own streams."""

    def __init__(self, hbm_budget_bytes, max_slots=4, device=0):
        lib = load_library()
        self._s = _P()
        _check(lib.fvim_server_create(int(hbm_budget_bytes), int(max_slots), int(device), ctypes.byref(self._s)))

    def submit(self, grid, h, W_steps, **kw):
        r, keep = make_request(grid, h, W_steps, **kw)
        rid = ctypes.c_uint64()
        _check(_LIB.fvim_server_submit(self._s, ctypes.byref(r), ctypes.byref(rid)))
        del keep
        return rid.value

    def poll(self, rid, wait=False):
        """None while pending or running; else a dict with the result (arrays copied)."""
        import numpy as np
        res = _Result()
        rc = _LIB.fvim_server_poll(self._s, ctypes.c_uint64(rid), 1 if wait else 0, ctypes.byref(res))
        if rc < 0:
            _check(rc)
        if rc == 0:
            return None
        out = {f: getattr(res, f) for f in ("status", "t_submit", "t_admit", "t_done", "contact_fraction")}
        out["info"] = {f: getattr(res.info, f) for f, _ in _EPInfo._fields_}
        out["error"] = res.error.decode(errors="replace")
        out["p"] = out["u3p"] = None
        return out, res

    def result_arrays(self, res, shape):
        import numpy as np
        n = shape[0] * shape[1]
        p = np.ctypeslib.as_array((ctypes.c_double * n).from_address(res.p)).reshape(shape).copy()
        u = np.ctypeslib.as_array((ctypes.c_double * n).from_address(res.u3p)).reshape(shape).copy()
        return p, u

    def wait(self, rid, shape):
        out, res = self.poll(rid, wait=True)
        if out["status"] == 0:
            out["p"], out["u3p"] = self.result_arrays(res, shape)
        _check(_LIB.fvim_server_release(self._s, ctypes.c_uint64(rid)))
        return out

    def stats(self):
        st = _ServerStats()
        _check(_LIB.fvim_server_get_stats(self._s, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _ServerStats._fields_}

    def close(self):
        if self._s:
            _LIB.fvim_server_destroy(self._s)
            self._s = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
