"""Thin Python binding of librbffd (include/rbffd.h): argument marshalling only.

Every function takes torch tensors that live on the context's GPU, checks
their dtype, shape and contiguity, and passes raw device pointers to the
C ABI. All arithmetic happens in the library's HIP kernels; if the library
is missing this module raises at import time.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# RBFFD_LIBRARY may point at another build of the same library
LIB_PATH = os.environ.get("RBFFD_LIBRARY", os.path.join(_HERE, "librbffd.so"))
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1509_02615_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, ESINGULAR, ENONFINITE = 0, -1, -2, -3, -4, -5
DX, DZ, LAP, HYPERLAP, DZZ, DXX = 1, 2, 3, 4, 5, 6
SOLVE_FP64, SOLVE_FP32_IR = 0, 1
F64, F32, BF16 = 0, 1, 2
PHYS_ADVECTION, PHYS_NS = 1, 2
RK4, WSRK3 = 0, 1

_vp = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class Op(ctypes.Structure):
    _fields_ = [("kind", _i32), ("k", _i32), ("phs_order", _i32), ("reserved", _i32)]


class Stencils(ctypes.Structure):
    _fields_ = [("n_nodes", _i64), ("xy", _vp), ("period_x", _f64), ("n_centers", _i64),
                ("centers", _vp), ("n_max", _i32), ("n_per", _vp), ("m_uniform", _i32),
                ("m_per", _vp), ("l_uniform", _i32), ("l_per", _vp), ("idx_in", _vp)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("physics", _i32), ("field_dtype", _i32), ("weight_dtype", _i32), ("n", _i32),
                ("n_total", _i64), ("n_active", _i64), ("ensemble", _i32), ("reserved0", _i32),
                ("idx", _vp), ("w", _vp), ("xy", _vp), ("hv_coeff", _f64),
                ("vel_u", _vp), ("vel_v", _vp), ("vel_period", _f64),
                ("c_p", _f64), ("c_v", _f64), ("R_d", _f64), ("g", _f64), ("theta_bar", _f64),
                ("mu", _f64), ("u_bar", _f64), ("n_bnd", _i32), ("reserved1", _i32), ("bnd_nodes", _vp),
                ("bnd_ghosts", _vp), ("bnd_normal", _vp), ("bnd_d1", _vp), ("bnd_d2", _vp),
                ("mirror_src", _vp)]


_lib.rbffd_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp]
_lib.rbffd_destroy.argtypes = [_vp]
_lib.rbffd_last_error.argtypes = [_vp]
_lib.rbffd_last_error.restype = ctypes.c_char_p
_lib.rbffd_sync.argtypes = [_vp]
_lib.rbffd_knn.argtypes = [_vp, ctypes.POINTER(Stencils), _vp]
_lib.rbffd_weights.argtypes = [_vp, ctypes.POINTER(Stencils), ctypes.POINTER(Op), ctypes.c_int,
                               ctypes.c_int, _vp, _vp, _vp]
_lib.rbffd_weights_tune.argtypes = [_vp, ctypes.POINTER(Stencils), ctypes.POINTER(Op), ctypes.c_int,
                                    ctypes.c_int, _vp, _vp, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_f64)]
_lib.rbffd_weights_noalloc.argtypes = [_vp, ctypes.POINTER(Stencils), ctypes.POINTER(Op), ctypes.c_int,
                                       ctypes.c_int, _vp, _vp, _vp]
_lib.rbffd_model_create.argtypes = [_vp, ctypes.POINTER(ModelDesc), ctypes.POINTER(_vp)]
_lib.rbffd_model_destroy.argtypes = [_vp]
_lib.rbffd_ghost.argtypes = [_vp, _vp, _vp]
_lib.rbffd_rhs.argtypes = [_vp, _vp, _f64, _vp, _vp]
_lib.rbffd_step.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_f64), _f64, _i64, ctypes.c_int]
_lib.rbffd_model_bytes_per_node.argtypes = [_vp]
_lib.rbffd_model_bytes_per_node.restype = _i64
_lib.rbffd_model_profile.argtypes = [_vp, ctypes.c_int]
_lib.rbffd_model_profile_read.argtypes = [_vp, ctypes.POINTER(_f64), ctypes.POINTER(_i64)]
_lib.rbffd_stream_copy.argtypes = [_vp, _vp, _vp, _i64]
_lib.rbffd_mfma_probe.argtypes = [_vp, ctypes.c_int, _vp, _i64, ctypes.c_int, ctypes.POINTER(_i64)]
_lib.rbffd_model_tune.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_f64)]


class ClosureDesc(ctypes.Structure):
    _fields_ = [("max_samples", _i64), ("init_params", _vp), ("node_feature", _vp),
                ("in_scale", ctypes.c_float * 4), ("out_scale", ctypes.c_float * 4),
                ("activation", ctypes.c_int32)]


ACT_TANH, ACT_RELU = 0, 1
CLOSURE_NPARAMS = 128 * 160 + 128 + 128 * 128 + 128 + 16 * 128 + 16
_lib.rbffd_closure_create.argtypes = [_vp, _vp, ctypes.POINTER(ClosureDesc), ctypes.POINTER(_vp)]
_lib.rbffd_closure_destroy.argtypes = [_vp]
_lib.rbffd_closure_params.argtypes = [_vp]
_lib.rbffd_closure_params.restype = _vp
_lib.rbffd_closure_forward.argtypes = [_vp, _vp, _vp, _vp]
_lib.rbffd_closure_tune.argtypes = [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_f64)]
_lib.rbffd_closure_gradient.argtypes = [_vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_f64)]
_lib.rbffd_closure_train_step.argtypes = [_vp, _vp, _vp, _vp, _f64, ctypes.POINTER(_f64)]
_lib.rbffd_closure_step.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_f64), _f64, _i64, ctypes.c_int,
                                    ctypes.POINTER(_i64)]

EXPORTS = ["rbffd_create", "rbffd_destroy", "rbffd_last_error", "rbffd_sync", "rbffd_knn",
           "rbffd_weights", "rbffd_weights_tune", "rbffd_weights_noalloc", "rbffd_model_create", "rbffd_model_destroy", "rbffd_ghost",
           "rbffd_rhs", "rbffd_step", "rbffd_model_bytes_per_node", "rbffd_model_profile",
           "rbffd_model_profile_read", "rbffd_stream_copy", "rbffd_mfma_probe", "rbffd_model_tune", "rbffd_closure_create",
           "rbffd_closure_destroy", "rbffd_closure_params", "rbffd_closure_forward", "rbffd_closure_tune", "rbffd_closure_gradient",
           "rbffd_closure_train_step", "rbffd_closure_step"]


class RbffdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rbffd error {code}: {msg}")
        self.code = code


def _ptr(t, dtype, shape=None, name="array"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


class Context:
    """rbffd_create on ``device`` ordered on torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = _vp()
        rc = _lib.rbffd_create(ctypes.byref(h), device, _vp(stream.cuda_stream))
        if rc != OK:
            raise RbffdError(rc, "rbffd_create failed")
        self.h = h

    def close(self, _destroy=_lib.rbffd_destroy):
        # the destroy function is bound at class creation so that objects
        # collected at interpreter exit still release their handle
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    __del__ = close

    def check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise RbffdError(rc, _lib.rbffd_last_error(self.h).decode())
        return rc

    def sync(self):
        self.check(_lib.rbffd_sync(self.h))


def _stencils(xy, n_max, period_x, centers, n_per, m, l, m_per, l_per, idx_in, n_centers=None):
    N = xy.shape[0]
    nc = centers.shape[0] if centers is not None else (
        n_per.shape[0] if n_per is not None else (idx_in.shape[0] if idx_in is not None else (
            n_centers if n_centers is not None else N)))
    st = Stencils(n_nodes=N, xy=_ptr(xy, torch.float64, (N, 2), "xy"), period_x=float(period_x),
                  n_centers=nc, centers=_ptr(centers, torch.int32, (nc,), "centers"),
                  n_max=int(n_max), n_per=_ptr(n_per, torch.int32, (nc,), "n_per"),
                  m_uniform=int(m), m_per=_ptr(m_per, torch.int32, (nc,), "m_per"),
                  l_uniform=int(l), l_per=_ptr(l_per, torch.int32, (nc,), "l_per"),
                  idx_in=_ptr(idx_in, torch.int32, (nc, n_max), "idx_in"))
    return st, nc


def rbffd_knn(ctx: Context, xy, n_max, period_x=0.0, centers=None, n_per=None, out=None, n_centers=None):
    """A1: int32 [Nc][n_max] nearest-node stencils (see rbffd.h). Without
    ``centers`` the centres are nodes 0..n_centers-1 (default: all)."""
    st, nc = _stencils(xy, n_max, period_x, centers, n_per, 1, 0, None, None, None, n_centers)
    if out is None:
        out = torch.empty((nc, n_max), dtype=torch.int32, device=xy.device)
    ctx.check(_lib.rbffd_knn(ctx.h, ctypes.byref(st), _ptr(out, torch.int32, (nc, n_max), "idx")))
    return out


NOALLOC_MAX_NODES = NOALLOC_MAX_CENTERS = 2097152
WEIGHT_BUCKETS = 6
WEIGHT_SHAPES = [4, 2, 2, 4, 4, 4]     # launch shapes per size bucket


def rbffd_weights(ctx: Context, xy, ops, n_max, m=0, l=0, period_x=0.0, centers=None, n_per=None,
                  m_per=None, l_per=None, idx_in=None, precision=SOLVE_FP64, out=None, n_centers=None,
                  _entry=None):
    """A1-A4: returns (idx [Nc][n_max], w [n_ops][Nc][n_max] FP64, status [Nc], rc).
    ops: list of (kind, k, phs_order). rc is OK or ESINGULAR."""
    entry = _lib.rbffd_weights if _entry is None else _entry
    st, nc = _stencils(xy, n_max, period_x, centers, n_per, m, l, m_per, l_per, idx_in, n_centers)
    dev = xy.device
    op_arr = (Op * len(ops))(*[Op(kind, k, order, 0) for (kind, k, order) in ops])
    if out is None:
        idx = idx_in if idx_in is not None else torch.empty((nc, n_max), dtype=torch.int32, device=dev)
        w = torch.empty((len(ops), nc, n_max), dtype=torch.float64, device=dev)
        status = torch.empty((nc,), dtype=torch.int32, device=dev)
    else:
        idx, w, status = out
    idx_out = None if idx_in is not None else _ptr(idx, torch.int32, (nc, n_max), "idx")
    rc = ctx.check(entry(ctx.h, ctypes.byref(st), op_arr, len(ops), int(precision), idx_out,
                                      _ptr(w, torch.float64, (len(ops), nc, n_max), "w"),
                                      _ptr(status, torch.int32, (nc,), "status")), allow=(ESINGULAR,))
    return idx, w, status, rc


def rbffd_weights_tune(ctx: Context, xy, ops, n_max, shapes=None, **kw):
    """rbffd_weights that also picks each size bucket's launch shape (kept in
    the context for later calls). ``shapes``: per-bucket list, -1 = tune,
    >= 0 = force. Returns (idx, w, status, rc, chosen shapes, ms per bucket)."""
    sh = (_i32 * WEIGHT_BUCKETS)(*([-1] * WEIGHT_BUCKETS if shapes is None else shapes))
    ms = (_f64 * WEIGHT_BUCKETS)()

    def entry(h, st, op_arr, n_ops, prec, idx_out, w, status):
        return _lib.rbffd_weights_tune(h, st, op_arr, n_ops, prec, idx_out, w, status, sh, ms)
    idx, w, status, rc = rbffd_weights(ctx, xy, ops, n_max, _entry=entry, **kw)
    return idx, w, status, rc, list(sh), list(ms)


def rbffd_weights_noalloc(ctx: Context, xy, ops, n_max, out, **kw):
    """rbffd_weights without any device allocation inside the library (its
    scratch is a fixed per-device region): the outputs ``out`` = (idx, w,
    status) are the caller's. Same results as rbffd_weights."""
    return rbffd_weights(ctx, xy, ops, n_max, out=out, _entry=_lib.rbffd_weights_noalloc, **kw)


class Model:
    """rbffd_model_create / rbffd_ghost / rbffd_rhs / rbffd_step."""

    def __init__(self, ctx: Context, physics, idx, w, xy, n_active, field_dtype=F64, weight_dtype=F64,
                 ensemble=1, hv_coeff=0.0, vel_u=None, vel_v=None, vel_period=1.0, consts=None,
                 bnd_nodes=None, bnd_ghosts=None, bnd_normal=None, bnd_d1=None, bnd_d2=None, mirror_src=None):
        self.ctx = ctx
        N = xy.shape[0]
        na, n = idx.shape
        self.N, self.Na, self.n, self.E = N, na, n, ensemble
        self.F = 4 if physics == PHYS_NS else 1
        self.dtype = torch.float64 if field_dtype == F64 else torch.float32
        n_ops = 4 if physics == PHYS_NS else 3
        c = consts or {}
        d = ModelDesc(physics=physics, field_dtype=field_dtype, weight_dtype=weight_dtype, n=n,
                      n_total=N, n_active=na, ensemble=ensemble,
                      idx=_ptr(idx, torch.int32, (na, n), "idx"),
                      w=_ptr(w, torch.float64, (n_ops, na, n), "w"),
                      xy=_ptr(xy, torch.float64, (N, 2), "xy"), hv_coeff=float(hv_coeff),
                      vel_u=_ptr(vel_u, torch.float64, (N,), "vel_u"),
                      vel_v=_ptr(vel_v, torch.float64, (N,), "vel_v"), vel_period=float(vel_period),
                      c_p=c.get("c_p", 0.0), c_v=c.get("c_v", 0.0), R_d=c.get("R_d", 0.0),
                      g=c.get("g", 0.0), theta_bar=c.get("theta_bar", 0.0), mu=c.get("mu", 0.0),
                      u_bar=c.get("u_bar", 0.0))
        if bnd_nodes is not None:
            nr = bnd_nodes.shape[0]
            d.n_bnd = nr
            d.bnd_nodes = _ptr(bnd_nodes, torch.int32, (nr,), "bnd_nodes")
            d.bnd_ghosts = _ptr(bnd_ghosts, torch.int32, (nr,), "bnd_ghosts")
            d.bnd_normal = _ptr(bnd_normal, torch.int32, (nr,), "bnd_normal")
            d.bnd_d1 = _ptr(bnd_d1, torch.float64, (nr, n), "bnd_d1")
            d.bnd_d2 = _ptr(bnd_d2, torch.float64, (nr, n), "bnd_d2")
        if mirror_src is not None:
            d.mirror_src = _ptr(mirror_src, torch.int32, (N - na,), "mirror_src")
        h = _vp()
        ctx.check(_lib.rbffd_model_create(ctx.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h

    def close(self, _destroy=_lib.rbffd_model_destroy):
        # the destroy function is bound at class creation so that objects
        # collected at interpreter exit still release their handle
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    __del__ = close

    def state_shape(self):
        return (self.N, self.E, self.F)

    def _state(self, s, name="state"):
        return _ptr(s, self.dtype, self.state_shape(), name)

    def bytes_per_node(self):
        return int(_lib.rbffd_model_bytes_per_node(self.h))

    def profile(self, enable=True):
        self.ctx.check(_lib.rbffd_model_profile(self.h, int(enable)))

    def profile_read(self):
        """(summed fused-RHS kernel ms, launches) since the last read."""
        ms, n = _f64(), _i64()
        self.ctx.check(_lib.rbffd_model_profile_read(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


def rbffd_model_create(ctx, *args, **kw) -> Model:
    return Model(ctx, *args, **kw)


def rbffd_ghost(ctx: Context, model: Model, state):
    ctx.check(_lib.rbffd_ghost(ctx.h, model.h, model._state(state)))


def rbffd_rhs(ctx: Context, model: Model, t, state, tendency):
    ctx.check(_lib.rbffd_rhs(ctx.h, model.h, float(t), model._state(state),
                             model._state(tendency, "tendency")))


def rbffd_model_tune(ctx: Context, model: Model, state, shape=-1):
    """Pick the fastest stage-kernel launch shape on this model's data (or
    keep `shape` if it is not -1); returns (shape index, microseconds per
    launch)."""
    ch, us = ctypes.c_int(shape), _f64()
    ctx.check(_lib.rbffd_model_tune(ctx.h, model.h, model._state(state), ctypes.byref(ch), ctypes.byref(us)))
    return ch.value, us.value


def rbffd_stream_copy(ctx: Context, dst, src):
    """Plain streaming copy of src into dst (same size, CUDA/HIP tensors)."""
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("contiguous device tensors required")
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("size mismatch")
    ctx.check(_lib.rbffd_stream_copy(ctx.h, dst.data_ptr(), src.data_ptr(), nb))


def rbffd_mfma_probe(ctx: Context, out, iters, shape=1):
    """Matrix-core throughput probe (shape 0: 16x16x32, 1: 32x32x16 BF16
    products) into `out` (float32 device tensor of at least 1024 x CUs
    values); returns the launch's flop count."""
    if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()):
        raise ValueError("contiguous float32 device tensor required")
    fl = _i64(0)
    ctx.check(_lib.rbffd_mfma_probe(ctx.h, int(shape), out.data_ptr(), out.numel(), int(iters), ctypes.byref(fl)))
    return fl.value


def rbffd_step(ctx: Context, model: Model, state, t, dt, n_steps, tableau=RK4):
    """Advance in place; returns the new time. Raises on ENONFINITE."""
    tt = _f64(float(t))
    ctx.check(_lib.rbffd_step(ctx.h, model.h, model._state(state), ctypes.byref(tt), float(dt),
                              int(n_steps), int(tableau)))
    return tt.value


class Closure:
    """rbffd_closure_*: the learned coarse correction bound to an FP32
    Navier-Stokes model."""

    def __init__(self, ctx: Context, model: Model, init_params, node_feature, in_scale, out_scale,
                 max_samples=None, activation=ACT_TANH):
        self.ctx, self.model = ctx, model
        d = ClosureDesc(max_samples=int(max_samples or model.Na * model.E),
                        init_params=_ptr(init_params, torch.float32, (CLOSURE_NPARAMS,), "init_params"),
                        node_feature=_ptr(node_feature, torch.float64, (model.Na,), "node_feature"),
                        activation=int(activation))
        d.in_scale[:] = [float(v) for v in in_scale]
        d.out_scale[:] = [float(v) for v in out_scale]
        h = _vp()
        ctx.check(_lib.rbffd_closure_create(ctx.h, model.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h

    def close(self, _destroy=_lib.rbffd_closure_destroy):
        # the destroy function is bound at class creation so that objects
        # collected at interpreter exit still release their handle
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    __del__ = close

    def params(self):
        """A copy of the FP32 master parameters (torch tensor on the device)."""
        p = _lib.rbffd_closure_params(self.h)
        out = torch.empty(CLOSURE_NPARAMS, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        _copy_device(out.data_ptr(), p, 4 * CLOSURE_NPARAMS)
        return out

    def _t(self, t, name):
        m = self.model
        return _ptr(t, torch.float32, (m.Na, m.E, 4), name)

    def forward(self, state):
        out = torch.empty((self.model.Na, self.model.E, 4), dtype=torch.float32, device="cuda")
        self.ctx.check(_lib.rbffd_closure_forward(self.ctx.h, self.h, self.model._state(state), out.data_ptr()))
        return out

    def tune(self, state, shape=-1):
        """rbffd_closure_tune: (chosen launch shape, us per forward call);
        ``shape`` >= 0 forces that shape."""
        ch, us = ctypes.c_int(shape), _f64()
        self.ctx.check(_lib.rbffd_closure_tune(self.ctx.h, self.h, self.model._state(state), ctypes.byref(ch),
                                               ctypes.byref(us)))
        return ch.value, us.value

    def gradient(self, state, target):
        g = torch.empty(CLOSURE_NPARAMS, dtype=torch.float32, device="cuda")
        loss = _f64()
        self.ctx.check(_lib.rbffd_closure_gradient(self.ctx.h, self.h, self.model._state(state),
                                                   self._t(target, "target"), g.data_ptr(), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, state, target, lr):
        loss = _f64()
        self.ctx.check(_lib.rbffd_closure_train_step(self.ctx.h, self.h, self.model._state(state),
                                                     self._t(target, "target"), float(lr), ctypes.byref(loss)))
        return loss.value

    def step(self, state, t, dt, n_steps, tableau=RK4):
        tt, fb = _f64(float(t)), _i64()
        self.ctx.check(_lib.rbffd_closure_step(self.ctx.h, self.h, self.model._state(state), ctypes.byref(tt),
                                               float(dt), int(n_steps), int(tableau), ctypes.byref(fb)))
        return tt.value, fb.value


_hip = None


def _copy_device(dst, src, nbytes):
    """Device-to-device copy through the HIP runtime the library links."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [_vp, _vp, ctypes.c_size_t, ctypes.c_int]
    rc = _hip.hipMemcpy(_vp(dst), _vp(src), nbytes, 3)      # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed ({rc})")
