"""ctypes binding of the casclb C ABI (``include/casclb.h``).

Argument marshalling only: every function has the name and meaning of the C
function it wraps, takes numpy arrays for host buffers and raw integers
(``tensor.data_ptr()``, ``stream.cuda_stream``) for device pointers and
streams, and raises :class:`LbError` when the C call returns an error code.
All computation happens in the HIP library; there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcasclb.so")

LB_ABI_VERSION = 1
LB_OK, LB_EINVAL, LB_ENOMEM, LB_EHIP, LB_ENONFINITE, LB_ESTATE = 0, -1, -2, -3, -4, -5
LB_D2Q9, LB_D2Q9_D2Q5, LB_D3Q27, LB_D3Q15 = 0, 1, 2, 3
LB_PERIODIC, LB_HALFWAY_BB = 0, 1
LB_STORE_F64, LB_STORE_F32_DEV, LB_STORE_F16_DEV = 0, 1, 2
LB_DTYPE_F64, LB_DTYPE_F32 = 0, 1
LB_MEM_HOST, LB_MEM_DEVICE = 0, 1
LB_TIME_CONSTANT, LB_TIME_COS = 0, 1
LB_MOMENTS_OUTPUT, LB_MOMENTS_HALF_FORCED = 0, 1
LB_FLAG_EXTERNAL_BUFFERS, LB_FLAG_XCD_REMAP, LB_FLAG_DEBUG_POISON, LB_FLAG_F16_NEAREST = 1, 2, 4, 8

_ERRNAMES = {LB_EINVAL: "LB_EINVAL", LB_ENOMEM: "LB_ENOMEM", LB_EHIP: "LB_EHIP", LB_ENONFINITE: "LB_ENONFINITE",
             LB_ESTATE: "LB_ESTATE"}


class LbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class lb_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("lattice", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("bc", ctypes.c_int32 * 3),
        ("residual_interval", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("omega_bulk", ctypes.c_double),
        ("omega_third", ctypes.c_double),
        ("omega_fourth", ctypes.c_double),
        ("D_phi", ctypes.c_double),
        ("omega_phi_high", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("plane_pad", ctypes.c_int64),
        ("block_x", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("rows_per_thread", ctypes.c_int32),
        ("x_pairs", ctypes.c_int32),
    ]


class lb_info(ctypes.Structure):
    _fields_ = [
        ("nodes", ctypes.c_int64),
        ("q", ctypes.c_int32),
        ("q_scalar", ctypes.c_int32),
        ("plane_stride", ctypes.c_int64),
        ("elem_bytes", ctypes.c_int32),
        ("block_x", ctypes.c_int32),
        ("bytes_per_update", ctypes.c_double),
        ("buf_current", ctypes.c_void_p),
        ("buf_other", ctypes.c_void_p),
        ("step_kernel", ctypes.c_char_p),
    ]


class lb_batch_domain(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("force_x", ctypes.c_double),
        ("lorentz", ctypes.c_double),
    ]


class lb_batch_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("check_interval", ctypes.c_int32),
        ("rho0", ctypes.c_double),
        ("omega_bulk", ctypes.c_double),
        ("omega_third", ctypes.c_double),
        ("omega_fourth", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("block", ctypes.c_int32),
        ("lds_policy", ctypes.c_int32),
        ("lds_bytes", ctypes.c_int32),
        ("routed", ctypes.c_int32),
        ("routed_cus", ctypes.c_int32),
    ]


LB_BATCH_NOT_RUN, LB_BATCH_CONVERGED, LB_BATCH_STATIONARY, LB_BATCH_MAX_STEPS, LB_BATCH_NONFINITE = 0, 1, 2, 3, 4

LB_UNET_ABI_VERSION = 1
LB_UNET_MAX_LEVELS = 6


class lb_unet_config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("channels", ctypes.c_int32 * LB_UNET_MAX_LEVELS),
        ("in_channels", ctypes.c_int32),
        ("out_channels", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]

class lb_warm_channel(ctypes.Structure):
    _fields_ = [("src", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("scale", ctypes.c_double),
                ("offset", ctypes.c_double)]


LB_WARM_MAX_L = 2048
LB_WARM_MAX_CHANNELS = 16
LB_WARM_MAX_K2 = 8

_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

# C function name -> (restype, argtypes)
SIGNATURES = {
    "lb_config_default": (None, [ctypes.POINTER(lb_config)]),
    "lb_validate_config": (ctypes.c_int, [ctypes.POINTER(lb_config), ctypes.c_char_p, ctypes.c_size_t]),
    "lb_required_bytes": (ctypes.c_size_t, [ctypes.POINTER(lb_config)]),
    "lb_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(lb_config)]),
    "lb_destroy": (None, [_P]),
    "lb_last_error": (ctypes.c_char_p, [_P]),
    "lb_bind_buffers": (ctypes.c_int, [_P, _P, _P, ctypes.c_size_t]),
    "lb_init_equilibrium": (ctypes.c_int, [_P, _P, _P, _P]),
    "lb_set_force_uniform": (ctypes.c_int, [_P, _D, _D, _D]),
    "lb_set_force_field": (ctypes.c_int, [_P, _P, _I32, _I32]),
    "lb_set_force_time": (ctypes.c_int, [_P, _I32, _D]),
    "lb_set_source_uniform": (ctypes.c_int, [_P, _D]),
    "lb_set_source_field": (ctypes.c_int, [_P, _P, _I32, _I32]),
    "lb_set_source_time": (ctypes.c_int, [_P, _I32, _D]),
    "lb_step": (ctypes.c_int, [_P, _I64]),
    "lb_synchronize": (ctypes.c_int, [_P]),
    "lb_get_step": (_I64, [_P]),
    "lb_set_step": (ctypes.c_int, [_P, _I64]),
    "lb_read_moments": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
    "lb_read_populations": (ctypes.c_int, [_P, _P, _P]),
    "lb_write_populations": (ctypes.c_int, [_P, _P, _P]),
    "lb_read_populations_box": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), _P, _P]),
    "lb_totals": (ctypes.c_int, [_P, ctypes.POINTER(_D)]),
    "lb_totals_noalloc": (ctypes.c_int, [_P, _P]),
    "lb_residual": (ctypes.c_int, [_P, ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "lb_residual_scalar": (ctypes.c_int, [_P, ctypes.POINTER(_D)]),
    "lb_set_wall_velocity": (ctypes.c_int, [_P, _I32, _I32, _D, _D, _D]),
    "lb_set_scalar_wall": (ctypes.c_int, [_P, _I32, _I32, _I32, _D]),
    "lb_set_viscous_heating": (ctypes.c_int, [_P, _D]),
    "lb_set_lorentz": (ctypes.c_int, [_P, _D]),
    "lb_get_info": (ctypes.c_int, [_P, ctypes.POINTER(lb_info)]),
    "lb_stream_copy": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "lb_stream_bench": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _I32, _I32, _I64, _P]),
    "lb_batch_config_default": (None, [ctypes.POINTER(lb_batch_config)]),
    "lb_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(lb_batch_config),
                                       ctypes.POINTER(lb_batch_domain), _I32]),
    "lb_batch_destroy": (None, [_P]),
    "lb_batch_last_error": (ctypes.c_char_p, [_P]),
    "lb_batch_init": (ctypes.c_int, [_P]),
    "lb_batch_run": (ctypes.c_int, [_P, _I64, _D]),
    "lb_batch_results": (ctypes.c_int, [_P, _P, _P, _P]),
    "lb_batch_read_moments": (ctypes.c_int, [_P, _I32, _P, _P]),
    "lb_batch_read_populations": (ctypes.c_int, [_P, _I32, _P]),
    "lb_batch_write_populations": (ctypes.c_int, [_P, _I32, _P]),
    "lb_batch_autotune": (ctypes.c_int, [_P, _I64, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                         ctypes.POINTER(_D)]),
    "lb_unet_config_default": (None, [ctypes.POINTER(lb_unet_config)]),
    "lb_unet_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.POINTER(lb_unet_config)]),
    "lb_unet_destroy": (None, [_P]),
    "lb_unet_last_error": (ctypes.c_char_p, [_P]),
    "lb_unet_num_params": (_I64, [_P]),
    "lb_unet_set_params": (ctypes.c_int, [_P, _P]),
    "lb_unet_get_params": (ctypes.c_int, [_P, _P]),
    "lb_unet_forward": (ctypes.c_int, [_P, _P, _I32, _P]),
    "lb_unet_loss_grad": (ctypes.c_int, [_P, _P, _P, _I32, ctypes.POINTER(_D), _P]),
    "lb_unet_adam": (ctypes.c_int, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]),
    "lb_unet_train_step": (ctypes.c_int, [_P, _P, _P, _I32, ctypes.c_float, ctypes.POINTER(_D)]),
    "lb_unet_macs_per_image": (_D, [_P]),
    "lb_unet_set_lowpass_loss": (ctypes.c_int, [_P, _I32, ctypes.c_float]),
    "lb_init_equilibrium_device": (ctypes.c_int, [_P, _P, _P, _P]),
    "lb_reset_moments_device": (ctypes.c_int, [_P, _P, _P, _P]),
    "lb_read_moments_device": (ctypes.c_int, [_P, _I32, _P, _P, _P]),
    "lb_warm_restrict": (ctypes.c_int, [_P, _I32, _I32, _D, _P, _P]),
    "lb_warm_prolong": (ctypes.c_int, [_P, _I32, _I32, _D, _P, _P]),
    "lb_warm_axpby": (ctypes.c_int, [_I64, _D, _P, _D, _P, _P, _P]),
    "lb_warm_project": (ctypes.c_int, [_P, _I32, _I32, _I32, _P]),
    "lb_warm_pack": (ctypes.c_int, [ctypes.POINTER(lb_warm_channel), _I32, _I32, _I64, _P, _P]),
    "lb_warm_unpack": (ctypes.c_int, [_P, ctypes.POINTER(lb_warm_channel), _I32, _I32, _I64, _P]),
    "lb_warm_initial_state": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I64, _D, _I32, _P, _P, _P, _P]),
}


def lib():
    """The loaded HIP library.  Raises if it has not been built: there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(ctx, rc):
    if rc != LB_OK:
        msg = lib().lb_last_error(ctx)
        raise LbError(rc, msg.decode() if msg else "")


def _host(a, n=None, writable=False):
    """float64 C-contiguous numpy array -> void*, or None."""
    if a is None:
        return None
    if not (isinstance(a, np.ndarray) and a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]):
        raise TypeError("host arrays must be C-contiguous float64 numpy arrays")
    if writable and not a.flags["WRITEABLE"]:
        raise TypeError("output array is read-only")
    if n is not None and a.size < n:
        raise ValueError(f"array of {a.size} elements, {n} required")
    return a.ctypes.data


# ---------------------------------------------------------------------------
# wrappers (same names as the C functions)
# ---------------------------------------------------------------------------

def lb_config_default(**overrides):
    """A filled lb_config; keyword arguments override fields (bc as a 3-sequence)."""
    c = lb_config()
    lib().lb_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        if k == "bc":
            for i in range(3):
                c.bc[i] = v[i] if i < len(v) else LB_PERIODIC
        else:
            setattr(c, k, v)
    return c


def lb_validate_config(cfg):
    buf = ctypes.create_string_buffer(256)
    rc = lib().lb_validate_config(ctypes.byref(cfg), buf, 256)
    return rc, buf.value.decode()


def lb_required_bytes(cfg):
    return int(lib().lb_required_bytes(ctypes.byref(cfg)))


def lb_create(cfg):
    h = ctypes.c_void_p()
    rc = lib().lb_create(ctypes.byref(h), ctypes.byref(cfg))
    if rc != LB_OK:
        raise LbError(rc, lib().lb_last_error(None).decode())
    return h.value


def lb_destroy(ctx):
    lib().lb_destroy(ctx)


def lb_last_error(ctx):
    m = lib().lb_last_error(ctx)
    return m.decode() if m else ""


def lb_bind_buffers(ctx, buf_a: int, buf_b: int, bytes_each: int):
    _check(ctx, lib().lb_bind_buffers(ctx, buf_a, buf_b, bytes_each))


def lb_init_equilibrium(ctx, rho=None, u=None, phi=None):
    _check(ctx, lib().lb_init_equilibrium(ctx, _host(rho), _host(u), _host(phi)))


def lb_init_equilibrium_device(ctx, rho=None, u=None, phi=None):
    """Device pointers (integers) or None; asynchronous on the context's stream."""
    _check(ctx, lib().lb_init_equilibrium_device(ctx, rho, u, phi))


def lb_reset_moments_device(ctx, rho, u, phi=None):
    """Device pointers (integers); asynchronous on the context's stream."""
    _check(ctx, lib().lb_reset_moments_device(ctx, rho, u, phi))


def lb_set_force_uniform(ctx, fx, fy, fz=0.0):
    _check(ctx, lib().lb_set_force_uniform(ctx, float(fx), float(fy), float(fz)))


def lb_set_force_field(ctx, F, dtype=LB_DTYPE_F64, mem=LB_MEM_HOST):
    """F: numpy [dims][N] (host), an integer device pointer (mem=LB_MEM_DEVICE), or None."""
    if F is None:
        ptr = None
    elif mem == LB_MEM_DEVICE:
        ptr = int(F)
    else:
        want = np.float64 if dtype == LB_DTYPE_F64 else np.float32
        if not (isinstance(F, np.ndarray) and F.dtype == want and F.flags["C_CONTIGUOUS"]):
            raise TypeError("host field must be a C-contiguous array of the given dtype")
        ptr = F.ctypes.data
    _check(ctx, lib().lb_set_force_field(ctx, ptr, dtype, mem))


def lb_set_force_time(ctx, mode, omega=0.0):
    _check(ctx, lib().lb_set_force_time(ctx, mode, float(omega)))


def lb_set_source_uniform(ctx, s):
    _check(ctx, lib().lb_set_source_uniform(ctx, float(s)))


def lb_set_source_field(ctx, S, dtype=LB_DTYPE_F64, mem=LB_MEM_HOST):
    if S is None:
        ptr = None
    elif mem == LB_MEM_DEVICE:
        ptr = int(S)
    else:
        want = np.float64 if dtype == LB_DTYPE_F64 else np.float32
        if not (isinstance(S, np.ndarray) and S.dtype == want and S.flags["C_CONTIGUOUS"]):
            raise TypeError("host field must be a C-contiguous array of the given dtype")
        ptr = S.ctypes.data
    _check(ctx, lib().lb_set_source_field(ctx, ptr, dtype, mem))


def lb_set_source_time(ctx, mode, omega=0.0):
    _check(ctx, lib().lb_set_source_time(ctx, mode, float(omega)))


def lb_step(ctx, nsteps):
    _check(ctx, lib().lb_step(ctx, int(nsteps)))


def lb_synchronize(ctx):
    _check(ctx, lib().lb_synchronize(ctx))


def lb_get_step(ctx):
    return int(lib().lb_get_step(ctx))


def lb_set_step(ctx, n):
    _check(ctx, lib().lb_set_step(ctx, int(n)))


def lb_read_moments(ctx, kind, rho, u, phi=None):
    _check(ctx, lib().lb_read_moments(ctx, kind, _host(rho, writable=True), _host(u, writable=True),
                                      _host(phi, writable=True)))


def lb_read_moments_device(ctx, kind, rho=None, u=None, phi=None):
    """Device pointers (integers) or None; asynchronous on the context's stream."""
    _check(ctx, lib().lb_read_moments_device(ctx, kind, rho, u, phi))


def lb_read_populations(ctx, f, g=None):
    _check(ctx, lib().lb_read_populations(ctx, _host(f, writable=True), _host(g, writable=True)))


def lb_write_populations(ctx, f, g=None):
    _check(ctx, lib().lb_write_populations(ctx, _host(f), _host(g)))


def lb_read_populations_box(ctx, lo, ext, f, g=None):
    lo_a = (ctypes.c_int64 * 3)(*[int(v) for v in lo])
    ext_a = (ctypes.c_int64 * 3)(*[int(v) for v in ext])
    _check(ctx, lib().lb_read_populations_box(ctx, lo_a, ext_a, _host(f, writable=True), _host(g, writable=True)))


def lb_totals(ctx):
    out = (ctypes.c_double * 5)()
    _check(ctx, lib().lb_totals(ctx, out))
    return np.array(out[:])


def lb_totals_noalloc(ctx, out_device: int):
    """Enqueues the totals into 5 doubles of device memory at out_device (no allocation)."""
    _check(ctx, lib().lb_totals_noalloc(ctx, out_device))


def lb_set_lorentz(ctx, s):
    _check(ctx, lib().lb_set_lorentz(ctx, float(s)))


def lb_residual(ctx):
    """(r, at_step, totals[5]); raises LbError(LB_ENONFINITE) if the check found NaN/inf."""
    r = ctypes.c_double()
    at = ctypes.c_int64()
    tot = (ctypes.c_double * 5)()
    _check(ctx, lib().lb_residual(ctx, ctypes.byref(r), ctypes.byref(at), tot))
    return r.value, at.value, np.array(tot[:])


def lb_set_wall_velocity(ctx, axis, side, ux, uy, uz=0.0):
    _check(ctx, lib().lb_set_wall_velocity(ctx, int(axis), int(side), float(ux), float(uy), float(uz)))


def lb_set_scalar_wall(ctx, axis, side, fixed, value=0.0):
    _check(ctx, lib().lb_set_scalar_wall(ctx, int(axis), int(side), int(bool(fixed)), float(value)))


def lb_set_viscous_heating(ctx, coefficient):
    _check(ctx, lib().lb_set_viscous_heating(ctx, float(coefficient)))


def lb_residual_scalar(ctx):
    """Scalar residual of the latest check (coupled lattice only)."""
    r = ctypes.c_double()
    _check(ctx, lib().lb_residual_scalar(ctx, ctypes.byref(r)))
    return r.value


def lb_get_info(ctx):
    info = lb_info()
    _check(ctx, lib().lb_get_info(ctx, ctypes.byref(info)))
    return info


def lb_stream_copy(dst: int, src: int, nbytes: int, stream: int = 0):
    rc = lib().lb_stream_copy(dst, src, nbytes, stream)
    if rc != LB_OK:
        raise LbError(rc, "lb_stream_copy failed")


def lb_stream_bench(dst: int, src: int, nbytes: int, mode: int, width: int = 16, blocks: int = 0, stream: int = 0):
    """mode 0 copy, 1 read-only, 2 write-only (HBM ceiling measurement)."""
    rc = lib().lb_stream_bench(dst, src, nbytes, mode, width, blocks, stream)
    if rc != LB_OK:
        raise LbError(rc, "lb_stream_bench failed")


# ---------------------------------------------------------------------------
# batched independent channels
# ---------------------------------------------------------------------------

def _bcheck(b, rc):
    if rc != LB_OK:
        msg = lib().lb_batch_last_error(b)
        raise LbError(rc, msg.decode() if msg else "")


def lb_batch_config_default(**overrides):
    c = lb_batch_config()
    lib().lb_batch_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        setattr(c, k, v)
    return c


def lb_batch_create(cfg, domains):
    """domains: sequence of (nx, ny, nu, force_x, lorentz)."""
    arr = (lb_batch_domain * len(domains))(*[lb_batch_domain(int(d[0]), int(d[1]), float(d[2]), float(d[3]),
                                                             float(d[4])) for d in domains])
    h = ctypes.c_void_p()
    rc = lib().lb_batch_create(ctypes.byref(h), ctypes.byref(cfg), arr, len(domains))
    if rc != LB_OK:
        raise LbError(rc, lib().lb_batch_last_error(None).decode())
    return h.value


def lb_batch_destroy(b):
    lib().lb_batch_destroy(b)


def lb_batch_last_error(b):
    m = lib().lb_batch_last_error(b)
    return m.decode() if m else ""


def lb_batch_init(b):
    _bcheck(b, lib().lb_batch_init(b))


def lb_batch_run(b, max_steps, tol):
    _bcheck(b, lib().lb_batch_run(b, int(max_steps), float(tol)))


def lb_batch_results(b, ndomains):
    steps = np.zeros(ndomains, dtype=np.int64)
    res = np.zeros(ndomains)
    status = np.zeros(ndomains, dtype=np.int32)
    _bcheck(b, lib().lb_batch_results(b, steps.ctypes.data, res.ctypes.data, status.ctypes.data))
    return steps, res, status


def lb_batch_read_moments(b, domain, rho, u):
    _bcheck(b, lib().lb_batch_read_moments(b, int(domain), _host(rho, writable=True), _host(u, writable=True)))


def lb_batch_read_populations(b, domain, f):
    _bcheck(b, lib().lb_batch_read_populations(b, int(domain), _host(f, writable=True)))


def lb_batch_write_populations(b, domain, f):
    _bcheck(b, lib().lb_batch_write_populations(b, int(domain), _host(f)))


def lb_batch_autotune(b, sample_steps):
    blk = ctypes.c_int32()
    pol = ctypes.c_int32()
    ms = ctypes.c_double()
    _bcheck(b, lib().lb_batch_autotune(b, int(sample_steps), ctypes.byref(blk), ctypes.byref(pol), ctypes.byref(ms)))
    return blk.value, pol.value, ms.value


# ---------------------------------------------------------------------------
# warm-start surrogate network (include/casclb_unet.h)
# ---------------------------------------------------------------------------

def _ucheck(net, rc):
    if rc != LB_OK:
        msg = lib().lb_unet_last_error(net)
        raise LbError(rc, msg.decode() if msg else "")


def lb_unet_config_default(**overrides):
    c = lb_unet_config()
    lib().lb_unet_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        if k == "channels":
            for i, ch in enumerate(v):
                c.channels[i] = int(ch)
        else:
            setattr(c, k, v)
    return c


def lb_unet_create(cfg):
    h = _P()
    _ucheck(None, lib().lb_unet_create(ctypes.byref(h), ctypes.byref(cfg)))
    return h.value


def lb_unet_destroy(net):
    lib().lb_unet_destroy(net)


def lb_unet_last_error(net):
    m = lib().lb_unet_last_error(net)
    return m.decode() if m else ""


def lb_unet_num_params(net):
    return int(lib().lb_unet_num_params(net))


def lb_unet_set_params(net, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == lb_unet_num_params(net)
    _ucheck(net, lib().lb_unet_set_params(net, p.ctypes.data))


def lb_unet_get_params(net):
    p = np.empty(lb_unet_num_params(net), dtype=np.float32)
    _ucheck(net, lib().lb_unet_get_params(net, p.ctypes.data))
    return p


def lb_unet_forward(net, x_dev: int, batch: int, y_dev: int):
    """Device pointers (float32 NHWC) x [batch][H][W][in], y [batch][H][W][out]."""
    _ucheck(net, lib().lb_unet_forward(net, x_dev, int(batch), y_dev))


def lb_unet_loss_grad(net, x_dev: int, t_dev: int, batch: int, want_grad=True):
    """(loss, flat float32 gradient or None)."""
    loss = ctypes.c_double()
    g = np.empty(lb_unet_num_params(net), dtype=np.float32) if want_grad else None
    _ucheck(net, lib().lb_unet_loss_grad(net, x_dev, t_dev, int(batch), ctypes.byref(loss),
                                         g.ctypes.data if want_grad else None))
    return loss.value, g


def lb_unet_adam(net, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _ucheck(net, lib().lb_unet_adam(net, float(lr), float(beta1), float(beta2), float(eps)))


def lb_unet_train_step(net, x_dev: int, t_dev: int, batch: int, lr: float, want_loss=True):
    loss = ctypes.c_double()
    _ucheck(net, lib().lb_unet_train_step(net, x_dev, t_dev, int(batch), float(lr),
                                          ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def lb_unet_macs_per_image(net):
    return float(lib().lb_unet_macs_per_image(net))


def lb_unet_set_lowpass_loss(net, levels, weight):
    _ucheck(net, lib().lb_unet_set_lowpass_loss(net, int(levels), float(weight)))


# ---------------------------------------------------------------------------
# warm-start field operations (include/casclb_warm.h); device pointers are ints
# ---------------------------------------------------------------------------

def _wcheck(rc, name):
    if rc != LB_OK:
        raise LbError(rc, f"{name}: invalid arguments" if rc == LB_EINVAL else f"{name}: HIP error")


def lb_warm_restrict(src, planes, L, scale, dst, stream=None):
    _wcheck(lib().lb_warm_restrict(src, int(planes), int(L), float(scale), dst, stream), "lb_warm_restrict")


def lb_warm_prolong(src, planes, Lc, scale, dst, stream=None):
    _wcheck(lib().lb_warm_prolong(src, int(planes), int(Lc), float(scale), dst, stream), "lb_warm_prolong")


def lb_warm_axpby(n, a, x, b, y, out, stream=None):
    _wcheck(lib().lb_warm_axpby(int(n), float(a), x, float(b), y, out, stream), "lb_warm_axpby")


def lb_warm_project(data, planes, L, k2max=0, stream=None):
    _wcheck(lib().lb_warm_project(data, int(planes), int(L), int(k2max), stream), "lb_warm_project")


def _channels(chs):
    arr = (lb_warm_channel * len(chs))()
    for i, c in enumerate(chs):
        arr[i] = lb_warm_channel(c.get("src"), c.get("dst"), float(c.get("scale", 1.0)), float(c.get("offset", 0.0)))
    return arr


def lb_warm_pack(channels, batch, n, out, stream=None):
    """channels: list of dicts with src (device pointer or None), scale, offset."""
    arr = _channels(channels)
    _wcheck(lib().lb_warm_pack(arr, len(channels), int(batch), int(n), out, stream), "lb_warm_pack")


def lb_warm_unpack(y, channels, batch, n, stream=None):
    """channels: list of dicts with src, dst (device pointers) and scale."""
    arr = _channels(channels)
    _wcheck(lib().lb_warm_unpack(y, arr, len(channels), int(batch), int(n), stream), "lb_warm_unpack")


def lb_warm_initial_state(drho, u, phi, F, S, batch, n, rho0, zero_momentum, rho_out, u_out, phi_out, stream=None):
    _wcheck(lib().lb_warm_initial_state(drho, u, phi, F, S, int(batch), int(n), float(rho0), int(bool(zero_momentum)),
                                        rho_out, u_out, phi_out, stream), "lb_warm_initial_state")
