"""ctypes binding of libefm.so: the C-ABI functions under the same names.

Argument marshalling only -- every step of the computation runs in the HIP
library.  Device arrays may be passed as torch tensors (their data_ptr() is
used; torch is only the allocator) or as integer device addresses.  Streams
default to torch's current stream on the current device.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libefm.so")

EC_OK = 0
EC_ERR_ARG, EC_ERR_DEVICE, EC_ERR_OOM, EC_ERR_UNSUPPORTED, EC_ERR_DOMAIN = -1, -2, -3, -4, -5
EC_KERNEL_MAXWELL, EC_KERNEL_HARD_SPHERE, EC_KERNEL_VHS = 0, 1, 2
EC_TRUNC_BOX, EC_TRUNC_BALL = 0, 1
EC_FP64, EC_FP32, EC_BF16X3 = 0, 1, 2
EC_NMON = 11
EC_SCHED_PIPELINE, EC_SCHED_TWO_PASS, EC_SCHED_FUSED, EC_SCHED_LINES, EC_SCHED_TERMS = 0, 1, 2, 3, 4
EC_PROF_KERNELS = 6
EC_TUNE_REMEASURE = 1
PROF_KERNEL_NAMES = ["k_fwd", "k_pencil", "k_slab", "k_pipe", "reserved", "k_fused"]
MON_NAMES = ["mass", "sumQ", "entropy_prod", "eta", "minF", "eps_pos", "sumabsQ",
             "momQ_x", "momQ_y", "momQ_z", "energyQ"]

_c_int, _c_double, _c_i64, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_int64, ctypes.c_void_p


class EcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"EC error {code}: {msg}")
        self.code = code


class ec_kernel(ctypes.Structure):
    _fields_ = [("kind", _c_int), ("gamma", _c_double), ("R", _c_double), ("n_radial", _c_int),
                ("unfiltered", _c_int), ("truncation", _c_int), ("n_bcos", _c_int),
                ("bcos", _c_double * 8)]


_SIGS = {
    "ec_last_error": ([], ctypes.c_char_p),
    "ec_setup_kernel": ([_c_int, _c_int, _c_double, ctypes.POINTER(ec_kernel), _c_int,
                         ctypes.POINTER(_vp)], _c_int),
    "ec_plan_destroy": ([_vp], _c_int),
    "ec_plan_terms": ([_vp, ctypes.POINTER(_c_int)], _c_int),
    "ec_plan_tables": ([_vp, ctypes.POINTER(_c_double)], _c_int),
    "ec_host_tables": ([_c_int, _c_int, _c_double, ctypes.POINTER(ec_kernel), _c_int,
                        ctypes.POINTER(_c_int), ctypes.POINTER(_c_double)], _c_int),
    "ec_host_table_modes": ([_c_int, _c_int, _c_double, ctypes.POINTER(ec_kernel), _c_int, _c_i64,
                             ctypes.POINTER(_c_i64), ctypes.POINTER(_c_int),
                             ctypes.POINTER(_c_double)], _c_int),
    "ec_batch_create": ([ctypes.POINTER(_vp), ctypes.POINTER(_c_i64), _c_int, _c_int,
                         ctypes.POINTER(_vp)], _c_int),
    "ec_batch_destroy": ([_vp], _c_int),
    "ec_batch_size": ([_vp, ctypes.POINTER(_c_i64), ctypes.POINTER(_c_i64)], _c_int),
    "ec_batch_offsets": ([_vp, ctypes.POINTER(_c_i64)], _c_int),
    "ec_batch_set_chunk": ([_vp, _c_int, _c_int], _c_int),
    "ec_collide": ([_vp, _vp, _vp, _vp], _c_int),
    "ec_collide_noalloc": ([_vp, _c_int, _c_i64, _vp, _vp, _vp], _c_int),
    "ec_entropy_prod": ([_vp, _vp, _vp, _vp, _vp, _vp], _c_int),
    "ec_monitors": ([_vp, _vp, _vp, _vp, _vp], _c_int),
    "ec_step": ([_vp, _vp, _c_double, _c_int, _vp, _vp], _c_int),
    "ec_step_graph": ([_vp, _vp, _c_double, _c_int, _vp, _vp], _c_int),
    "ec_step_ssprk3": ([_vp, _vp, _c_double, _c_int, _vp, _vp], _c_int),
    "ec_batch_set_schedule": ([_vp, _c_int, _c_int, _c_int, _c_int], _c_int),
    "ec_batch_get_schedule": ([_vp, _c_int, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int),
                               ctypes.POINTER(_c_int)], _c_int),
    "ec_copy": ([_vp, _vp, _c_i64, _vp], _c_int),
    "ec_valu_probe": ([_c_int, ctypes.POINTER(_c_double), _vp], _c_int),
    "ec_autotune": ([_vp, _vp, _vp, ctypes.c_char_p, _c_int, _vp], _c_int),
    "ec_surrogate_create": ([_c_int, _c_int, _c_int, _c_int, ctypes.c_uint64, _c_int,
                             ctypes.POINTER(_vp)], _c_int),
    "ec_surrogate_destroy": ([_vp], _c_int),
    "ec_surrogate_num_params": ([_vp, ctypes.POINTER(_c_i64)], _c_int),
    "ec_surrogate_get_params": ([_vp, _vp], _c_int),
    "ec_surrogate_set_params": ([_vp, _vp], _c_int),
    "ec_surrogate_get_grads": ([_vp, _vp], _c_int),
    "ec_surrogate_prepare": ([_vp, _vp, _vp, _vp, _c_i64, _c_int, _vp, _vp, _vp], _c_int),
    "ec_surrogate_forward": ([_vp, _vp, _vp, _c_int, _vp], _c_int),
    "ec_surrogate_train_step": ([_vp, _vp, _vp, _c_int, ctypes.c_float, _c_int,
                                 ctypes.POINTER(_c_double), _vp], _c_int),
    "ec_surrogate_train": ([_vp, _vp, _vp, _c_int, ctypes.c_float, _c_int,
                            ctypes.POINTER(_c_double), _vp], _c_int),
    "ec_surrogate_collide": ([_vp, _vp, _vp, _vp, _c_double, _c_double, _vp, _vp,
                              ctypes.POINTER(_c_i64), _vp], _c_int),
    "ec_profile": ([_vp, _c_int], _c_int),
    "ec_profile_read": ([_vp, ctypes.POINTER(_c_double), ctypes.POINTER(_c_i64),
                         ctypes.POINTER(_c_i64)], _c_int),
}

_lib = None


def lib():
    """Load libefm.so; raise if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1704_07369_amd.build`")
        # torch ships its own HIP runtime with the same soname
        # (libamdhip64.so.7).  Loading torch first makes the dynamic loader
        # reuse that copy for libefm.so, so one HIP runtime serves both the
        # allocator/streams and the kernels of this library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS.keys())


def _check(rc):
    if rc != EC_OK:
        raise EcError(rc, lib().ec_last_error().decode())
    return rc


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError(f"cannot take a device address of {type(x)}")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


EC_MAX_BCOS = 8


def make_kernel(kind=EC_KERNEL_HARD_SPHERE, gamma=1.0, R=6.0, n_radial=0, unfiltered=False,
                truncation=0, bcos=None):
    """bcos: coefficients of b(cos theta) = sum_i bcos[i] cos^i theta (None: b = 1)."""
    bc = list(bcos or [])
    if len(bc) > EC_MAX_BCOS:
        raise ValueError(f"at most {EC_MAX_BCOS} coefficients of b(cos theta)")
    arr = (_c_double * 8)(*(bc + [0.0] * (8 - len(bc))))
    return ec_kernel(kind, gamma, R, n_radial, 1 if unfiltered else 0, truncation, len(bc), arr)


# ---- same-name wrappers -----------------------------------------------------

def ec_last_error():
    return lib().ec_last_error().decode()


def ec_setup_kernel(N, d, L, kernel, M):
    h = _vp()
    _check(lib().ec_setup_kernel(N, d, L, ctypes.byref(kernel), M, ctypes.byref(h)))
    return h.value


def ec_plan_destroy(plan):
    return _check(lib().ec_plan_destroy(plan))


def ec_plan_terms(plan):
    t = _c_int()
    _check(lib().ec_plan_terms(plan, ctypes.byref(t)))
    return t.value


def ec_plan_tables(plan, n_points):
    J = ec_plan_terms(plan) + 1
    out = np.empty(2 * J * n_points)
    _check(lib().ec_plan_tables(plan, out.ctypes.data_as(ctypes.POINTER(_c_double))))
    return (out[0::2] + 1j * out[1::2]).reshape(J, n_points)


def ec_host_tables(N, d, L, kernel, M):
    t = _c_int()
    _check(lib().ec_host_tables(N, d, L, ctypes.byref(kernel), M, ctypes.byref(t), None))
    n = N ** d
    out = np.empty(2 * (t.value + 1) * n)
    _check(lib().ec_host_tables(N, d, L, ctypes.byref(kernel), M, ctypes.byref(t),
                                out.ctypes.data_as(ctypes.POINTER(_c_double))))
    return (out[0::2] + 1j * out[1::2]).reshape(t.value + 1, n)


def ec_host_table_modes(N, d, L, kernel, M, modes):
    """Table entries [M'+1][len(modes)] at flat mode indices of the table
    layout (ec_plan_tables)."""
    idx = np.ascontiguousarray(modes, dtype=np.int64)
    t = _c_int()
    _check(lib().ec_host_table_modes(N, d, L, ctypes.byref(kernel), M, 0, None, ctypes.byref(t),
                                     None))
    out = np.empty(2 * (t.value + 1) * idx.size)
    _check(lib().ec_host_table_modes(N, d, L, ctypes.byref(kernel), M, idx.size,
                                     idx.ctypes.data_as(ctypes.POINTER(_c_i64)), ctypes.byref(t),
                                     out.ctypes.data_as(ctypes.POINTER(_c_double))))
    return (out[0::2] + 1j * out[1::2]).reshape(t.value + 1, idx.size)


def ec_batch_create(plans, counts, precision=EC_FP64):
    n = len(plans)
    pa = (_vp * n)(*plans)
    ca = (_c_i64 * n)(*counts)
    h = _vp()
    _check(lib().ec_batch_create(pa, ca, n, precision, ctypes.byref(h)))
    return h.value


def ec_batch_destroy(batch):
    return _check(lib().ec_batch_destroy(batch))


def ec_batch_size(batch):
    c, e = _c_i64(), _c_i64()
    _check(lib().ec_batch_size(batch, ctypes.byref(c), ctypes.byref(e)))
    return c.value, e.value


def ec_batch_offsets(batch):
    n, _ = ec_batch_size(batch)
    out = np.empty(n, dtype=np.int64)
    _check(lib().ec_batch_offsets(batch, out.ctypes.data_as(ctypes.POINTER(_c_i64))))
    return out


def ec_batch_set_chunk(batch, group, cells_per_pass):
    return _check(lib().ec_batch_set_chunk(batch, group, cells_per_pass))


def ec_collide(batch, f, Q, stream=None):
    return _check(lib().ec_collide(batch, _ptr(f), _ptr(Q), _stream(stream)))


def ec_collide_noalloc(plan, precision, n_cells, f, Q, stream=None):
    return _check(lib().ec_collide_noalloc(plan, precision, n_cells, _ptr(f), _ptr(Q),
                                           _stream(stream)))


def ec_entropy_prod(batch, f, Q, out, n_nonpos=None, stream=None):
    return _check(lib().ec_entropy_prod(batch, _ptr(f), _ptr(Q), _ptr(out), _ptr(n_nonpos),
                                        _stream(stream)))


def ec_monitors(batch, f, Q, out, stream=None):
    return _check(lib().ec_monitors(batch, _ptr(f), _ptr(Q), _ptr(out), _stream(stream)))


def ec_step_graph(batch, f, dt, n_steps, monitors=None, stream=None):
    return _check(lib().ec_step_graph(batch, _ptr(f), dt, n_steps, _ptr(monitors),
                                      _stream(stream)))


def ec_step(batch, f, dt, n_steps, monitors=None, stream=None):
    return _check(lib().ec_step(batch, _ptr(f), dt, n_steps, _ptr(monitors), _stream(stream)))


def ec_step_ssprk3(batch, f, dt, n_steps, monitors=None, stream=None):
    return _check(lib().ec_step_ssprk3(batch, _ptr(f), dt, n_steps, _ptr(monitors),
                                       _stream(stream)))


def ec_profile(batch, enable=True):
    return _check(lib().ec_profile(batch, 1 if enable else 0))


def ec_batch_set_schedule(batch, group, mode, cells_per_pass=0, term_groups=0):
    return _check(lib().ec_batch_set_schedule(batch, group, mode, cells_per_pass, term_groups))


def ec_batch_get_schedule(batch, group):
    m, c, g = _c_int(), _c_int(), _c_int()
    _check(lib().ec_batch_get_schedule(batch, group, ctypes.byref(m), ctypes.byref(c),
                                       ctypes.byref(g)))
    return m.value, c.value, g.value


def ec_profile_read(batch, n_groups):
    ms = np.zeros(EC_PROF_KERNELS * n_groups)
    la = np.zeros(EC_PROF_KERNELS * n_groups, dtype=np.int64)
    ce = np.zeros(n_groups, dtype=np.int64)
    _check(lib().ec_profile_read(batch, ms.ctypes.data_as(ctypes.POINTER(_c_double)),
                                 la.ctypes.data_as(ctypes.POINTER(_c_i64)),
                                 ce.ctypes.data_as(ctypes.POINTER(_c_i64))))
    return ms.reshape(n_groups, EC_PROF_KERNELS), la.reshape(n_groups, EC_PROF_KERNELS), ce


def ec_copy(src, dst, n, stream=None):
    return _check(lib().ec_copy(_ptr(src), _ptr(dst), n, _stream(stream)))


def ec_valu_probe(precision=EC_FP64, stream=None):
    t = _c_double()
    _check(lib().ec_valu_probe(precision, ctypes.byref(t), _stream(stream)))
    return t.value


def ec_autotune(batch, f, Q, cache_path=None, flags=0, stream=None):
    cp = cache_path.encode() if cache_path else None
    return _check(lib().ec_autotune(batch, _ptr(f), _ptr(Q), cp, flags, _stream(stream)))


def ec_surrogate_create(N, modes, channels, layers, seed, max_batch):
    h = _vp()
    _check(lib().ec_surrogate_create(N, modes, channels, layers, seed, max_batch, ctypes.byref(h)))
    return h.value


def ec_surrogate_destroy(s):
    return _check(lib().ec_surrogate_destroy(s))


def ec_surrogate_num_params(s):
    n = _c_i64()
    _check(lib().ec_surrogate_num_params(s, ctypes.byref(n)))
    return n.value


def ec_surrogate_get_params(s):
    out = np.empty(ec_surrogate_num_params(s), dtype=np.float32)
    _check(lib().ec_surrogate_get_params(s, out.ctypes.data))
    return out


def ec_surrogate_set_params(s, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == ec_surrogate_num_params(s)
    return _check(lib().ec_surrogate_set_params(s, p.ctypes.data))


def ec_surrogate_get_grads(s):
    out = np.empty(ec_surrogate_num_params(s), dtype=np.float32)
    _check(lib().ec_surrogate_get_grads(s, out.ctypes.data))
    return out


def ec_surrogate_prepare(s, batch, f, Q, cell0, B, Fin, target, stream=None):
    return _check(lib().ec_surrogate_prepare(s, batch, _ptr(f), _ptr(Q), cell0, B, _ptr(Fin),
                                             _ptr(target), _stream(stream)))


def ec_surrogate_forward(s, Fin, y, B, stream=None):
    return _check(lib().ec_surrogate_forward(s, _ptr(Fin), _ptr(y), B, _stream(stream)))


def ec_surrogate_train(s, Fin, target, B, lr, update=True, want_loss=True, stream=None):
    loss = _c_double(float("nan"))
    _check(lib().ec_surrogate_train(s, _ptr(Fin), _ptr(target), B, lr, 1 if update else 0,
                                    ctypes.byref(loss) if want_loss else None, _stream(stream)))
    return loss.value


def ec_surrogate_train_step(s, Fin, target, B, lr, update=True, want_loss=True, stream=None):
    loss = _c_double(float("nan"))
    _check(lib().ec_surrogate_train_step(s, _ptr(Fin), _ptr(target), B, lr, 1 if update else 0,
                                         ctypes.byref(loss) if want_loss else None,
                                         _stream(stream)))
    return loss.value


def ec_surrogate_collide(s, batch, f, Q, tau_m, tau_e, fell_back=None, screen=None, stream=None):
    nf = _c_i64()
    _check(lib().ec_surrogate_collide(s, batch, _ptr(f), _ptr(Q), tau_m, tau_e, _ptr(fell_back),
                                      _ptr(screen), ctypes.byref(nf), _stream(stream)))
    return nf.value
