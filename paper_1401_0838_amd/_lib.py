"""ctypes binding of libpic.so: the C ABI of include/pic_api.h, same names.

Argument marshalling only.  The library must have been built in-tree
(paper_1401_0838_amd/build.py); loading fails loudly otherwise -- there is no
fallback implementation.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK = 0
PIC_EINVAL = -1
PIC_ECOURANT = -2
PIC_EPSI = -3
PIC_ENOMEM = -4
PIC_EHIP = -5
PIC_ENONFINITE = -6
PIC_EPARTICLE = -7
PIC_EUNSUPPORTED = -8
PIC_ESTATE = -9
PIC_ERANGE = -10

PIC_GALERKIN, PIC_UNIFORM, PIC_MOMENTUM = 0, 1, 2
PIC_YEE, PIC_CK = 0, 1
PIC_CORR_NONE, PIC_CORR_SPLIT, PIC_CORR_RATIO = 0, 1, 2
PIC_FP64, PIC_FP32 = 0, 1
PIC_IONS_CHARGE, PIC_IONS_CHARGE_AND_CURRENT = 0, 1
PIC_FIELD_E, PIC_FIELD_B, PIC_FIELD_J, PIC_FIELD_SEEN_E, PIC_FIELD_SEEN_B, PIC_FIELD_RHO = range(6)
PIC_GET, PIC_SET = 0, 1
PIC_SCHED_BATCHED, PIC_SCHED_PLAIN = 0, 1

_D = C.POINTER(C.c_double)


class pic_config(C.Structure):
    _fields_ = [("dims", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double), ("cdt", C.c_double),
                ("shape_order", C.c_int), ("interp", C.c_int), ("precision", C.c_int),
                ("correction", C.c_int), ("psi_deg", C.c_int),
                ("psi_e", C.c_double * 9), ("psi_b", C.c_double * 9),
                ("filter_npass", C.c_int), ("filter_w", C.c_double * 8),
                ("q", C.c_double), ("m", C.c_double), ("weight", C.c_double),
                ("ion_mode", C.c_int), ("tile", C.c_int * 3), ("block", C.c_int),
                ("trace_capacity", C.c_int), ("adjoint_steps", C.c_int), ("adjoint_ckpt", C.c_int),
                ("solver", C.c_int)]


class pic_particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", _D * 3), ("mom", _D * 3)]


class pic_diag_t(C.Structure):
    _fields_ = [("WE", C.c_double * 3), ("WB", C.c_double * 3), ("Wkin", C.c_double),
                ("gauss_l2", C.c_double), ("gauss_linf", C.c_double), ("charge", C.c_double),
                ("rho_max", C.c_double), ("n_particles", C.c_int64), ("step", C.c_int64),
                ("nonfinite", C.c_int), ("particle_error", C.c_int), ("resorts", C.c_int),
                ("slow_tiles", C.c_int), ("current_range", C.c_int)]


class pic_timing_t(C.Structure):
    _fields_ = [("yee_ms", C.c_double), ("seen_ms", C.c_double), ("particle_ms", C.c_double),
                ("resort_ms", C.c_double), ("step_ms", C.c_double), ("steps", C.c_int)]


class PicError(RuntimeError):
    def __init__(self, code, where, detail=""):
        super().__init__("%s failed: %s (%d) %s" % (where, strerror(code), code, detail))
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "pic_psi_coeffs": (C.c_int, [C.c_int, C.c_double, C.c_int, _D, _D]),
    "pic_plan": (C.c_int, [C.POINTER(pic_config), C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]),
    "pic_init": (C.c_int, [C.POINTER(pic_config), C.c_int, C.POINTER(pic_particles), C.c_void_p,
                           C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "pic_init_static": (C.c_int, [C.POINTER(pic_config), C.c_int, C.POINTER(pic_particles), C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "pic_step": (C.c_int, [C.c_void_p, C.c_int]),
    "pic_prepare": (C.c_int, [C.c_void_p, C.c_int]),
    "pic_set_option": (C.c_int, [C.c_void_p, C.c_char_p, C.c_int]),
    "pic_get_option": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_int)]),
    "pic_set_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "pic_fields": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, _D, C.c_size_t, C.c_int]),
    "pic_get_particles": (C.c_int, [C.c_void_p, C.c_int, _D * 3, _D * 3, C.c_int64]),
    "pic_diag": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(pic_diag_t)]),
    "pic_read_trace": (C.c_int, [C.c_void_p, C.c_int, _D, C.c_int, C.POINTER(C.c_int)]),
    "pic_profile": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(pic_timing_t)]),
    "pic_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "pic_adjoint_forward": (C.c_int, [C.c_void_p, C.c_int, _D]),
    "pic_adjoint_backward": (C.c_int, [C.c_void_p, _D]),
    "pic_destroy": (None, [C.c_void_p]),
    "pic_strerror": (C.c_char_p, [C.c_int]),
    "pic_last_error": (C.c_char_p, []),
}

EXPORTED = tuple(_SIGS)


def load():
    """Load libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libpic.so not built: run paper_1401_0838_amd/build.py (%s)" % LIB_PATH)
        # torch first: libpic.so must bind to the HIP runtime torch brings into the
        # process.  Loaded before torch, it would pull in a second HIP runtime
        # that sees no device once torch has initialised its own.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def strerror(code):
    return load().pic_strerror(code).decode()


def last_error():
    return load().pic_last_error().decode()


def check(code, where):
    if code != PIC_OK:
        raise PicError(code, where, last_error())
    return code


def dptr(arr):
    """float64 numpy array -> double*."""
    import numpy as np
    assert arr.dtype == np.float64 and arr.flags.c_contiguous
    return arr.ctypes.data_as(_D)


# thin same-name wrappers --------------------------------------------------

def pic_psi_coeffs(interp, alpha, deg=4):
    import numpy as np
    a = np.zeros(deg + 1)
    b = np.zeros(deg + 1)
    rc = load().pic_psi_coeffs(int(interp), float(alpha), int(deg), dptr(a), dptr(b))
    return rc, a, b


def pic_plan(cfgs, n_particles):
    n = len(cfgs)
    arr = (pic_config * n)(*cfgs)
    nps = (C.c_int64 * n)(*[int(v) for v in n_particles])
    out = C.c_size_t(0)
    check(load().pic_plan(arr, n, nps, C.byref(out)), "pic_plan")
    return out.value


def pic_init(cfgs, parts, arena_ptr, arena_bytes, stream_ptr):
    n = len(cfgs)
    arr = (pic_config * n)(*cfgs)
    parr = (pic_particles * n)(*parts)
    st = C.c_void_p(0)
    check(load().pic_init(arr, n, parr, C.c_void_p(arena_ptr), C.c_size_t(arena_bytes),
                          C.c_void_p(stream_ptr), C.byref(st)), "pic_init")
    return st


def pic_init_static(cfgs, parts, stream_ptr):
    n = len(cfgs)
    arr = (pic_config * n)(*cfgs)
    parr = (pic_particles * n)(*parts)
    st = C.c_void_p(0)
    check(load().pic_init_static(arr, n, parr, C.c_void_p(stream_ptr), C.byref(st)), "pic_init_static")
    return st


def pic_step(st, nsteps):
    return check(load().pic_step(st, int(nsteps)), "pic_step")


def pic_prepare(st, nsteps):
    return check(load().pic_prepare(st, int(nsteps)), "pic_prepare")


def pic_set_option(st, name, value):
    return check(load().pic_set_option(st, name.encode(), int(value)), "pic_set_option(%s)" % name)


def pic_get_option(st, name):
    v = C.c_int(0)
    check(load().pic_get_option(st, name.encode(), C.byref(v)), "pic_get_option(%s)" % name)
    return v.value


def pic_set_schedule(st, sched, use_graph):
    return check(load().pic_set_schedule(st, int(sched), int(use_graph)), "pic_set_schedule")


def pic_fields(st, inst, which, comp, host, direction=PIC_GET):
    return check(load().pic_fields(st, int(inst), int(which), int(comp), dptr(host), host.size,
                                   int(direction)), "pic_fields")


def pic_get_particles(st, inst, pos, mom, n):
    P = (_D * 3)(*[dptr(p) if p is not None else None for p in pos])
    M = (_D * 3)(*[dptr(m) for m in mom])
    return check(load().pic_get_particles(st, int(inst), P, M, int(n)), "pic_get_particles")


def pic_diag(st, inst):
    d = pic_diag_t()
    rc = load().pic_diag(st, int(inst), C.byref(d))
    return rc, d


def pic_read_trace(st, inst, out):
    cnt = C.c_int(0)
    check(load().pic_read_trace(st, int(inst), dptr(out), out.shape[0], C.byref(cnt)), "pic_read_trace")
    return cnt.value


def pic_profile(st, nsteps):
    t = pic_timing_t()
    check(load().pic_profile(st, int(nsteps), C.byref(t)), "pic_profile")
    return t


def pic_info(st):
    ni, npart, nc = C.c_int(0), C.c_int64(0), C.c_int64(0)
    check(load().pic_info(st, C.byref(ni), C.byref(npart), C.byref(nc)), "pic_info")
    return ni.value, npart.value, nc.value


def pic_adjoint_forward(st, nsteps, n_inst):
    import numpy as np
    loss = np.zeros(n_inst)
    check(load().pic_adjoint_forward(st, int(nsteps), dptr(loss)), "pic_adjoint_forward")
    return loss


def pic_adjoint_backward(st, n_inst):
    import numpy as np
    grad = np.zeros(n_inst * 9)
    check(load().pic_adjoint_backward(st, dptr(grad)), "pic_adjoint_backward")
    return grad.reshape(n_inst, 9)


def pic_destroy(st):
    load().pic_destroy(st)
