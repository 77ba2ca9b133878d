"""Thin ctypes binding of libz2h (include/z2h.h): same names, argument
marshalling only.  Device buffers are torch tensors (PyTorch supplies device
memory and streams); every computation runs in the HIP library.

There is no fallback: if libz2h.so is missing or fails to load, every entry
point raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# Z2H_LIB names another build of the same library (the sanitizer build of
# the host code used by the CPU tests); default: the in-tree gfx950 build.
LIB_PATH = os.environ.get("Z2H_LIB") or os.path.join(_HERE, "libz2h.so")

Z2H_OK = 0
Z2H_ERR_INVALID = -1
Z2H_ERR_UNSUPPORTED = -2
Z2H_ERR_OOM = -3
Z2H_ERR_HIP = -4
Z2H_ERR_NUMERIC = -5
Z2H_ERR_WORKSPACE = -6

Z2H_C64 = 0
Z2H_C128 = 1

Z2H_INIT_PSI1 = 0
Z2H_INIT_PSI1P = 1
Z2H_INIT_ZERO = 2
Z2H_INIT_PLUS = 3

Z2H_MAX_LOOPS = 8
Z2H_DOS_BINS = 33
Z2H_OBS_DOUBLES = 56


class Z2HError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"z2h error {code}: {msg}")
        self.code = code


class z2h_couplings(ctypes.Structure):
    _fields_ = [("JA", ctypes.c_double), ("JB", ctypes.c_double),
                ("hx", ctypes.c_double), ("hz", ctypes.c_double)]


class z2h_schedule(ctypes.Structure):
    _fields_ = [("start", z2h_couplings), ("end", z2h_couplings),
                ("steps", ctypes.c_int64), ("dt", ctypes.c_double),
                ("k_begin", ctypes.c_int64), ("k_end", ctypes.c_int64),
                ("sampling", ctypes.c_int32), ("order", ctypes.c_int32),
                ("renorm", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sZ", ctypes.POINTER(ctypes.c_double)), ("sX", ctypes.POINTER(ctypes.c_double))]


class z2h_path(ctypes.Structure):
    _fields_ = [("nvert", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("vert", ctypes.POINTER(z2h_couplings)), ("steps", ctypes.POINTER(ctypes.c_int64)),
                ("dt", ctypes.c_double), ("sampling", ctypes.c_int32), ("order", ctypes.c_int32),
                ("renorm", ctypes.c_int32), ("trace_every", ctypes.c_int32)]


class z2h_gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("theta", ctypes.c_double)]


Z2H_GATE_H, Z2H_GATE_RX, Z2H_GATE_RZ, Z2H_GATE_CNOT, Z2H_GATE_PROJ0, Z2H_GATE_NORM = range(6)


class z2h_obs(ctypes.Structure):
    _fields_ = [("norm", ctypes.c_double), ("energy", ctypes.c_double),
                ("sumA", ctypes.c_double), ("sumB", ctypes.c_double),
                ("mx", ctypes.c_double), ("mz", ctypes.c_double),
                ("zloop", ctypes.c_double * Z2H_MAX_LOOPS),
                ("xloop", ctypes.c_double * Z2H_MAX_LOOPS),
                ("dos", ctypes.c_double * Z2H_DOS_BINS),
                ("xnorm", ctypes.c_double)]


# Every symbol the header declares, with its ctypes signature.
_P = ctypes.c_void_p
_i32, _i64, _sz, _dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
SIGNATURES = {
    "z2h_link_bit": (_i32, [_i32, _i32, _i32, _i32, _i32, ctypes.POINTER(_i32)]),
    "z2h_masks": (_i32, [_i32, _i32, _P, _P]),
    "z2h_loop_masks": (_i32, [_i32, _i32, _P, ctypes.POINTER(_i32), _P, ctypes.POINTER(_i32)]),
    "z2h_plan_create": (_i32, [_i32, _i32, _i32, _i32, ctypes.POINTER(_P)]),
    "z2h_plan_destroy": (None, [_P]),
    "z2h_plan_sizes": (_i32, [_P, ctypes.POINTER(_sz), ctypes.POINTER(_sz), ctypes.POINTER(_sz),
                              ctypes.POINTER(_sz)]),
    "z2h_plan_info": (_i32, [_P, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                             ctypes.POINTER(_i32)]),
    "z2h_plan_describe": (_i32, [_P, ctypes.c_char_p, _sz]),
    "z2h_state_init": (_i32, [_P, _P, _i32, _P]),
    "z2h_evolve": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_schedule), _P, _P]),
    "z2h_evolve_noalloc": (_i32, [_P, _P, ctypes.POINTER(z2h_schedule), _P, _P]),
    "z2h_observe": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_couplings), _P, _i32, _P, _i32,
                           ctypes.POINTER(z2h_obs), _P, _P]),
    "z2h_adjoint": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_schedule), ctypes.POINTER(z2h_couplings),
                           _P, _P, ctypes.POINTER(_dbl), _P]),
    "z2h_batch_create": (_i32, [_i32, _P, _P, ctypes.POINTER(z2h_schedule), _P,
                                ctypes.POINTER(z2h_couplings), _i32, ctypes.POINTER(_P),
                                ctypes.POINTER(_sz), ctypes.POINTER(_sz), _P]),
    "z2h_batch_run": (_i32, [_P, _P, _P, _sz, _P, _P]),
    "z2h_batch_destroy": (None, [_P]),
    "z2h_batch_timing": (_i32, [_P, _P, _P]),
    "z2h_autotune": (_i32, [_i32, _i32, _i32, _i32, ctypes.c_char_p, ctypes.c_char_p, _sz, ctypes.POINTER(_dbl)]),
    "z2h_tune_load": (_i32, [ctypes.c_char_p]),
    "z2h_plan_create_config": (_i32, [_i32, _i32, _i32, ctypes.c_char_p, ctypes.POINTER(_P)]),
    "z2h_tune_candidates": (_i32, [_i32, _i32, _i32, ctypes.c_char_p, _sz]),
    "z2h_batch_trace_sizes": (_i32, [_P, _i32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_sz)]),
    "z2h_batch_run_trace": (_i32, [_P, _P, _P, _sz, _P, _i32, _P, _P]),
    "z2h_path_evolve": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_path), _P, _i32, _P, _i32, _P,
                                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), _P]),
    "z2h_hamiltonian_apply": (_i32, [_P, _P, _P, ctypes.POINTER(z2h_couplings), _P]),
    "z2h_lanczos_sizes": (_i32, [_P, _i32, ctypes.POINTER(_sz)]),
    "z2h_lanczos_ground": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_couplings), _i32, _dbl, _P, _P,
                                  ctypes.POINTER(_i32), ctypes.POINTER(_dbl), _P]),
    "z2h_exact_sizes": (_i32, [_P, _i32, ctypes.POINTER(_sz)]),
    "z2h_exact_evolve": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_schedule), _i32, ctypes.POINTER(_dbl), _P]),
    "z2h_lanczos_vector_sizes": (_i32, [_P, _i32, ctypes.POINTER(_sz)]),
    "z2h_lanczos_vector": (_i32, [_P, _P, _P, _sz, ctypes.POINTER(z2h_couplings), _P, _P, _i32,
                                  ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), _P]),
    "z2h_overlap": (_i32, [_P, _P, _P, _P, _sz, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), _P]),
    "z2h_tridiag_lowest": (_i32, [_i32, _P, _P, ctypes.POINTER(_dbl)]),
    "z2h_tridiag_expv": (_i32, [_i32, _P, _P, _dbl, _P, _P]),
    "z2h_circuit_step": (_i32, [_i32, _i32, ctypes.POINTER(z2h_couplings), ctypes.POINTER(z2h_couplings), _dbl, _i32,
                                 _P, _i32, ctypes.POINTER(_i32)]),
    "z2h_circuit_prep": (_i32, [_i32, _i32, _i32, _P, _i32, ctypes.POINTER(_i32)]),
    "z2h_gates_ws_bytes": (_sz, [_i32]),
    "z2h_gates_run": (_i32, [_i32, _i32, _P, _P, _sz, _P, _i32, _i32, _P]),
    "z2h_gates_schedule": (_i32, [_i32, _i32, _P, _i32, _i32, _P, _P]),
    "z2h_circuit_evolve": (_i32, [_i32, _i32, _i32, _P, _P, _sz, ctypes.POINTER(z2h_schedule), _i32, _P]),
    "z2h_paths_sizes": (_i32, [_P, _i32, _P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_sz)]),
    "z2h_paths_evolve": (_i32, [_P, _i32, _P, _P, _sz, _P, _P, _i32, _P, _i32, _P, _P]),
    "z2h_timing_enable": (_i32, [_i32]),
    "z2h_timing_read": (_i32, [_P, _P]),
    "z2h_version": (ctypes.c_char_p, []),
    "z2h_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libz2h.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime under the same soname as the
        # system's; load it first so that the library and torch share one
        # runtime instance (the other order leaves torch without devices)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_2108_13410_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code):
    if code != Z2H_OK:
        raise Z2HError(code, lib().z2h_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def couplings(JA=1.0, JB=1.0, hx=0.0, hz=0.0):
    return z2h_couplings(float(JA), float(JB), float(hx), float(hz))


def schedule(start, end, steps, dt, k_begin=0, k_end=None, sampling=0, order=0, renorm=0,
             sZ=None, sX=None):
    """Build a z2h_schedule; sZ/sX are kept alive on the returned object."""
    s = z2h_schedule()
    s.start = start if isinstance(start, z2h_couplings) else couplings(*start)
    s.end = end if isinstance(end, z2h_couplings) else couplings(*end)
    s.steps = int(steps)
    s.dt = float(dt)
    s.k_begin = int(k_begin)
    s.k_end = int(steps if k_end is None else k_end)
    s.sampling = int(sampling)
    s.order = int(order)
    s.renorm = int(renorm)
    keep = []
    for name, arr in (("sZ", sZ), ("sX", sX)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64)
            keep.append(a)
            setattr(s, name, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    s._keep = keep
    return s


# ------------------------------------------------------------------ entry points

def z2h_version():
    return lib().z2h_version().decode()


def z2h_last_error():
    return lib().z2h_last_error().decode()


def z2h_link_bit(Lx, Ly, x, y, d):
    b = ctypes.c_int32()
    _check(lib().z2h_link_bit(Lx, Ly, x, y, d, ctypes.byref(b)))
    return b.value


def z2h_masks(Lx, Ly):
    st = np.zeros(Lx * Ly, np.uint64)
    pl = np.zeros(Lx * Ly, np.uint64)
    _check(lib().z2h_masks(Lx, Ly, st.ctypes.data_as(_P), pl.ctypes.data_as(_P)))
    return st, pl


def z2h_loop_masks(Lx, Ly):
    """(zloops, xloops) lists of the loop masks batches report."""
    z = np.zeros(Z2H_MAX_LOOPS, np.uint64)
    x = np.zeros(Z2H_MAX_LOOPS, np.uint64)
    nz, nx = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().z2h_loop_masks(Lx, Ly, z.ctypes.data_as(_P), ctypes.byref(nz), x.ctypes.data_as(_P),
                                ctypes.byref(nx)))
    return [int(v) for v in z[:nz.value]], [int(v) for v in x[:nx.value]]


class Plan:
    """Owns a z2h_plan*; destroyed with the object."""

    def __init__(self, handle, Lx, Ly, dtype):
        self.handle = handle
        self.Lx, self.Ly, self.dtype = Lx, Ly, dtype
        self.n = 2 * Lx * Ly

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.z2h_plan_destroy(self.handle)
            self.handle = None


def z2h_plan_create(Lx, Ly, dtype, max_tile_bits=0):
    h = ctypes.c_void_p()
    _check(lib().z2h_plan_create(Lx, Ly, dtype, max_tile_bits, ctypes.byref(h)))
    return Plan(h, Lx, Ly, dtype)


def z2h_plan_destroy(plan):
    if plan.handle:
        lib().z2h_plan_destroy(plan.handle)
        plan.handle = None


def z2h_plan_sizes(plan):
    v = [ctypes.c_size_t() for _ in range(4)]
    _check(lib().z2h_plan_sizes(plan.handle, *[ctypes.byref(x) for x in v]))
    return dict(zip(("state", "ws_evolve", "ws_observe", "ws_adjoint"), [x.value for x in v]))


def z2h_plan_info(plan):
    v = [ctypes.c_int32() for _ in range(4)]
    _check(lib().z2h_plan_info(plan.handle, *[ctypes.byref(x) for x in v]))
    return dict(zip(("n", "groups", "passes_per_step", "tile_bits"), [x.value for x in v]))


def z2h_plan_describe(plan):
    import json
    buf = ctypes.create_string_buffer(8192)
    _check(lib().z2h_plan_describe(plan.handle, buf, len(buf)))
    return json.loads(buf.value.decode())


def z2h_state_init(plan, state, kind, stream=None):
    _check(lib().z2h_state_init(plan.handle, _ptr(state), kind, _stream(stream)))


def z2h_evolve(plan, state, ws, sched, norms=None, stream=None):
    _check(lib().z2h_evolve(plan.handle, _ptr(state), _ptr(ws), ws.numel() * ws.element_size(),
                            ctypes.byref(sched), _ptr(norms), _stream(stream)))


def z2h_evolve_noalloc(plan, state, sched, norms=None, stream=None):
    _check(lib().z2h_evolve_noalloc(plan.handle, _ptr(state), ctypes.byref(sched), _ptr(norms),
                                    _stream(stream)))


Z2H_NOALLOC_SCRATCH_BYTES = 16 << 20


def _masks_arg(masks):
    if masks is None or len(masks) == 0:
        return None, 0, None
    a = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    return a.ctypes.data_as(_P), int(a.size), a


def obs_to_dict(o):
    return {
        "norm": o.norm, "energy": o.energy, "sumA": o.sumA, "sumB": o.sumB, "mx": o.mx, "mz": o.mz,
        "zloop": list(o.zloop), "xloop": list(o.xloop), "dos": list(o.dos), "xnorm": o.xnorm,
    }


def z2h_observe(plan, state, ws, H, zmasks=None, xmasks=None, d_out=None, host=True, stream=None):
    zp, nz, za = _masks_arg(zmasks)
    xp, nx, xa = _masks_arg(xmasks)
    out = z2h_obs() if host else None
    Hc = H if isinstance(H, z2h_couplings) else couplings(*H)
    _check(lib().z2h_observe(plan.handle, _ptr(state), _ptr(ws), ws.numel() * ws.element_size(),
                             ctypes.byref(Hc), zp, nz, xp, nx,
                             ctypes.byref(out) if out is not None else None, _ptr(d_out), _stream(stream)))
    del za, xa
    return obs_to_dict(out) if out is not None else None


def z2h_adjoint(plan, psi_final, ws, sched, lossH, gradZ, gradX, stream=None):
    loss = ctypes.c_double()
    Hc = lossH if isinstance(lossH, z2h_couplings) else couplings(*lossH)
    _check(lib().z2h_adjoint(plan.handle, _ptr(psi_final), _ptr(ws), ws.numel() * ws.element_size(),
                             ctypes.byref(sched), ctypes.byref(Hc), _ptr(gradZ), _ptr(gradX),
                             ctypes.byref(loss), _stream(stream)))
    return loss.value


def make_path(vertices, steps, dt, sampling=1, order=0, renorm=0, every=0):
    """z2h_path for a list of coupling 4-tuples and per-leg step counts; the
    returned object keeps its arrays alive."""
    nv = len(vertices)
    if len(steps) != nv - 1:
        raise ValueError("need one step count per leg")
    verts = (z2h_couplings * nv)(*[v if isinstance(v, z2h_couplings) else couplings(*v) for v in vertices])
    st = (ctypes.c_int64 * (nv - 1))(*[int(m) for m in steps])
    p = z2h_path(nv, 0, verts, st, float(dt), int(sampling), int(order), int(renorm), int(every))
    p._keep = (verts, st)
    return p


def z2h_path_evolve(plan, state, ws, path, zmasks=None, xmasks=None, stream=None):
    """Evolve along a path; returns the device trace (samples x Z2H_OBS_DOUBLES)."""
    import torch
    zp, nz, za = _masks_arg(zmasks)
    xp, nx, xa = _masks_arg(xmasks)
    ns = ctypes.c_int64()
    L = lib()
    _check(L.z2h_path_evolve(plan.handle, None, None, 0, ctypes.byref(path), zp, nz, xp, nx, None, 0,
                             ctypes.byref(ns), None))
    trace = torch.empty((ns.value, Z2H_OBS_DOUBLES), dtype=torch.float64, device=state.device)
    _check(L.z2h_path_evolve(plan.handle, _ptr(state), _ptr(ws), ws.numel() * ws.element_size(),
                             ctypes.byref(path), zp, nz, xp, nx, _ptr(trace), ns.value, None, _stream(stream)))
    return trace


# ------------------------------------------------------------------ exact solvers

def z2h_hamiltonian_apply(plan, x, y, H, stream=None):
    """y = H x (device states of the plan; must not overlap)."""
    Hc = H if isinstance(H, z2h_couplings) else couplings(*H)
    _check(lib().z2h_hamiltonian_apply(plan.handle, _ptr(x), _ptr(y), ctypes.byref(Hc), _stream(stream)))


def z2h_lanczos_sizes(plan, max_iter):
    n = ctypes.c_size_t()
    _check(lib().z2h_lanczos_sizes(plan.handle, int(max_iter), ctypes.byref(n)))
    return n.value


def z2h_lanczos_ground(plan, v, ws, H, max_iter=300, tol=1e-13, stream=None):
    """Ground energy by Lanczos from the start vector v (overwritten).
    Returns (e0, iterations, alpha, beta) with alpha / beta numpy arrays."""
    import numpy as np
    Hc = H if isinstance(H, z2h_couplings) else couplings(*H)
    a = np.zeros(int(max_iter))
    b = np.zeros(int(max_iter))
    it = ctypes.c_int32()
    e0 = ctypes.c_double()
    _check(lib().z2h_lanczos_ground(plan.handle, _ptr(v), _ptr(ws), ws.numel() * ws.element_size(),
                                    ctypes.byref(Hc), int(max_iter), float(tol), a.ctypes.data_as(_P),
                                    b.ctypes.data_as(_P), ctypes.byref(it), ctypes.byref(e0), _stream(stream)))
    return e0.value, it.value, a[:it.value].copy(), b[:it.value].copy()


def z2h_lanczos_vector_sizes(plan, iters):
    """Workspace bytes of z2h_lanczos_vector for a recurrence of iters steps."""
    n = ctypes.c_size_t()
    _check(lib().z2h_lanczos_vector_sizes(plan.handle, int(iters), ctypes.byref(n)))
    return n.value


def z2h_lanczos_vector(plan, v, H, alpha, beta, stream=None):
    """Ground-state vector into v (which must hold the start vector of the
    z2h_lanczos_ground run that produced alpha, beta).  Returns (energy,
    residual)."""
    import numpy as np
    Hc = H if isinstance(H, z2h_couplings) else couplings(*H)
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    n = ctypes.c_size_t()
    _check(lib().z2h_lanczos_vector_sizes(plan.handle, len(a), ctypes.byref(n)))
    ws = alloc_bytes(n.value, device=v.device)
    e, r = ctypes.c_double(), ctypes.c_double()
    _check(lib().z2h_lanczos_vector(plan.handle, _ptr(v), _ptr(ws), n.value, ctypes.byref(Hc), a.ctypes.data_as(_P),
                                    b.ctypes.data_as(_P), len(a), ctypes.byref(e), ctypes.byref(r), _stream(stream)))
    del ws
    return e.value, r.value


def z2h_overlap(plan, a, b, stream=None):
    """<a|b> as a Python complex."""
    ws = alloc_bytes(32768, device=a.device)
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().z2h_overlap(plan.handle, _ptr(a), _ptr(b), _ptr(ws), 32768, ctypes.byref(re), ctypes.byref(im),
                             _stream(stream)))
    return complex(re.value, im.value)


def z2h_exact_sizes(plan, krylov_dim):
    n = ctypes.c_size_t()
    _check(lib().z2h_exact_sizes(plan.handle, int(krylov_dim), ctypes.byref(n)))
    return n.value


def z2h_exact_evolve(plan, state, ws, sched, krylov_dim=16, stream=None):
    """Stepwise exact evolution of state (in place); returns the Krylov
    truncation error estimate summed over steps."""
    err = ctypes.c_double()
    _check(lib().z2h_exact_evolve(plan.handle, _ptr(state), _ptr(ws), ws.numel() * ws.element_size(),
                                  ctypes.byref(sched), int(krylov_dim), ctypes.byref(err), _stream(stream)))
    return err.value


def z2h_tridiag_lowest(alpha, beta):
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    out = ctypes.c_double()
    _check(lib().z2h_tridiag_lowest(len(a), a.ctypes.data_as(_P), b.ctypes.data_as(_P) if len(b) else None,
                                    ctypes.byref(out)))
    return out.value


def z2h_tridiag_expv(alpha, beta, tau):
    import numpy as np
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    re = np.zeros(len(a))
    im = np.zeros(len(a))
    _check(lib().z2h_tridiag_expv(len(a), a.ctypes.data_as(_P), b.ctypes.data_as(_P) if len(b) else None,
                                  float(tau), re.ctypes.data_as(_P), im.ctypes.data_as(_P)))
    return re + 1j * im


# ------------------------------------------------------------------ gate-level circuits

def _gate_list(fn, *args):
    cnt = ctypes.c_int32()
    code = fn(*args, None, 0, ctypes.byref(cnt))
    if code not in (Z2H_OK, -6):
        _check(code)
    arr = (z2h_gate * max(cnt.value, 1))()
    _check(fn(*args, arr, cnt.value, ctypes.byref(cnt)))
    return arr, cnt.value


def z2h_circuit_step(Lx, Ly, cx, cz, dt, order=0):
    """The gates of one Trotter step (ctypes array, count)."""
    cxs = cx if isinstance(cx, z2h_couplings) else couplings(*cx)
    czs = cz if isinstance(cz, z2h_couplings) else couplings(*cz)
    return _gate_list(lib().z2h_circuit_step, int(Lx), int(Ly), ctypes.byref(cxs), ctypes.byref(czs), float(dt),
                      int(order))


def z2h_circuit_prep(Lx, Ly, which=Z2H_INIT_PSI1):
    return _gate_list(lib().z2h_circuit_prep, int(Lx), int(Ly), int(which))


def gates_to_list(arr, n):
    return [(g.kind, g.q0, g.q1, g.theta) for g in arr[:n]]


def z2h_gates_ws_bytes(nq):
    return int(lib().z2h_gates_ws_bytes(int(nq)))


def z2h_gates_schedule(nq, dtype, gates, ngates, fuse=1):
    """The passes z2h_gates_run would make (host only): (pass index of each
    gate as a list, number of passes)."""
    pass_of = (ctypes.c_int32 * max(int(ngates), 1))()
    npasses = ctypes.c_int32()
    _check(lib().z2h_gates_schedule(int(nq), int(dtype), gates, int(ngates), int(fuse), pass_of,
                                    ctypes.byref(npasses)))
    return list(pass_of[:int(ngates)]), npasses.value


def z2h_gates_run(nq, dtype, state, ws, gates, ngates, fuse=1, stream=None):
    _check(lib().z2h_gates_run(int(nq), int(dtype), _ptr(state), _ptr(ws), ws.numel() * ws.element_size(),
                               gates, int(ngates), int(fuse), _stream(stream)))


def z2h_circuit_evolve(Lx, Ly, dtype, state, ws, sched, fuse=1, stream=None):
    _check(lib().z2h_circuit_evolve(int(Lx), int(Ly), int(dtype), _ptr(state), _ptr(ws),
                                    ws.numel() * ws.element_size(), ctypes.byref(sched), int(fuse), _stream(stream)))


def z2h_paths_sizes(plan, paths):
    """(trace samples, workspace bytes) of z2h_paths_evolve for these paths."""
    arr = (z2h_path * len(paths))(*paths)
    ns = ctypes.c_int64()
    wsb = ctypes.c_size_t()
    _check(lib().z2h_paths_sizes(plan.handle, len(paths), arr, ctypes.byref(ns), ctypes.byref(wsb)))
    return ns.value, wsb.value


def z2h_paths_evolve(plan, paths, states=None, inits=None, zmasks=None, xmasks=None, stream=None):
    """Run several paths of one lattice together.  paths: list of make_path
    objects; states: device tensor of len(paths) * 2^n complex elements (or
    None: allocated and initialised from inits, Z2H_INIT_* per path).
    Returns (states, trace) with trace shaped (samples, len(paths), 56)."""
    import torch
    n = plan.n
    npaths = len(paths)
    arr = (z2h_path * npaths)(*paths)
    ns = ctypes.c_int64()
    wsb = ctypes.c_size_t()
    L = lib()
    _check(L.z2h_paths_sizes(plan.handle, npaths, arr, ctypes.byref(ns), ctypes.byref(wsb)))
    if states is None:
        dt = torch.complex128 if plan.dtype == Z2H_C128 else torch.complex64
        states = torch.empty(npaths << n, dtype=dt, device="cuda")
        for j in range(npaths):
            z2h_state_init(plan, states[j << n:(j + 1) << n], (inits or [Z2H_INIT_PSI1] * npaths)[j], stream=stream)
    ws = alloc_bytes(wsb.value, device=states.device)
    trace = torch.empty((ns.value, npaths, Z2H_OBS_DOUBLES), dtype=torch.float64, device=states.device)
    zp, nz, za = _masks_arg(zmasks)
    xp, nx, xa = _masks_arg(xmasks)
    _check(L.z2h_paths_evolve(plan.handle, npaths, _ptr(states), _ptr(ws), wsb.value, arr, zp, nz, xp, nx,
                              _ptr(trace), _stream(stream)))
    del za, xa, arr
    return states, trace


class Batch:
    def __init__(self, handle, njobs, states_bytes, ws_bytes, offsets):
        self.handle = handle
        self.njobs = njobs
        self.states_bytes = states_bytes
        self.ws_bytes = ws_bytes
        self.offsets = offsets

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.z2h_batch_destroy(self.handle)
            self.handle = None


def z2h_batch_create(Lx, Ly, scheds, inits, obsH, dtype):
    nj = len(scheds)
    Lxa = np.ascontiguousarray(Lx, dtype=np.int32)
    Lya = np.ascontiguousarray(Ly, dtype=np.int32)
    ina = np.ascontiguousarray(inits, dtype=np.int32)
    S = (z2h_schedule * nj)(*scheds)
    Hs = (z2h_couplings * nj)(*[h if isinstance(h, z2h_couplings) else couplings(*h) for h in obsH])
    h = ctypes.c_void_p()
    sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    offs = np.zeros(nj, np.uint64)
    _check(lib().z2h_batch_create(nj, Lxa.ctypes.data_as(_P), Lya.ctypes.data_as(_P), S,
                                  ina.ctypes.data_as(_P), Hs, dtype, ctypes.byref(h),
                                  ctypes.byref(sb), ctypes.byref(wb), offs.ctypes.data_as(_P)))
    return Batch(h, nj, sb.value, wb.value, offs)


def z2h_batch_run(batch, states, ws, d_obs, stream=None):
    _check(lib().z2h_batch_run(batch.handle, _ptr(states), _ptr(ws), ws.numel() * ws.element_size(),
                               _ptr(d_obs), _stream(stream)))


def z2h_batch_trace_sizes(batch, every):
    ns = ctypes.c_int64()
    wb = ctypes.c_size_t()
    _check(lib().z2h_batch_trace_sizes(batch.handle, int(every), ctypes.byref(ns), ctypes.byref(wb)))
    return ns.value, wb.value


def z2h_batch_run_trace(batch, states, ws, d_obs, every, d_trace, stream=None):
    _check(lib().z2h_batch_run_trace(batch.handle, _ptr(states), _ptr(ws), ws.numel() * ws.element_size(),
                                     _ptr(d_obs), int(every), _ptr(d_trace), _stream(stream)))


def z2h_batch_destroy(batch):
    if batch.handle:
        lib().z2h_batch_destroy(batch.handle)
        batch.handle = None


def z2h_batch_timing(batch):
    c = np.zeros(4, np.int64)
    m = np.zeros(4, np.float64)
    _check(lib().z2h_batch_timing(batch.handle, c.ctypes.data_as(_P), m.ctypes.data_as(_P)))
    return c, m


def z2h_autotune(Lx, Ly, dtype, batch, cache_path=None):
    """Returns (schedule string, ms per Trotter step) of the fastest candidate."""
    buf = ctypes.create_string_buffer(512)
    ms = ctypes.c_double()
    _check(lib().z2h_autotune(Lx, Ly, dtype, batch, None if cache_path is None else cache_path.encode(),
                              buf, len(buf), ctypes.byref(ms)))
    return buf.value.decode(), ms.value


def z2h_plan_create_config(Lx, Ly, dtype, schedule):
    h = ctypes.c_void_p()
    _check(lib().z2h_plan_create_config(Lx, Ly, dtype, schedule.encode(), ctypes.byref(h)))
    return Plan(h, Lx, Ly, dtype)


def z2h_tune_candidates(Lx, Ly, dtype):
    buf = ctypes.create_string_buffer(16384)
    _check(lib().z2h_tune_candidates(Lx, Ly, dtype, buf, len(buf)))
    return [l for l in buf.value.decode().split("\n") if l]


def z2h_tune_load(cache_path):
    _check(lib().z2h_tune_load(cache_path.encode()))


def z2h_timing_enable(on):
    _check(lib().z2h_timing_enable(1 if on else 0))


def z2h_timing_read():
    c = np.zeros(4, np.int64)
    m = np.zeros(4, np.float64)
    _check(lib().z2h_timing_read(c.ctypes.data_as(_P), m.ctypes.data_as(_P)))
    return c, m


# ------------------------------------------------------------------ plumbing helpers

def alloc_state(plan, device="cuda"):
    """Uninitialized device tensor of 2^n complex elements for a plan."""
    import torch
    dt = torch.complex128 if plan.dtype == Z2H_C128 else torch.complex64
    return torch.empty(1 << plan.n, dtype=dt, device=device)


def alloc_bytes(nbytes, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
