"""Thin ctypes binding of ``libwadg.so`` (the C ABI in ``include/wadg.h``).

Functions carry the C names and only marshal arguments: every step of the
sweep runs in the HIP kernels of the library.  Device arrays may be passed
as torch tensors (contiguous, float64, on a HIP device) or as raw integer
device addresses; streams as ``torch.cuda.Stream`` objects, raw handles or
``None`` (the current torch stream).

The library must have been built (``python paper_1608_03836_amd/build.py``);
importing this module without it raises immediately -- there is no
fallback implementation.
"""

import ctypes
import os

import numpy as np

# WADG_LIBRARY names another build of the same library (the host-sanitizer
# build that the CPU tests load); by default the in-tree libwadg.so
LIB_PATH = os.environ.get("WADG_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libwadg.so")

WADG_OK = 0
WADG_E_INVALID = -1
WADG_E_GEOMETRY = -2
WADG_E_UNSUPPORTED = -3
WADG_E_DEVICE = -4
WADG_E_NONFINITE = -5
WADG_MAX_N = 4
WADG_KERNEL_AUTO = 0
WADG_KERNEL_STREAMED = 1
WADG_KERNEL_RESIDENT = 2
WADG_KERNEL_SPLIT = 3
WADG_KERNEL_PIPE = 4
WADG_CFL_MAX = 1.25
WADG_NORMS_NOALLOC_MAX_S = 1024
TILE_LANES = 64

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)


class WadgError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{message} (status {status})")
        self.status = status


class wadg_mesh(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nq1", ctypes.c_int32), ("K", ctypes.c_int32),
                ("x", _c_double_p), ("y", _c_double_p),
                ("etoe", _c_int32_p), ("etof", _c_int32_p), ("c2q", _c_double_p),
                ("tau_p", ctypes.c_double), ("tau_u", ctypes.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python paper_1608_03836_amd/build.py`")
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # soname, requested under its unversioned name), so torch is loaded first
    # and the library's dependency then resolves to that copy.  Loading the
    # library first would bring in a second runtime, and device selection in
    # one of them fails.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "wadg_quadrature_points": (ctypes.c_int, [ctypes.POINTER(wadg_mesh), _c_double_p, _c_double_p]),
        "wadg_geometry": (ctypes.c_int, [ctypes.POINTER(wadg_mesh), _c_double_p, _c_double_p]),
        "wadg_cfl_number": (ctypes.c_int, [ctypes.POINTER(wadg_mesh), ctypes.c_double,
                                           ctypes.c_double, _c_double_p]),
        "wadg_create": (ctypes.c_int, [ctypes.POINTER(wadg_mesh), ctypes.c_int32, ctypes.POINTER(vp)]),
        "wadg_destroy": (None, [vp]),
        "wadg_state_doubles": (ctypes.c_int, [vp, ctypes.POINTER(sz)]),
        "wadg_workspace_bytes": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(sz)]),
        "wadg_rhs": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, vp]),
        "wadg_integrate": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, ctypes.c_double,
                                          ctypes.c_int32, vp]),
        "wadg_workspace_bytes_fp32": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(sz)]),
        "wadg_integrate_fp32": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, ctypes.c_double,
                                               ctypes.c_int32, vp]),
        "wadg_parareal_workspace_bytes": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32,
                                                         ctypes.POINTER(sz)]),
        "wadg_parareal": (ctypes.c_int, [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double), vp]),
        "wadg_norms_workspace_bytes": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(sz)]),
        "wadg_norms": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, vp, sz, _c_double_p, vp]),
        "wadg_norms_noalloc": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, _c_double_p, vp]),
        "wadg_l2_norms_workspace_bytes": (ctypes.c_int, [vp, ctypes.c_int32,
                                                         ctypes.POINTER(sz)]),
        "wadg_l2_norms": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, vp, sz, _c_double_p, vp]),
        "wadg_set_schedule": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32]),
        "wadg_set_kernel": (ctypes.c_int, [vp, ctypes.c_int32]),
        "wadg_set_c2_scale": (ctypes.c_int, [vp, ctypes.c_double]),
        "wadg_batch_create": (ctypes.c_int, [ctypes.POINTER(wadg_mesh), ctypes.c_int32,
                                             _c_int32_p, ctypes.c_int32, ctypes.POINTER(vp)]),
        "wadg_batch_destroy": (None, [vp]),
        "wadg_batch_layout": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64), _c_int32_p]),
        "wadg_batch_workspace_bytes": (ctypes.c_int, [vp, ctypes.POINTER(sz)]),
        "wadg_batch_integrate": (ctypes.c_int, [vp, vp, vp, _c_double_p, ctypes.c_int32, vp]),
        "wadg_batch_set_schedule": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32]),
        "wadg_batch_set_runs": (ctypes.c_int, [vp, ctypes.c_int32]),
        "wadg_batch_tune": (ctypes.c_int, [vp, vp, vp, _c_double_p, ctypes.c_int32, _c_int32_p,
                                           _c_int32_p, _c_int32_p, _c_double_p, vp]),
        "wadg_batch_capture": (ctypes.c_int, [vp, vp, vp, _c_double_p, ctypes.c_int32]),
        "wadg_batch_replay": (ctypes.c_int, [vp, vp]),
        "wadg_batch_release_graph": (ctypes.c_int, [vp]),
        "wadg_adjoint_workspace_bytes": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(sz)]),
        "wadg_forward_checkpoints": (ctypes.c_int, [vp, vp, vp, ctypes.c_int32, ctypes.c_double,
                                                    ctypes.c_int32, vp]),
        "wadg_adjoint": (ctypes.c_int, [vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int32, ctypes.POINTER(ctypes.c_double), vp]),
        "wadg_kernel_in_use": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_int32)]),
        "wadg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "wadg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("wadg_quadrature_points", "wadg_geometry", "wadg_cfl_number", "wadg_create", "wadg_destroy",
            "wadg_state_doubles", "wadg_workspace_bytes", "wadg_rhs", "wadg_integrate",
            "wadg_workspace_bytes_fp32", "wadg_integrate_fp32",
            "wadg_parareal_workspace_bytes", "wadg_parareal",
            "wadg_norms_workspace_bytes", "wadg_norms", "wadg_norms_noalloc",
            "wadg_l2_norms_workspace_bytes",
            "wadg_l2_norms", "wadg_set_schedule", "wadg_set_kernel", "wadg_kernel_in_use",
            "wadg_set_c2_scale", "wadg_adjoint_workspace_bytes", "wadg_forward_checkpoints",
            "wadg_adjoint", "wadg_batch_create", "wadg_batch_destroy", "wadg_batch_layout",
            "wadg_batch_workspace_bytes", "wadg_batch_integrate", "wadg_batch_set_schedule",
            "wadg_batch_set_runs",
            "wadg_batch_tune", "wadg_batch_capture", "wadg_batch_replay",
            "wadg_batch_release_graph",
            "wadg_status_string", "wadg_last_error")


def _check(status):
    if status != WADG_OK:
        msg = LIB.wadg_last_error().decode() or LIB.wadg_status_string(status).decode()
        raise WadgError(status, msg)


# ----------------------------------------------------------------- marshalling
class MeshDesc:
    """Owns the host arrays behind a ``wadg_mesh`` struct.

    ``x, y``: [K][(N+1)^2] GLL node coordinates; ``etoe, etof``: [K][4];
    ``c2q``: [K][nq1^2] or None.
    """

    def __init__(self, N, nq1, x, y, etoe, etof, c2q=None, tau_p=1.0, tau_u=1.0):
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.y = np.ascontiguousarray(y, dtype=np.float64)
        self.etoe = np.ascontiguousarray(etoe, dtype=np.int32)
        self.etof = np.ascontiguousarray(etof, dtype=np.int32)
        self.c2q = None if c2q is None else np.ascontiguousarray(c2q, dtype=np.float64)
        self.N, self.nq1, self.K = int(N), int(nq1), int(self.x.shape[0])
        self.tau_p, self.tau_u = float(tau_p), float(tau_u)
        # the library reads K rows of each array; it rejects an unsupported
        # degree or quadrature before reading any of them
        if 1 <= self.N <= WADG_MAX_N and self.N + 1 <= self.nq1 <= self.N + 3:
            K, np1 = self.K, (self.N + 1) ** 2
            want = {"x": (K, np1), "y": (K, np1), "etoe": (K, 4), "etof": (K, 4)}
            if self.c2q is not None:
                want["c2q"] = (K, self.nq1 ** 2)
            for name, shape in want.items():
                got = getattr(self, name).shape
                if got != shape:
                    raise ValueError(f"MeshDesc: {name} has shape {got}, expected {shape}")

    def struct(self):
        return wadg_mesh(
            self.N, self.nq1, self.K,
            self.x.ctypes.data_as(_c_double_p), self.y.ctypes.data_as(_c_double_p),
            self.etoe.ctypes.data_as(_c_int32_p), self.etof.ctypes.data_as(_c_int32_p),
            None if self.c2q is None else self.c2q.ctypes.data_as(_c_double_p),
            self.tau_p, self.tau_u)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("device tensors must be contiguous")
        return a.data_ptr()
    raise TypeError(f"cannot pass {type(a)} as a device pointer")


def _dev(a, nbytes, name, f64=True):
    """Device pointer of `a` for a call that reads or writes nbytes through
    it.  Tensors must be contiguous device tensors (float64 for states) of at
    least nbytes; raw integer pointers pass through unchecked, as in C."""
    if a is not None and not isinstance(a, int) and hasattr(a, "data_ptr"):
        dev = getattr(a, "device", None)
        if dev is not None and getattr(dev, "type", "cuda") != "cuda":
            raise ValueError(f"{name} must be a device tensor (it is on {dev})")
        if f64 and str(getattr(a, "dtype", "torch.float64")) != "torch.float64":
            raise ValueError(f"{name} must hold float64 values (it holds {a.dtype})")
        have = a.numel() * a.element_size()
        if have < nbytes:
            raise ValueError(f"{name} holds {have} bytes; this call needs {nbytes}")
    return _ptr(a)


def _need(fn, *args):
    """A size query for the checks above; 0 when the arguments are invalid
    (the call itself then reports them)."""
    try:
        return fn(*args)
    except WadgError:
        return 0


def _slice_bytes(ctx):
    return _need(wadg_state_doubles, ctx) * 8


def _stream(stream):
    if stream is None:
        try:
            import torch
            return torch.cuda.current_stream().cuda_stream
        except Exception:   # no torch / no device: the null stream
            return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------------ C names
def wadg_quadrature_points(mesh):
    Nq = mesh.nq1 * mesh.nq1
    xq = np.empty((mesh.K, Nq))
    yq = np.empty((mesh.K, Nq))
    m = mesh.struct()
    _check(LIB.wadg_quadrature_points(ctypes.byref(m), xq.ctypes.data_as(_c_double_p),
                                      yq.ctypes.data_as(_c_double_p)))
    return xq, yq


def wadg_geometry(mesh):
    Nq = mesh.nq1 * mesh.nq1
    vol = np.empty((6, Nq, mesh.K))
    face = np.empty((3, 4, mesh.nq1, mesh.K))
    m = mesh.struct()
    _check(LIB.wadg_geometry(ctypes.byref(m), vol.ctypes.data_as(_c_double_p),
                             face.ctypes.data_as(_c_double_p)))
    return vol, face


def wadg_cfl_number(mesh, dt, c2_scale=1.0):
    nu = ctypes.c_double()
    m = mesh.struct()
    _check(LIB.wadg_cfl_number(ctypes.byref(m), float(dt), float(c2_scale), ctypes.byref(nu)))
    return nu.value


def wadg_create(mesh, device=-1):
    h = ctypes.c_void_p()
    m = mesh.struct()
    _check(LIB.wadg_create(ctypes.byref(m), int(device), ctypes.byref(h)))
    return h


def wadg_destroy(ctx):
    LIB.wadg_destroy(ctx)


def wadg_state_doubles(ctx):
    n = ctypes.c_size_t()
    _check(LIB.wadg_state_doubles(ctx, ctypes.byref(n)))
    return n.value


def wadg_workspace_bytes(ctx, S):
    n = ctypes.c_size_t()
    _check(LIB.wadg_workspace_bytes(ctx, int(S), ctypes.byref(n)))
    return n.value


def wadg_rhs(ctx, Q, dQdt, S, stream=None):
    n = int(S) * _slice_bytes(ctx)
    _check(LIB.wadg_rhs(ctx, _dev(Q, n, "Q"), _dev(dQdt, n, "dQdt"), int(S), _stream(stream)))


def wadg_integrate(ctx, Q, work, S, dt, nsteps, stream=None):
    q = _dev(Q, int(S) * _slice_bytes(ctx), "Q")
    w = _dev(work, _need(wadg_workspace_bytes, ctx, S), "work", f64=False)
    _check(LIB.wadg_integrate(ctx, q, w, int(S), float(dt), int(nsteps), _stream(stream)))


def wadg_workspace_bytes_fp32(ctx, S):
    n = ctypes.c_size_t()
    _check(LIB.wadg_workspace_bytes_fp32(ctx, int(S), ctypes.byref(n)))
    return n.value


def wadg_integrate_fp32(ctx, Q, work, S, dt, nsteps, stream=None):
    q = _dev(Q, int(S) * _slice_bytes(ctx), "Q")
    w = _dev(work, _need(wadg_workspace_bytes_fp32, ctx, S), "work", f64=False)
    _check(LIB.wadg_integrate_fp32(ctx, q, w, int(S), float(dt), int(nsteps), _stream(stream)))


def wadg_parareal_workspace_bytes(ctx, S, fine_fp32=False):
    n = ctypes.c_size_t()
    _check(LIB.wadg_parareal_workspace_bytes(ctx, int(S), int(bool(fine_fp32)), ctypes.byref(n)))
    return n.value


def wadg_parareal(ctx, y0, U, work, S, dt, nsteps_fine, nsteps_coarse, max_iter, tol,
                  fine_fp32=False, stream=None):
    """Returns (iterations, last relative change)."""
    it = ctypes.c_int32()
    ch = ctypes.c_double()
    n1 = _slice_bytes(ctx)
    y0 = _dev(y0, n1, "y0")
    U = _dev(U, (int(S) + 1) * n1, "U")
    work = _dev(work, _need(wadg_parareal_workspace_bytes, ctx, S, fine_fp32), "work", f64=False)
    _check(LIB.wadg_parareal(ctx, y0, U, work, int(S), float(dt),
                             int(nsteps_fine), int(nsteps_coarse), int(max_iter), float(tol),
                             int(bool(fine_fp32)), ctypes.byref(it), ctypes.byref(ch),
                             _stream(stream)))
    return it.value, ch.value


def wadg_norms_workspace_bytes(ctx, S):
    n = ctypes.c_size_t()
    _check(LIB.wadg_norms_workspace_bytes(ctx, int(S), ctypes.byref(n)))
    return n.value


def _scratch(scratch, need, nbytes):
    """Device pointer and byte size of a scratch buffer: a tensor (its own
    size is passed, so the library refuses one that is too short) or a raw
    integer address taken to hold `nbytes` (or `need` if None), as in C."""
    if scratch is None:
        return None, 0
    if isinstance(scratch, int):
        return scratch, int(need if nbytes is None else nbytes)
    p = _dev(scratch, 0, "scratch", f64=False)
    return p, scratch.numel() * scratch.element_size()


def wadg_norms(ctx, A, B, S, scratch, stream=None, check_finite=True, scratch_bytes=None):
    out = np.empty((int(S), 4))
    n = int(S) * _slice_bytes(ctx)
    sp, sb = _scratch(scratch, _need(wadg_norms_workspace_bytes, ctx, S), scratch_bytes)
    st = LIB.wadg_norms(ctx, _dev(A, n, "A"), _dev(B, n, "B"), int(S), sp, sb,
                        out.ctypes.data_as(_c_double_p), _stream(stream))
    if st == WADG_E_NONFINITE and not check_finite:
        return out
    _check(st)
    return out


def wadg_norms_noalloc(ctx, A, B, S, stream=None, check_finite=True):
    out = np.empty((int(S), 4))
    n = int(S) * _slice_bytes(ctx)
    st = LIB.wadg_norms_noalloc(ctx, _dev(A, n, "A"), _dev(B, n, "B"), int(S),
                                out.ctypes.data_as(_c_double_p), _stream(stream))
    if st == WADG_E_NONFINITE and not check_finite:
        return out
    _check(st)
    return out


def wadg_l2_norms_workspace_bytes(ctx, S):
    n = ctypes.c_size_t()
    _check(LIB.wadg_l2_norms_workspace_bytes(ctx, int(S), ctypes.byref(n)))
    return n.value


def wadg_l2_norms(ctx, A, B, S, scratch, stream=None, check_finite=True, scratch_bytes=None):
    out = np.empty((int(S), 2))
    n = int(S) * _slice_bytes(ctx)
    sp, sb = _scratch(scratch, _need(wadg_l2_norms_workspace_bytes, ctx, S), scratch_bytes)
    st = LIB.wadg_l2_norms(ctx, _dev(A, n, "A"), _dev(B, n, "B"), int(S), sp, sb,
                           out.ctypes.data_as(_c_double_p), _stream(stream))
    if st == WADG_E_NONFINITE and not check_finite:
        return out
    _check(st)
    return out


def wadg_set_schedule(ctx, groups_per_tile, slices_per_tile=0):
    _check(LIB.wadg_set_schedule(ctx, int(groups_per_tile), int(slices_per_tile)))


def wadg_set_kernel(ctx, kernel):
    _check(LIB.wadg_set_kernel(ctx, int(kernel)))


def wadg_kernel_in_use(ctx, rhs=False, fp32=False):
    out = ctypes.c_int32()
    _check(LIB.wadg_kernel_in_use(ctx, 1 if rhs else 0, 1 if fp32 else 0, ctypes.byref(out)))
    return out.value


def wadg_set_c2_scale(ctx, scale):
    _check(LIB.wadg_set_c2_scale(ctx, float(scale)))


def wadg_adjoint_workspace_bytes(ctx, nsteps):
    out = ctypes.c_size_t()
    _check(LIB.wadg_adjoint_workspace_bytes(ctx, int(nsteps), ctypes.byref(out)))
    return out.value


def wadg_forward_checkpoints(ctx, chk, work, S, dt, nsteps, stream=None):
    c = _dev(chk, (int(S) + 1) * _slice_bytes(ctx), "chk")
    w = _dev(work, _need(wadg_adjoint_workspace_bytes, ctx, nsteps), "work", f64=False)
    _check(LIB.wadg_forward_checkpoints(ctx, c, w, int(S), float(dt), int(nsteps),
                                        _stream(stream)))


def wadg_adjoint(ctx, chk, seed, grad, work, S, dt, nsteps, stream=None):
    """Returns dJ_dscale (gamma dJ/dgamma); grad is written on the device."""
    out = ctypes.c_double()
    n1 = _slice_bytes(ctx)
    args = (_dev(chk, (int(S) + 1) * n1, "chk"), _dev(seed, n1, "seed"), _dev(grad, n1, "grad"),
            _dev(work, _need(wadg_adjoint_workspace_bytes, ctx, nsteps), "work", f64=False))
    _check(LIB.wadg_adjoint(ctx, *args, int(S), float(dt), int(nsteps), ctypes.byref(out),
                            _stream(stream)))
    return out.value


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_c_double_p)


_BATCH_NPROB = {}   # problems per live batch handle (host arrays are sized by it)


def _batch_nprob(b):
    return _BATCH_NPROB.get(getattr(b, "value", b))


def wadg_batch_create(meshes, S, device=-1):
    """meshes: list of MeshDesc (same N, nq1, tau); S: slices per problem."""
    s = np.ascontiguousarray(S, dtype=np.int32)
    if s.shape != (len(meshes),):
        raise ValueError("S must hold one slice count per mesh")
    arr = (wadg_mesh * len(meshes))(*[m.struct() for m in meshes])
    h = ctypes.c_void_p()
    _check(LIB.wadg_batch_create(arr, len(meshes), s.ctypes.data_as(_c_int32_p), int(device),
                                 ctypes.byref(h)))
    _BATCH_NPROB[h.value] = len(meshes)
    return h


def wadg_batch_destroy(b):
    LIB.wadg_batch_destroy(b)
    _BATCH_NPROB.pop(getattr(b, "value", b), None)


def _batch_dt(b, dt):
    d, dp = _f64(dt)
    n = _batch_nprob(b)
    if n is not None and d.size != n:
        raise ValueError(f"dt holds {d.size} values; the batch has {n} problems")
    return d, dp


def _batch_state(b, Q, work):
    wb = _need(wadg_batch_workspace_bytes, b)
    return _dev(Q, wb // 2, "Q"), _dev(work, wb, "work", f64=False)


def wadg_batch_layout(b, nprob):
    n = _batch_nprob(b)
    if n is not None and int(nprob) != n:
        raise ValueError(f"nprob is {nprob}; the batch has {n} problems")
    off = np.zeros(nprob + 1, dtype=np.int64)
    pack = np.zeros(nprob, dtype=np.int32)
    _check(LIB.wadg_batch_layout(b, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 pack.ctypes.data_as(_c_int32_p)))
    return off, pack


def wadg_batch_workspace_bytes(b):
    out = ctypes.c_size_t()
    _check(LIB.wadg_batch_workspace_bytes(b, ctypes.byref(out)))
    return out.value


def wadg_batch_integrate(b, Q, work, dt, nsteps, stream=None):
    d, dp = _batch_dt(b, dt)
    q, w = _batch_state(b, Q, work)
    _check(LIB.wadg_batch_integrate(b, q, w, dp, int(nsteps), _stream(stream)))


def wadg_batch_set_schedule(b, wg_per_cu, order):
    _check(LIB.wadg_batch_set_schedule(b, int(wg_per_cu), int(order)))


def wadg_batch_set_runs(b, run_slices):
    _check(LIB.wadg_batch_set_runs(b, int(run_slices)))


def wadg_batch_tune(b, Q, work, dt, reps=3, stream=None):
    """(wg_per_cu, order, run_slices, best_us) of the fastest candidate."""
    d, dp = _batch_dt(b, dt)
    q, w = _batch_state(b, Q, work)
    wg, order, runs, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(LIB.wadg_batch_tune(b, q, w, dp, int(reps), ctypes.byref(wg), ctypes.byref(order),
                               ctypes.byref(runs), ctypes.byref(us), _stream(stream)))
    return wg.value, order.value, runs.value, us.value


def wadg_batch_capture(b, Q, work, dt, nsteps):
    d, dp = _batch_dt(b, dt)
    q, w = _batch_state(b, Q, work)
    _check(LIB.wadg_batch_capture(b, q, w, dp, int(nsteps)))


def wadg_batch_replay(b, stream=None):
    _check(LIB.wadg_batch_replay(b, _stream(stream)))


def wadg_batch_release_graph(b):
    _check(LIB.wadg_batch_release_graph(b))


def pack_batch_problem(Qn, pack):
    """Natural [S][3][Np][K] states of one problem -> its packed tiled
    values ([ceil(S/P)] virtual slices of P side-by-side copies)."""
    Qn = np.asarray(Qn, dtype=np.float64)
    S, _, Np, K = Qn.shape
    P = int(pack)
    Sv = -(-S // P)
    q = np.zeros((Sv * P, 3, Np, K))
    q[:S] = Qn
    q = q.reshape(Sv, P, 3, Np, K).transpose(0, 2, 3, 1, 4).reshape(Sv, 3, Np, P * K)
    return tile_state(q).reshape(-1)


def unpack_batch_problem(vals, S, K, Np, pack):
    """Inverse of pack_batch_problem."""
    P = int(pack)
    Sv = -(-S // P)
    G = -(-(P * K) // TILE_LANES)
    q = untile_state(np.asarray(vals).reshape(Sv, G, 3, Np, TILE_LANES), P * K)
    q = q.reshape(Sv, 3, Np, P, K).transpose(0, 3, 1, 2, 4).reshape(Sv * P, 3, Np, K)
    return q[:S]


def wadg_status_string(status):
    return LIB.wadg_status_string(int(status)).decode()


def wadg_last_error():
    return LIB.wadg_last_error().decode()


# --------------------------------------------------------------- layout
def tile_state(Qn):
    """Natural layout [..., 3, Np, K] -> tiled [..., G, 3, Np, 64] (padding 0)."""
    Qn = np.asarray(Qn, dtype=np.float64)
    *lead, F, Np, K = Qn.shape
    G = (K + TILE_LANES - 1) // TILE_LANES
    pad = np.zeros(tuple(lead) + (F, Np, G * TILE_LANES))
    pad[..., :K] = Qn
    t = pad.reshape(tuple(lead) + (F, Np, G, TILE_LANES))
    return np.ascontiguousarray(np.moveaxis(t, -2, -4))


def untile_state(Qt, K):
    """Tiled [..., G, 3, Np, 64] -> natural [..., 3, Np, K]."""
    Qt = np.asarray(Qt)
    *lead, G, F, Np, L = Qt.shape
    n = np.moveaxis(Qt, -4, -2).reshape(tuple(lead) + (F, Np, G * L))
    return np.ascontiguousarray(n[..., :K])
