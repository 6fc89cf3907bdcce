"""Python binding of libfm.so (include/fm.h): argument marshalling only.

Device buffers are torch tensors (float64, on the problem's device); streams
are torch streams.  Every computation runs in the HIP library; there is no
fallback path: if libfm.so is missing or fails to load, every call raises.
"""
import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfm.so")

FM_OK, FM_E_INVALID, FM_E_NOMEM, FM_E_HIP, FM_E_NOT_CONVERGED = 0, -1, -2, -3, -4
FM_E_BREAKDOWN, FM_E_PENCIL, FM_E_NONFINITE, FM_E_REJECTED, FM_E_BUSY = -5, -6, -7, -8, -9
STATUS_NAMES = {0: "FM_OK", -1: "FM_E_INVALID", -2: "FM_E_NOMEM", -3: "FM_E_HIP", -4: "FM_E_NOT_CONVERGED",
                -5: "FM_E_BREAKDOWN", -6: "FM_E_PENCIL", -7: "FM_E_NONFINITE", -8: "FM_E_REJECTED",
                -9: "FM_E_BUSY"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
KERNEL_CLASSES = ["matvec", "modez", "xy", "mdot", "mupdate", "finish", "restart", "coupling"]
MAPS = {"uniform": 0, "quadratic": 1, "pow": 2, "sin": 3}
PRECONDS = {"block_jacobi": 1, "coupled": 2}   # fm_prec_variant


class FmDim(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("n", ctypes.c_int), ("R", ctypes.c_double), ("map", ctypes.c_int)]


class FmDesc(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double * 3), ("charge", ctypes.c_double * 3), ("J", ctypes.c_int),
                ("tau", ctypes.c_int), ("x", FmDim * 3), ("y", FmDim * 3), ("z", FmDim * 3),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("nu", ctypes.c_double),
                ("vhat", ctypes.c_int), ("device", ctypes.c_int), ("precond", ctypes.c_int),
                ("exchange", ctypes.c_int), ("zhalf", ctypes.c_int), ("mode_fit_tol", ctypes.c_double)]


class FmSolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("rtol", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("prec", ctypes.c_int), ("x0_is_guess", ctypes.c_int), ("graphs", ctypes.c_int)]


class FmSolveResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("min_abs_denominator", ctypes.c_double), ("status", ctypes.c_int)]

    def as_dict(self):
        return {"iters": self.iters, "restarts": self.restarts, "rel_residual": self.rel_residual,
                "min_abs_denominator": self.min_abs_denominator, "status": STATUS_NAMES.get(self.status)}


class FmEigsOpts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int), ("ncv", ctypes.c_int), ("tol", ctypes.c_double),
                ("max_restarts", ctypes.c_int), ("inner", FmSolveOpts)]


class FmEigsInfo(ctypes.Structure):
    _fields_ = [("nconv", ctypes.c_int), ("restarts", ctypes.c_int), ("solves", ctypes.c_int),
                ("inner_iters", ctypes.c_longlong), ("inner_failures", ctypes.c_int)]


class FmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libfm.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2005_05398_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, cd, ci = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
        pd = ctypes.POINTER(ctypes.c_double)
        L.fm_last_error.restype = ctypes.c_char_p
        L.fm_create_problem.argtypes = [ctypes.POINTER(FmDesc), ctypes.POINTER(vp)]
        L.fm_destroy_problem.argtypes = [vp]
        L.fm_problem_info.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t), ci,
                                      ctypes.POINTER(ctypes.c_size_t)]
        L.fm_apply_operator.argtypes = [vp, ci, pd, vp, vp, vp]
        L.fm_apply_precond.argtypes = [vp, ci, pd, vp, vp, ci, vp]
        L.fm_solve.argtypes = [vp, ci, pd, vp, vp, ctypes.POINTER(FmSolveOpts), ctypes.POINTER(FmSolveResult), vp]
        L.fm_apply_mass.argtypes = [vp, ci, vp, vp, vp]
        L.fm_apply_operator_noalloc.argtypes = [vp, ci, pd, vp, vp, vp]
        L.fm_apply_operator_complex.argtypes = [vp, ci, pd, pd, vp, vp, vp]
        L.fm_apply_precond_complex.argtypes = [vp, ci, pd, pd, vp, vp, vp]
        L.fm_solve_complex.argtypes = [vp, ci, pd, pd, vp, vp, ctypes.POINTER(FmSolveOpts),
                                       ctypes.POINTER(FmSolveResult), vp]
        L.fm_eigs.argtypes = [vp, cd, ctypes.POINTER(FmEigsOpts), vp, pd, pd, pd, vp, ctypes.POINTER(FmEigsInfo),
                              vp]
        L.fm_profile.argtypes = [vp, ci]
        L.fm_profile_read.argtypes = [vp, ci, pd, ctypes.POINTER(ctypes.c_longlong), pd, pd]
        for f in ("fm_create_problem", "fm_destroy_problem", "fm_problem_info", "fm_apply_operator",
                  "fm_apply_precond", "fm_solve", "fm_profile", "fm_profile_read", "fm_apply_mass", "fm_eigs",
                  "fm_apply_operator_noalloc", "fm_apply_operator_complex", "fm_apply_precond_complex",
                  "fm_solve_complex"):
            getattr(L, f).restype = ci
        _lib = L
    return _lib


def _check(status):
    if status != FM_OK:
        raise FmError(status, lib().fm_last_error().decode())


def make_c_desc(desc, device=0):
    d = FmDesc()
    for i in range(3):
        d.mass[i] = desc["masses"][i]
        d.charge[i] = desc["charges"][i]
    d.J, d.tau = desc["J"], desc["tau"]
    for key in ("x", "y", "z"):
        arr = getattr(d, key)
        for a in range(3):
            dd = desc[key][a]
            arr[a].degree, arr[a].n = dd["degree"], dd["n"]
            arr[a].R = dd.get("R", 2.0)
            arr[a].map = MAPS[dd.get("map", "uniform")]
    d.x0, d.nu, d.vhat = desc["x0"], desc["nu"], desc.get("vhat", 0)
    d.y0 = desc["y0"] if math.isfinite(desc["y0"]) else float("inf")
    d.device = device
    d.precond = PRECONDS[desc.get("precond", "block_jacobi")]
    d.exchange = int(desc.get("exchange", 0))
    d.zhalf = int(desc.get("zhalf", 0))
    d.mode_fit_tol = float(desc.get("mode_fit_tol", 0.0))
    return d


def _energies(E):
    E = [float(e) for e in (E if hasattr(E, "__len__") else [E])]
    return (ctypes.c_double * len(E))(*E), len(E)


def _complex_energies(E):
    E = [complex(e) for e in (E if hasattr(E, "__len__") else [E])]
    n = len(E)
    return (ctypes.c_double * n)(*[e.real for e in E]), (ctypes.c_double * n)(*[e.imag for e in E]), n


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, n, name):
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


class Problem:
    """A problem handle: energy-independent factors resident on the device."""

    def __init__(self, desc, device=0):
        self._h = ctypes.c_void_p()
        self.desc = desc
        self.device = device
        _check(lib().fm_create_problem(ctypes.byref(make_c_desc(desc, device)), ctypes.byref(self._h)))
        n = ctypes.c_size_t()
        r = ctypes.c_size_t()
        _check(lib().fm_problem_info(self._h, ctypes.byref(n), ctypes.byref(r), 1, None))
        self.N = n.value
        self.bytes_resident = r.value

    def bytes_per_request(self, restart):
        b = ctypes.c_size_t()
        _check(lib().fm_problem_info(self._h, None, None, int(restart), ctypes.byref(b)))
        return b.value

    def close(self):
        if self._h:
            lib().fm_destroy_problem(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_operator(self, E, x, y, stream=None):
        Ec, nb = _energies(E)
        _check(lib().fm_apply_operator(self._h, nb, Ec, _ptr(x, nb * self.N, "x"), _ptr(y, nb * self.N, "y"),
                                       _stream(stream)))
        return y

    def apply_operator_noalloc(self, E, x, y, stream=None):
        """fm_apply_operator_noalloc: the operator with its scratch in the
        library's static device array (nothing allocated)."""
        Ec, nb = _energies(E)
        _check(lib().fm_apply_operator_noalloc(self._h, nb, Ec, _ptr(x, nb * self.N, "x"),
                                               _ptr(y, nb * self.N, "y"), _stream(stream)))
        return y

    def apply_operator_complex(self, E, x, y, stream=None):
        """Complex energies E; x, y: float64 tensors of len(E) * 2N ([request][re, im][N])."""
        Er, Ei, nb = _complex_energies(E)
        _check(lib().fm_apply_operator_complex(self._h, nb, Er, Ei, _ptr(x, 2 * nb * self.N, "x"),
                                               _ptr(y, 2 * nb * self.N, "y"), _stream(stream)))
        return y

    def apply_precond_complex(self, E, r, z, stream=None):
        Er, Ei, nb = _complex_energies(E)
        _check(lib().fm_apply_precond_complex(self._h, nb, Er, Ei, _ptr(r, 2 * nb * self.N, "r"),
                                              _ptr(z, 2 * nb * self.N, "z"), _stream(stream)))
        return z

    def solve_complex(self, E, b, x, restart=30, rtol=1e-10, max_iters=2000, x0_is_guess=False, stream=None,
                      raise_on_error=True, graphs=False):
        """fm_solve_complex: b, x float64 tensors of len(E) * 2N ([request][re, im][N]).
        Returns (status, [per-request result dicts])."""
        Er, Ei, nb = _complex_energies(E)
        opts = FmSolveOpts(int(restart), float(rtol), int(max_iters), PRECISIONS["fp64"], int(bool(x0_is_guess)),
                           int(bool(graphs)))
        res = (FmSolveResult * nb)()
        st = lib().fm_solve_complex(self._h, nb, Er, Ei, _ptr(b, 2 * nb * self.N, "b"), _ptr(x, 2 * nb * self.N, "x"),
                                    ctypes.byref(opts), res, _stream(stream))
        out = [r.as_dict() for r in res]
        if st != FM_OK and raise_on_error and st != FM_E_NOT_CONVERGED:
            raise FmError(st, lib().fm_last_error().decode())
        return st, out

    def apply_precond(self, E, r, z, prec="fp64", stream=None):
        Ec, nb = _energies(E)
        _check(lib().fm_apply_precond(self._h, nb, Ec, _ptr(r, nb * self.N, "r"), _ptr(z, nb * self.N, "z"),
                                      PRECISIONS[prec], _stream(stream)))
        return z

    def apply_mass(self, x, y, stream=None):
        """y = S x for a batch of vectors (x.numel() // N of them)."""
        nb = x.numel() // self.N
        _check(lib().fm_apply_mass(self._h, nb, _ptr(x, nb * self.N, "x"), _ptr(y, nb * self.N, "y"),
                                   _stream(stream)))
        return y

    def eigs(self, sigma, nev=2, ncv=20, tol=1e-10, max_restarts=50, restart=60, rtol=1e-10, max_iters=4000,
             prec="fp64", vectors=None, v0=None, stream=None, raise_on_error=True, graphs=False):
        """Energies nearest sigma by shift-invert Arnoldi.  vectors: None or a
        device tensor of nev * N doubles.  Returns (status, energies (complex,
        nearest first), Ritz residuals, info dict)."""
        opts = FmEigsOpts(int(nev), int(ncv), float(tol), int(max_restarts),
                          FmSolveOpts(int(restart), float(rtol), int(max_iters), PRECISIONS[prec], 0,
                                      int(bool(graphs))))
        Er = (ctypes.c_double * nev)()
        Ei = (ctypes.c_double * nev)()
        rs = (ctypes.c_double * nev)()
        info = FmEigsInfo()
        vp = _ptr(vectors, nev * self.N, "vectors") if vectors is not None else None
        v0p = _ptr(v0, self.N, "v0") if v0 is not None else None
        st = lib().fm_eigs(self._h, float(sigma), ctypes.byref(opts), v0p, Er, Ei, rs, vp, ctypes.byref(info),
                           _stream(stream))
        if st != FM_OK and raise_on_error and st != FM_E_NOT_CONVERGED:
            raise FmError(st, lib().fm_last_error().decode())
        E = [complex(Er[i], Ei[i]) for i in range(nev)]
        inf = {"nconv": info.nconv, "restarts": info.restarts, "solves": info.solves,
               "inner_iters": info.inner_iters, "inner_failures": info.inner_failures}
        return st, E, list(rs), inf

    def profile(self, enable=True):
        """Enable (and reset) or disable per-kernel-class timing."""
        _check(lib().fm_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """{class: {"ms", "launches", "bytes", "flops"}} accumulated since profile(True)."""
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            ms, n, by, fl = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
            _check(lib().fm_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by),
                                         ctypes.byref(fl)))
            out[name] = {"ms": ms.value, "launches": n.value, "bytes": by.value, "flops": fl.value}
        return out

    def solve(self, E, b, x, restart=30, rtol=1e-10, max_iters=2000, prec="fp64", x0_is_guess=False,
              stream=None, raise_on_error=True, graphs=False):
        """Returns (status, [per-request result dicts])."""
        Ec, nb = _energies(E)
        opts = FmSolveOpts(int(restart), float(rtol), int(max_iters), PRECISIONS[prec], int(bool(x0_is_guess)),
                           int(bool(graphs)))
        res = (FmSolveResult * nb)()
        st = lib().fm_solve(self._h, nb, Ec, _ptr(b, nb * self.N, "b"), _ptr(x, nb * self.N, "x"),
                            ctypes.byref(opts), res, _stream(stream))
        out = [r.as_dict() for r in res]
        if st != FM_OK and raise_on_error and st != FM_E_NOT_CONVERGED:
            raise FmError(st, lib().fm_last_error().decode())
        return st, out


# -- host-only inspection (include/fm_host.h) --------------------------------

def _host_sigs(L):
    if getattr(L, "_host_sigs", False):
        return
    pd, ci = ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.fm_host_basis.argtypes = [ctypes.POINTER(FmDim), ci, pd, pd, pd, pd]
    L.fm_host_pencil.argtypes = [ci, pd, pd, pd, pd, pd, pd, ctypes.POINTER(ctypes.c_byte), pd]
    L.fm_host_setup_check.argtypes = [ctypes.POINTER(FmDesc), pd, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_size_t)]
    L.fm_host_coupling.argtypes = [ctypes.POINTER(FmDesc), pd, pd, ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_int)]
    L.fm_host_precond.argtypes = [ctypes.POINTER(FmDesc), ctypes.c_double, pd, pd]
    L.fm_host_slice_eigenvalues.argtypes = [ctypes.POINTER(FmDesc), ci, ci, pd, pd, pd, pd]
    for f in ("fm_host_basis", "fm_host_pencil", "fm_host_setup_check", "fm_host_coupling", "fm_host_precond",
              "fm_host_slice_eigenvalues"):
        getattr(L, f).restype = ci
    L._host_sigs = True


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def host_basis(dim, is_z):
    """(points, S, D1, D2) of one 1D basis as built by the library."""
    import numpy as np
    L = lib()
    _host_sigs(L)
    d = FmDim(dim["degree"], dim["n"], dim.get("R", 2.0), MAPS[dim.get("map", "uniform")])
    n = dim["n"]
    pts, S, D1, D2 = np.zeros(n), np.zeros((n, n)), np.zeros((n, n)), np.zeros((n, n))
    _check(L.fm_host_basis(ctypes.byref(d), int(is_z), _dptr(pts), _dptr(S), _dptr(D1), _dptr(D2)))
    return pts, S, D1, D2


def host_pencil(A1, A2):
    """(Wbar, W, lre, lim, type, err) of D(A1, A2) as computed by the library."""
    import numpy as np
    L = lib()
    _host_sigs(L)
    n = A1.shape[0]
    A1 = np.ascontiguousarray(A1, dtype=np.float64)
    A2 = np.ascontiguousarray(A2, dtype=np.float64)
    Wb, W = np.zeros((n, n)), np.zeros((n, n))
    lre, lim, err = np.zeros(n), np.zeros(n), np.zeros(1)
    ty = np.zeros(n, dtype=np.int8)
    _check(L.fm_host_pencil(n, _dptr(A1), _dptr(A2), _dptr(Wb), _dptr(W), _dptr(lre), _dptr(lim),
                            ty.ctypes.data_as(ctypes.POINTER(ctypes.c_byte)), _dptr(err)))
    return Wb, W, lre, lim, ty, float(err[0])


def host_setup_check(desc):
    """(max_err, complex_pairs, N) of the host factor build."""
    L = lib()
    _host_sigs(L)
    err = ctypes.c_double()
    pairs = ctypes.c_int()
    n = ctypes.c_size_t()
    _check(L.fm_host_setup_check(ctypes.byref(make_c_desc(desc)), ctypes.byref(err), ctypes.byref(pairs),
                                 ctypes.byref(n)))
    return err.value, pairs.value, n.value


def host_coupling(desc, x=None):
    """(C x or None, number of coupling pairs, number of cell tasks): the
    coupling term evaluated on the host from the library's grouped pairs."""
    import numpy as np
    L = lib()
    _host_sigs(L)
    npairs = ctypes.c_longlong()
    ntasks = ctypes.c_int()
    y = None
    if x is not None:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        _check(L.fm_host_coupling(ctypes.byref(make_c_desc(desc)), _dptr(x), _dptr(y), ctypes.byref(npairs),
                                  ctypes.byref(ntasks)))
    else:
        _check(L.fm_host_coupling(ctypes.byref(make_c_desc(desc)), None, None, ctypes.byref(npairs),
                                  ctypes.byref(ntasks)))
    return y, npairs.value, ntasks.value


# -- serving (fm_server_*) ----------------------------------------------------

def host_precond(desc, E, r):
    """z = L(E)^-1 r for one request, applied on the host from the library's
    factor tables (set-up check; small problems only)."""
    import numpy as np
    L = lib()
    _host_sigs(L)
    r = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros_like(r)
    _check(L.fm_host_precond(ctypes.byref(make_c_desc(desc)), float(E), _dptr(r), _dptr(z)))
    return z


def host_slice_eigenvalues(desc, alpha, slot):
    """(lx_re, lx_im, ly_re, ly_im) of one x-y slice of the preconditioner."""
    import numpy as np
    L = lib()
    _host_sigs(L)
    nx, ny = desc["x"][alpha]["n"], desc["y"][alpha]["n"]
    out = [np.zeros(nx), np.zeros(nx), np.zeros(ny), np.zeros(ny)]
    _check(L.fm_host_slice_eigenvalues(ctypes.byref(make_c_desc(desc)), int(alpha), int(slot), *[_dptr(a) for a in out]))
    return tuple(out)


class FmRequestResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("restart", ctypes.c_int)]


def _server_sigs(L):
    if getattr(L, "_server_sigs", False):
        return
    vp, ci = ctypes.c_void_p, ctypes.c_int
    L.fm_server_create.argtypes = [ctypes.c_size_t, ci, ci, ctypes.POINTER(vp)]
    L.fm_submit.argtypes = [vp, ctypes.POINTER(FmDesc), ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(FmSolveOpts), ctypes.c_uint64]
    L.fm_poll.argtypes = [vp, ctypes.POINTER(FmRequestResult), ci, ctypes.POINTER(ci), ci]
    L.fm_server_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ci),
                                  ctypes.POINTER(ctypes.c_longlong)]
    L.fm_server_destroy.argtypes = [vp]
    for f in ("fm_server_create", "fm_submit", "fm_poll", "fm_server_stats", "fm_server_destroy"):
        getattr(L, f).restype = ci
    L._server_sigs = True


class Server:
    """Continuous-batching solve server (host buffers in, host buffers out)."""

    def __init__(self, hbm_budget_bytes, max_batch=8, device=0):
        L = lib()
        _server_sigs(L)
        self._h = ctypes.c_void_p()
        _check(L.fm_server_create(int(hbm_budget_bytes), int(max_batch), int(device), ctypes.byref(self._h)))
        self._keep = {}

    def submit(self, desc, E, b, x, tag, restart=60, rtol=1e-10, max_iters=4000, prec="fp64", graphs=True):
        """b, x: contiguous float64 numpy arrays of N; x is written when the result is polled."""
        import numpy as np
        assert b.dtype == np.float64 and x.dtype == np.float64 and b.flags.c_contiguous and x.flags.c_contiguous
        opts = FmSolveOpts(int(restart), float(rtol), int(max_iters), PRECISIONS[prec], 0, int(bool(graphs)))
        self._keep[int(tag)] = (b, x)
        _check(lib().fm_submit(self._h, ctypes.byref(make_c_desc(desc)), float(E), _dptr(b), _dptr(x),
                               ctypes.byref(opts), ctypes.c_uint64(int(tag))))

    def poll(self, block=False, max_results=256):
        buf = (FmRequestResult * max_results)()
        n = ctypes.c_int()
        _check(lib().fm_poll(self._h, buf, max_results, ctypes.byref(n), int(bool(block))))
        out = []
        for i in range(n.value):
            r = buf[i]
            self._keep.pop(int(r.tag), None)
            out.append({"tag": int(r.tag), "status": STATUS_NAMES.get(r.status, r.status), "iters": r.iters,
                        "rel_residual": r.rel_residual, "t_submit": r.t_submit, "t_start": r.t_start,
                        "t_done": r.t_done, "restart": r.restart})
        return out

    def stats(self):
        b, l, o = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_longlong()
        _check(lib().fm_server_stats(self._h, ctypes.byref(b), ctypes.byref(l), ctypes.byref(o)))
        return {"bytes_in_use": b.value, "lanes": l.value, "outstanding": o.value}

    def close(self):
        if self._h:
            lib().fm_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

