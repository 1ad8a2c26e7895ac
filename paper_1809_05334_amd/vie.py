"""Python binding of libvie (include/vie.h): argument marshalling only.

Device memory for the library's workspace comes from PyTorch (one uint8
tensor on the GPU) and work runs on PyTorch's current HIP stream; every step
of the method runs in the library's HIP kernels.  The binding refuses to run
without the built library (no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvie.so")

VIE_OK, VIE_EINVAL, VIE_ESTATE, VIE_ENOMEM, VIE_ENOCONV, VIE_EWOOD, VIE_ESINGULAR, VIE_EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
VIE_TE, VIE_TM = 0, 1
VIE_FP64, VIE_MIXED_FP32, VIE_GRID_FP64 = 0, 1, 2

_STATUS = {0: "VIE_OK", -1: "VIE_EINVAL", -2: "VIE_ESTATE", -3: "VIE_ENOMEM", -4: "VIE_ENOCONV",
           -5: "VIE_EWOOD", -6: "VIE_ESINGULAR", -7: "VIE_EDEVICE"}


class VieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("refine_steps", C.c_int),
                ("true_rel_residual", C.c_double), ("t_fill_ms", C.c_double),
                ("t_factor_ms", C.c_double), ("t_solve_ms", C.c_double), ("converged", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FillStats(C.Structure):
    _fields_ = [("t_fill_ms", C.c_double), ("t_far_ms", C.c_double), ("t_near_ms", C.c_double),
                ("t_face_ms", C.c_double), ("far_pairs", C.c_int64), ("near_pairs", C.c_int64),
                ("face_pairs", C.c_int64), ("far_launches", C.c_int64), ("point_pair_flops", C.c_double),
                ("far_flops", C.c_double), ("nimg", C.c_int), ("nmode", C.c_int), ("far_symmetric", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FactorStats(C.Structure):
    _fields_ = [("t_factor_ms", C.c_double), ("t_update_ms", C.c_double), ("update_flops", C.c_double),
                ("factor_flops", C.c_double), ("update_launches", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None

VIE_OPT_GRAPH_STEPS, VIE_OPT_MATVEC_ROWS, VIE_OPT_TRSV_CHUNK, VIE_OPT_TRSV_COOP, VIE_OPT_LU_PIVOT = 1, 2, 3, 4, 5
VIE_OPT_SYM_FILL = 6
VIE_OPT_PRECOND = 7


class Tuning(C.Structure):
    _fields_ = [("matvec_ms", C.c_double * 6), ("apply_ms", C.c_double * 4),
                ("matvec_rows", C.c_int), ("trsv_chunk", C.c_int)]

    def as_dict(self):
        return {"matvec_ms": list(self.matvec_ms), "apply_ms": list(self.apply_ms),
                "matvec_rows": self.matvec_rows, "trsv_chunk": self.trsv_chunk}


_SIGS = {
    "vie_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "vie_destroy": (C.c_int, [C.c_void_p]),
    "vie_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vie_mesh_upload": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                  C.c_int32, C.c_double, C.c_double]),
    "vie_num_unknowns": (C.c_int64, [C.c_void_p]),
    "vie_domain_ranges": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vie_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int, C.c_int]),
    "vie_bind_workspace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_int]),
    "vie_bind_static_workspace": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "vie_fill": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_int]),
    "vie_precond_factor": (C.c_int, [C.c_void_p]),
    "vie_solve": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_int, C.c_int, C.POINTER(SolveInfo)]),
    "vie_solve_pair": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_int, C.POINTER(SolveInfo)]),
    "vie_absorption": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vie_absorption_pol": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vie_absorption_per_tet": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "vie_sample_field": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "vie_last_error": (C.c_char_p, [C.c_void_p]),
    "vie_export_faces": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vie_read_Z": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "vie_read_rhs": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vie_read_solution": (C.c_int, [C.c_void_p, C.c_void_p]),
    "vie_read_solution_pol": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "vie_pgf_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "vie_residual_history": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "vie_get_fill_stats": (C.c_int, [C.c_void_p, C.POINTER(FillStats)]),
    "vie_get_factor_stats": (C.c_int, [C.c_void_p, C.POINTER(FactorStats)]),
    "vie_bench_matvec": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double)]),
    "vie_apply_Z": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "vie_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "vie_set_option": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "vie_get_option": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    "vie_autotune": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "vie_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "vie_batch_destroy": (C.c_int, [C.c_void_p]),
    "vie_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "vie_batch_workspace_bytes": (C.c_size_t, [C.c_int]),
    "vie_batch_bind": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "vie_batch_set_option": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "vie_batch_fill": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vie_batch_factor": (C.c_int, [C.c_void_p]),
    "vie_batch_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_void_p]),
}
VIE_BATCH_GRAPH = 1


def load():
    """Load libvie.so (built in-tree by __graft_entry__.build / build.py)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libvie.so is not built ({LIB_PATH}); run __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _LIB = lib
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Solver:
    """One context = one unit cell on one device stream (not thread-safe).
    Without `stream`, the context gets a new stream of its own."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        # a stream of its own by default (the null stream cannot be captured in a graph)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = C.c_void_p()
        rc = self.lib.vie_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != VIE_OK:
            raise VieError(rc, "vie_create failed (no HIP device?)")
        self.h = h
        self.ws = None
        self.ndom = 0
        self.nt = 0

    def _ck(self, rc, allow=()):
        if rc != VIE_OK and rc not in allow:
            raise VieError(rc, self.lib.vie_last_error(self.h).decode())
        return rc

    def set_stream(self, stream):
        """Run this context's work on `stream` (a torch.cuda.Stream) from now on."""
        self._ck(self.lib.vie_set_stream(self.h, C.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def close(self):
        if getattr(self, "h", None):
            self.lib.vie_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- setup
    def upload(self, verts, tets, tet_domain, ndom, a, b):
        v = np.ascontiguousarray(verts, np.float64)
        t = np.ascontiguousarray(tets, np.int32)
        d = np.ascontiguousarray(tet_domain, np.int32)
        self._ck(self.lib.vie_mesh_upload(self.h, _p(v), len(v), _p(t), len(t), _p(d), int(ndom), float(a), float(b)))
        self.ndom = int(ndom)
        self.nt = len(t)
        return self.num_unknowns()

    def upload_mesh(self, mesh):
        return self.upload(mesh.verts, mesh.tets, mesh.tet_domain, mesh.ndom, mesh.a, mesh.b)

    def num_unknowns(self):
        return int(self.lib.vie_num_unknowns(self.h))

    def domain_ranges(self):
        out = np.zeros(2 * self.ndom, np.int64)
        self._ck(self.lib.vie_domain_ranges(self.h, _p(out)))
        return out.reshape(-1, 2)

    def workspace_bytes(self, precision=VIE_FP64, restart=100):
        return int(self.lib.vie_workspace_bytes(self.h, precision, restart))

    def bind(self, precision=VIE_FP64, restart=100, workspace=None):
        nbytes = self.workspace_bytes(precision, restart)
        if nbytes == 0:
            raise VieError(VIE_EINVAL, "workspace size unavailable (precision/restart)")
        if workspace is None:
            # allocated on the context's stream, so torch's caching allocator
            # does not hand the block to another stream while it is in use
            with self.torch.cuda.stream(self.stream):
                workspace = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=f"cuda:{self.device}")
        ptr = workspace.data_ptr()
        off = (-ptr) % 256
        self._ck(self.lib.vie_bind_workspace(self.h, C.c_void_p(ptr + off), workspace.numel() - off, precision, restart))
        self.ws = workspace
        self.precision = precision
        self.restart = restart
        return nbytes

    def bind_static(self, precision=VIE_FP64, restart=100):
        """Bind the library's own per-device workspace (no allocation); the
        previous context holding it loses it."""
        self._ck(self.lib.vie_bind_static_workspace(self.h, precision, restart))
        self.ws = None
        self.precision = precision
        self.restart = restart
        return self.workspace_bytes(precision, restart)

    # -------------------------------------------------------------- method
    def fill(self, lam, theta, phi, eps, precision=None):
        e = np.ascontiguousarray(np.asarray(eps, np.complex128))
        if len(e) != self.nt:
            raise ValueError("eps must have one value per tetrahedron")
        p = self.precision if precision is None else precision
        self._ck(self.lib.vie_fill(self.h, float(lam), float(theta), float(phi), _p(e), p))

    def factor(self):
        self._ck(self.lib.vie_precond_factor(self.h))

    def solve(self, pol, tol=1e-12, max_iter=2000, restart=None, allow_noconv=False):
        info = SolveInfo()
        rc = self.lib.vie_solve(self.h, int(pol), float(tol), int(max_iter), int(restart or self.restart),
                                C.byref(info))
        self._ck(rc, allow=(VIE_ENOCONV,) if allow_noconv else ())
        d = info.as_dict()
        d["converged"] = bool(d["converged"])
        return d

    def solve_pair(self, tol=1e-12, max_iter=2000, restart=None, allow_noconv=False):
        """TE and TM in lockstep (shared passes over Z and the factors); returns [TE info, TM info]."""
        info = (SolveInfo * 2)()
        rc = self.lib.vie_solve_pair(self.h, float(tol), int(max_iter), int(restart or self.restart), info)
        self._ck(rc, allow=(VIE_ENOCONV,) if allow_noconv else ())
        out = [info[0].as_dict(), info[1].as_dict()]
        for d in out:
            d["converged"] = bool(d["converged"])
        return out

    def absorption(self, want_rt=True, pol=None):
        """Absorptance per domain (and R, T) of the last solution, or of polarisation `pol`."""
        A = np.zeros(self.ndom)
        R = C.c_double(); T = C.c_double()
        rp, tp = (C.byref(R), C.byref(T)) if want_rt else (None, None)
        if pol is None:
            self._ck(self.lib.vie_absorption(self.h, _p(A), rp, tp))
        else:
            self._ck(self.lib.vie_absorption_pol(self.h, int(pol), _p(A), rp, tp))
        return (A, R.value, T.value) if want_rt else A

    def absorption_per_tet(self, pol=None):
        """Each tetrahedron's share of the absorptance (mesh order) of the last
        solution, or of polarisation `pol`; a domain's shares add up to its
        absorptance."""
        out = np.zeros(self.nt)
        self._ck(self.lib.vie_absorption_per_tet(self.h, -1 if pol is None else int(pol), _p(out)))
        return out

    def sample_field(self, points, pol=None):
        """E/E0 at points [n, 3] (nm) inside the structure for the last solution
        (or polarisation `pol`): (e [n, 3] complex, tet [n]; -1 and e = 0
        outside every tetrahedron)."""
        p = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
        e = np.zeros((len(p), 3), np.complex128)
        tet = np.zeros(len(p), np.int32)
        self._ck(self.lib.vie_sample_field(self.h, -1 if pol is None else int(pol), _p(p), len(p), _p(e), _p(tet)))
        return e, tet

    # -------------------------------------------------------------- diagnostics
    def read_Z(self, rows, cols):
        r = np.ascontiguousarray(rows, np.int64); c = np.ascontiguousarray(cols, np.int64)
        out = np.zeros(len(r), np.complex128)
        self._ck(self.lib.vie_read_Z(self.h, _p(r), _p(c), len(r), _p(out)))
        return out

    def read_rhs(self):
        out = np.zeros(self.num_unknowns(), np.complex128)
        self._ck(self.lib.vie_read_rhs(self.h, _p(out)))
        return out

    def read_solution(self, pol=None):
        out = np.zeros(self.num_unknowns(), np.complex128)
        if pol is None:
            self._ck(self.lib.vie_read_solution(self.h, _p(out)))
        else:
            self._ck(self.lib.vie_read_solution_pol(self.h, int(pol), _p(out)))
        return out

    def pgf(self, delta):
        d = np.ascontiguousarray(delta, np.float64).reshape(-1, 3)
        out = np.zeros(len(d), np.complex128)
        self._ck(self.lib.vie_pgf_eval(self.h, _p(d), len(d), _p(out)))
        return out

    def export_faces(self):
        N = self.num_unknowns()
        fv = np.zeros(3 * N, np.int32); tp = np.zeros(N, np.int32); tm = np.zeros(N, np.int32); dm = np.zeros(N, np.int32)
        self._ck(self.lib.vie_export_faces(self.h, _p(fv), _p(tp), _p(tm), _p(dm)))
        return fv.reshape(-1, 3), tp, tm, dm

    def residual_history(self, cap=100000):
        h = np.zeros(cap)
        n = self.lib.vie_residual_history(self.h, _p(h), cap)
        return h[:max(0, n)]

    def fill_stats(self):
        st = FillStats()
        self._ck(self.lib.vie_get_fill_stats(self.h, C.byref(st)))
        return st.as_dict()

    def factor_stats(self):
        st = FactorStats()
        self._ck(self.lib.vie_get_factor_stats(self.h, C.byref(st)))
        return st.as_dict()

    def precond_apply(self, v):
        """z = M^{-1} v with the block-diagonal preconditioner of the last factor()."""
        vin = np.ascontiguousarray(v, np.complex128)
        out = np.zeros(self.num_unknowns(), np.complex128)
        self._ck(self.lib.vie_precond_apply(self.h, _p(vin), _p(out)))
        return out

    def set_option(self, option, value):
        self._ck(self.lib.vie_set_option(self.h, int(option), int(value)))

    def get_option(self, option):
        v = C.c_int()
        self._ck(self.lib.vie_get_option(self.h, int(option), C.byref(v)))
        return v.value

    def autotune(self, reps=5):
        """Time the matvec and triangular-solve variants, keep the fastest (needs factor())."""
        t = Tuning()
        self._ck(self.lib.vie_autotune(self.h, int(reps), C.byref(t)))
        return t.as_dict()

    def apply_Z(self, x):
        """y = Z x with the bound operator of the last fill."""
        xin = np.ascontiguousarray(x, np.complex128)
        if len(xin) != self.num_unknowns():
            raise ValueError("x must have one value per unknown")
        out = np.zeros(len(xin), np.complex128)
        self._ck(self.lib.vie_apply_Z(self.h, _p(xin), _p(out)))
        return out

    def bench_matvec(self, reps=10):
        ms = C.c_double()
        self._ck(self.lib.vie_bench_matvec(self.h, int(reps), C.byref(ms)))
        return ms.value


class Batch:
    """Fused solves of several cells (Solver objects with a mesh uploaded and
    a workspace bound, one precision): one fill launch per kernel family for
    all of them, one block factorisation over all their domains, and GMRES
    with every cell's Arnoldi step in one launch sequence.  Each cell then
    answers absorption() / read_solution() as after its own solve."""

    def __init__(self, solvers, device=0, stream=None, graph=True):
        import torch
        self.torch = torch
        self.lib = load()
        self.cells = list(solvers)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = C.c_void_p()
        rc = self.lib.vie_batch_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != VIE_OK:
            raise VieError(rc, "vie_batch_create failed")
        self.h = h
        n = len(self.cells)
        nbytes = int(self.lib.vie_batch_workspace_bytes(n))
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{device}")
        ptr = self.ws.data_ptr()
        off = (-ptr) % 256
        arr = (C.c_void_p * n)(*[s.h.value for s in self.cells])
        self._ck(self.lib.vie_batch_bind(self.h, arr, n, C.c_void_p(ptr + off), self.ws.numel() - off))
        for s in self.cells:
            s.stream = self.stream
        self._ck(self.lib.vie_batch_set_option(self.h, VIE_BATCH_GRAPH, 1 if graph else 0))

    def _ck(self, rc, allow=()):
        if rc != VIE_OK and rc not in allow:
            raise VieError(rc, self.lib.vie_batch_last_error(self.h).decode())
        return rc

    def fill(self, lams, thetas, phis, eps_list):
        n = len(self.cells)
        lam = np.ascontiguousarray(lams, np.float64)
        th = np.ascontiguousarray(thetas, np.float64)
        ph = np.ascontiguousarray(phis, np.float64)
        eps = [np.ascontiguousarray(np.asarray(e, np.complex128)) for e in eps_list]
        for s, e in zip(self.cells, eps):
            if len(e) != s.nt:
                raise ValueError("eps must have one value per tetrahedron of its cell")
        ptrs = (C.c_void_p * n)(*[e.ctypes.data for e in eps])
        self._ck(self.lib.vie_batch_fill(self.h, _p(lam), _p(th), _p(ph), ptrs))

    def factor(self):
        self._ck(self.lib.vie_batch_factor(self.h))

    def solve(self, pols, tol=1e-10, max_iter=2000, restart=100, allow_noconv=False):
        n = len(self.cells)
        pp = np.ascontiguousarray(pols, np.int32)
        info = (SolveInfo * n)()
        rc = self.lib.vie_batch_solve(self.h, _p(pp), float(tol), int(max_iter), int(restart), info)
        self._ck(rc, allow=(VIE_ENOCONV,) if allow_noconv else ())
        out = [info[i].as_dict() for i in range(n)]
        for d in out:
            d["converged"] = bool(d["converged"])
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.vie_batch_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
