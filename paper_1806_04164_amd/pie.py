"""Python binding of libpie (same names as the C ABI; marshalling only).

Every step of the computation runs in libpie's HIP kernels; this module only
turns numpy arrays and torch device tensors into pointers and sizes.  There
is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import PIE_FP32, PIE_FP64, check, lib  # noqa: F401


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Mesh:
    """pie_mesh: RWG/pulse tables of a closed triangulated surface."""

    def __init__(self, V, T):
        self.V = np.ascontiguousarray(V, dtype=np.float64)
        self.T = np.ascontiguousarray(T, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib().pie_mesh_create(_ptr(self.V), self.V.shape[0], _ptr(self.T), self.T.shape[0],
                                    ctypes.byref(h)))
        self.h = h

    def __del__(self, _destroy=lib().pie_mesh_destroy):
        # the destroy function is bound at definition time: it stays callable
        # while the interpreter tears modules down
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    @classmethod
    def icosphere(cls, subdiv: int, radius: float, jitter: float = 0.0, seed: int = 0) -> "Mesh":
        """The library's icosphere generator (pie_mesh_icosphere)."""
        h = ctypes.c_void_p()
        check(lib().pie_mesh_icosphere(int(subdiv), float(radius), float(jitter), int(seed), ctypes.byref(h)))
        self = cls.__new__(cls)
        self.h = h
        self.V, self.T = self.geometry()
        return self

    def geometry(self):
        """(V [nv, 3] float64, T [nt, 3] int32) as held by the library."""
        nv, nt = ctypes.c_int64(), ctypes.c_int64()
        check(lib().pie_mesh_geometry(self.h, ctypes.byref(nv), ctypes.byref(nt), None, None))
        V = np.zeros((nv.value, 3), np.float64)
        T = np.zeros((nt.value, 3), np.int32)
        check(lib().pie_mesh_geometry(self.h, None, None, _ptr(V), _ptr(T)))
        return V, T

    def sizes(self):
        ne, nt = ctypes.c_int64(), ctypes.c_int64()
        check(lib().pie_mesh_sizes(self.h, ctypes.byref(ne), ctypes.byref(nt)))
        return ne.value, nt.value

    @property
    def N(self):
        ne, nt = self.sizes()
        return ne + nt

    def edges(self):
        ne, _ = self.sizes()
        e = np.zeros((ne, 2), np.int32)
        t = np.zeros((ne, 2), np.int32)
        f = np.zeros((ne, 2), np.int32)
        check(lib().pie_mesh_edges(self.h, _ptr(e), _ptr(t), _ptr(f)))
        return e, t, f


class Tree:
    """pie_tree: octree with near and interaction lists."""

    def __init__(self, mesh: Mesh, levels: int):
        self.mesh = mesh
        self.L = levels
        h = ctypes.c_void_p()
        check(lib().pie_tree_build(mesh.h, levels, ctypes.byref(h)))
        self.h = h

    def __del__(self, _destroy=lib().pie_tree_destroy):
        # the destroy function is bound at definition time: it stays callable
        # while the interpreter tears modules down
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def query(self, what: str, level: int = 0) -> np.ndarray:
        code = _lib.TQ[what]
        n = ctypes.c_int64()
        check(lib().pie_tree_query(self.h, code, level, ctypes.byref(n), None))
        if what == "NBOX":
            return np.array(n.value)
        out = np.zeros(n.value, np.int64)
        check(lib().pie_tree_query(self.h, code, level, ctypes.byref(n), _ptr(out)))
        return out


def _stream(stream):
    if stream is None:
        try:
            import torch
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            return None
    return ctypes.c_void_p(stream)


def _dev(t, N=None, R=None):
    """Device pointer of a contiguous complex128 torch tensor [N,R]."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise TypeError("expected a contiguous complex128 tensor on the GPU")
    if N is not None and t.shape[0] != N:
        raise ValueError(f"expected {N} rows, got {t.shape[0]}")
    if R is not None and (t.dim() == 1 and R != 1 or t.dim() == 2 and t.shape[1] != R):
        raise ValueError("column count mismatch")
    return ctypes.c_void_p(t.data_ptr())


class Graph:
    """pie_graph: one captured MVM of an operator on fixed x and y tensors,
    replayed with launch().  Keeps the operator and tensors alive."""

    def __init__(self, op, x, y, adjoint=False):
        R = op._R(x)
        self.op, self.x, self.y = op, x, y
        h = ctypes.c_void_p()
        check(lib().pie_graph_create(op.h, _dev(x, op.N), _dev(y, op.N, R), R, int(adjoint), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        check(lib().pie_graph_launch(self.h, _stream(stream)))
        return self.y

    def __del__(self, _destroy=lib().pie_graph_destroy):
        # the destroy function is bound at definition time: it stays callable
        # while the interpreter tears modules down
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Batch:
    """pie_batch: the MVMs y_i = Z_i x_i (or Z_i^H x_i) of several distinct
    operators in one call, each object on its own stream so that their
    kernels run concurrently.  Keeps the operators alive."""

    def __init__(self, ops):
        n = len(ops)
        if n == 0:
            raise ValueError("empty batch")
        self.ops = list(ops)
        P = ctypes.c_void_p
        hops = (P * n)(*[op.h.value for op in ops])
        h = P()
        check(lib().pie_batch_create(hops, n, ctypes.byref(h)))
        self.h = h

    def matvec(self, xs, ys=None, adjoint=False, stream=None):
        import torch
        n = len(self.ops)
        if len(xs) != n or (ys is not None and len(ys) != n):
            raise ValueError("one x (and y) per operator")
        if ys is None:
            ys = [torch.empty_like(x) for x in xs]
        P = ctypes.c_void_p
        Rs = [op._R(x) for op, x in zip(self.ops, xs)]
        hx = (P * n)(*[_dev(x, op.N).value for op, x in zip(self.ops, xs)])
        hy = (P * n)(*[_dev(y, op.N, R).value for op, y, R in zip(self.ops, ys, Rs)])
        hr = (ctypes.c_int64 * n)(*Rs)
        check(lib().pie_batch_matvec(self.h, hx, hy, hr, int(adjoint), _stream(stream)))
        return ys

    def __del__(self, _destroy=lib().pie_batch_destroy):
        # the destroy function is bound at definition time: it stays callable
        # while the interpreter tears modules down
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class BatchGraph:
    """pie_graph of an uneven batch: the MVMs y_i = Z_i x_i of several
    distinct operators captured one after another into one graph; launch()
    runs them all.  Keeps the operators and tensors alive."""

    def __init__(self, ops, xs, ys, adjoint=False):
        n = len(ops)
        if not (n == len(xs) == len(ys)) or n == 0:
            raise ValueError("ops, xs and ys must have the same non-zero length")
        self.ops, self.xs, self.ys = list(ops), list(xs), list(ys)
        P = ctypes.c_void_p
        Rs = [op._R(x) for op, x in zip(ops, xs)]
        hops = (P * n)(*[op.h.value for op in ops])
        hx = (P * n)(*[_dev(x, op.N).value for op, x in zip(ops, xs)])
        hy = (P * n)(*[_dev(y, op.N, R).value for op, y, R in zip(ops, ys, Rs)])
        hr = (ctypes.c_int64 * n)(*Rs)
        h = P()
        check(lib().pie_graph_create_batch(hops, n, hx, hy, hr, int(adjoint), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        check(lib().pie_graph_launch(self.h, _stream(stream)))
        return self.ys

    def __del__(self, _destroy=lib().pie_graph_destroy):
        # the destroy function is bound at definition time: it stays callable
        # while the interpreter tears modules down
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Operator:
    """pie_op: the PIE operator (near field + MLFMA far field) on the GPU."""

    def __init__(self, mesh: Mesh, tree: Tree, freq: float, near_prec=PIE_FP64, far_prec=PIE_FP64,
                 tau=0, x=0.0, n_theta=0, n_phi=0, max_rhs=1, flags=0, stream=None):
        self.mesh, self.tree = mesh, tree
        o = _lib.pie_options()
        lib().pie_options_default(ctypes.byref(o))
        o.near_prec, o.far_prec, o.tau, o.x = near_prec, far_prec, tau, x
        o.n_theta, o.n_phi, o.max_rhs, o.flags = n_theta, n_phi, max_rhs, flags
        h = ctypes.c_void_p()
        check(lib().pie_operator_create(mesh.h, tree.h, float(freq), ctypes.byref(o), _stream(stream),
                                        ctypes.byref(h)))
        self.h = h
        self.N = self.info("N")
        self.max_rhs = max_rhs

    def __del__(self, _destroy=lib().pie_operator_destroy):
        # the destroy function is bound at definition time: it stays callable
        # while the interpreter tears modules down
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None

    def info(self, what: str) -> int:
        v = ctypes.c_int64()
        check(lib().pie_operator_info(self.h, _lib.OI[what], ctypes.byref(v)))
        return v.value

    def tau_level(self, l: int) -> int:
        """Truncation number of Eq. (5) at level l (PIE_OI_TAU_LEVEL)."""
        v = ctypes.c_int64()
        check(lib().pie_operator_info(self.h, 100 + int(l), ctypes.byref(v)))
        return v.value

    def level(self, l: int):
        s, k, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(lib().pie_operator_level(self.h, l, ctypes.byref(s), ctypes.byref(k), ctypes.byref(d)))
        return s.value, k.value, d.value

    def profile(self, on=True):
        check(lib().pie_profile_enable(self.h, int(on)))

    def profile_read(self):
        ms = np.zeros(len(_lib.STAGES))
        n = np.zeros(len(_lib.STAGES), np.int64)
        check(lib().pie_profile_read(self.h, _ptr(ms), _ptr(n)))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(_lib.STAGES)}

    def _R(self, x):
        return 1 if x.dim() == 1 else x.shape[1]

    @property
    def schedule(self) -> dict:
        sc = _lib.pie_schedule()
        check(lib().pie_schedule_get(self.h, ctypes.byref(sc)))
        return {"near_fork": sc.near_fork, "il_fork": sc.il_fork, "max_chunk": sc.max_chunk}

    @schedule.setter
    def schedule(self, d: dict):
        cur = self.schedule
        cur.update(d)
        sc = _lib.pie_schedule(1, cur["near_fork"], cur["il_fork"], cur["max_chunk"])
        check(lib().pie_schedule_set(self.h, ctypes.byref(sc)))

    def autotune(self, x, y=None, reps=10, stream=None):
        """Times every schedule on x (R = its columns), keeps the fastest;
        returns (schedule dict, ms per MVM)."""
        import torch
        R = self._R(x)
        if y is None:
            y = torch.empty_like(x)
        sc, ms = _lib.pie_schedule(), ctypes.c_double()
        check(lib().pie_autotune(self.h, _dev(x, self.N), _dev(y, self.N, R), R, int(reps), _stream(stream),
                                 ctypes.byref(sc), ctypes.byref(ms)))
        return {"near_fork": sc.near_fork, "il_fork": sc.il_fork, "max_chunk": sc.max_chunk}, ms.value

    def graph(self, x, y, adjoint=False):
        """Captures y = Z x (fixed tensors) into a HIP graph; see Graph."""
        return Graph(self, x, y, adjoint)

    def matvec(self, x, y=None, adjoint=False, stream=None):
        import torch
        R = self._R(x)
        if y is None:
            y = torch.empty_like(x)
        check(lib().pie_matvec(self.h, _dev(x, self.N), _dev(y, self.N, R), R, int(adjoint), _stream(stream)))
        return y

    def matvec_near(self, x, y=None, stream=None):
        import torch
        R = self._R(x)
        if y is None:
            y = torch.empty_like(x)
        check(lib().pie_matvec_near(self.h, _dev(x, self.N), _dev(y, self.N, R), R, _stream(stream)))
        return y

    def matvec_far(self, x, y=None, stream=None):
        import torch
        R = self._R(x)
        if y is None:
            y = torch.empty_like(x)
        check(lib().pie_matvec_far(self.h, _dev(x, self.N), _dev(y, self.N, R), R, _stream(stream)))
        return y

    def rhs_planewave(self, khat, pol, amp, gauge=0, b=None, stream=None):
        import torch
        khat = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
        pol = np.ascontiguousarray(np.atleast_2d(pol), np.float64)
        amp = np.ascontiguousarray(np.atleast_1d(amp), np.complex128)
        R = khat.shape[0]
        if b is None:
            b = torch.empty((self.N, R), dtype=torch.complex128, device="cuda")
        check(lib().pie_rhs_planewave(self.h, R, _ptr(khat), _ptr(pol), _ptr(amp), gauge,
                                      _dev(b, self.N, R), _stream(stream)))
        return b

    def solve(self, b, x=None, res_op=None, tol=1e-6, restart=100, maxit=1000, refine=1,
              inner_tol=0.0, adjoint=False, precond=False, stream=None):
        import torch
        R = self._R(b)
        o = _lib.pie_solve_opts()
        lib().pie_solve_opts_default(ctypes.byref(o))
        o.tol, o.restart, o.maxit, o.refine, o.inner_tol = tol, restart, maxit, refine, inner_tol
        o.adjoint = int(adjoint)
        o.precond = int(precond)
        o.use_x0 = 0 if x is None else 1
        if x is None:
            x = torch.zeros_like(b)
        info = _lib.pie_solve_info()
        st = lib().pie_solve(self.h, res_op.h if res_op is not None else None, _dev(b, self.N),
                             _dev(x, self.N, R), R, ctypes.byref(o), ctypes.byref(info), _stream(stream))
        check(st)
        return x, {"iterations": info.iterations, "refinements": info.refinements,
                   "rel_residual": info.rel_residual, "converged": st == 0}

    def precond_apply(self, x, y=None, stream=None):
        """pie_precond_apply: y = blockdiag(Z_bb)^-1 x."""
        import torch
        R = self._R(x)
        if y is None:
            y = torch.empty_like(x)
        check(lib().pie_precond_apply(self.h, _dev(x, self.N, R), _dev(y, self.N, R), R, _stream(stream)))
        return y

    def charge(self, khat, pol, amp, x=None, gauge=0, tol=1e-6, restart=100, maxit=1000, refine=1,
               inner_tol=0.0, stream=None):
        """pie_charge: sigma = n.grad(Phi) [T,R] from Eq. (3) and, given the
        PIE solution x [N,R], the charge density rho [T,R]."""
        import torch
        khat = np.ascontiguousarray(np.atleast_2d(khat), np.float64)
        pol = np.ascontiguousarray(np.atleast_2d(pol), np.float64)
        amp = np.ascontiguousarray(np.atleast_1d(amp), np.complex128)
        R = khat.shape[0]
        T = self.mesh.sizes()[1]
        o = _lib.pie_solve_opts()
        lib().pie_solve_opts_default(ctypes.byref(o))
        o.tol, o.restart, o.maxit, o.refine, o.inner_tol = tol, restart, maxit, refine, inner_tol
        sigma = torch.empty((T, R), dtype=torch.complex128, device="cuda")
        rho = torch.empty((T, R), dtype=torch.complex128, device="cuda") if x is not None else None
        info = _lib.pie_solve_info()
        st = lib().pie_charge(self.h, R, _ptr(khat), _ptr(pol), _ptr(amp), gauge,
                              _dev(x, self.N, R) if x is not None else None,
                              ctypes.c_void_p(sigma.data_ptr()),
                              ctypes.c_void_p(rho.data_ptr()) if rho is not None else None,
                              ctypes.byref(o), ctypes.byref(info), _stream(stream))
        check(st)
        return sigma, rho, {"iterations": info.iterations, "refinements": info.refinements,
                            "rel_residual": info.rel_residual, "converged": st == 0}

    def farfield(self, x, dirs, stream=None):
        import torch
        R = self._R(x)
        dirs = np.ascontiguousarray(np.atleast_2d(dirs), np.float64)
        F = torch.empty((R, dirs.shape[0], 3), dtype=torch.complex128, device="cuda")
        check(lib().pie_farfield(self.h, _dev(x, self.N), R, _ptr(dirs), dirs.shape[0],
                                 ctypes.c_void_p(F.data_ptr()), _stream(stream)))
        return F

    def farfield_adjoint(self, gF, dirs, stream=None):
        import torch
        if not (gF.is_cuda and gF.dtype == torch.complex128 and gF.is_contiguous() and gF.dim() == 3):
            raise TypeError("gF must be a contiguous complex128 [R, nd, 3] GPU tensor")
        R = gF.shape[0]
        dirs = np.ascontiguousarray(np.atleast_2d(dirs), np.float64)
        gx = torch.empty((self.N, R), dtype=torch.complex128, device="cuda")
        check(lib().pie_farfield_adjoint(self.h, ctypes.c_void_p(gF.data_ptr()), R, _ptr(dirs), dirs.shape[0],
                                         ctypes.c_void_p(gx.data_ptr()), _stream(stream)))
        return gx
