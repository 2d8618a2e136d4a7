"""ctypes binding of libilu (include/ilu.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "include", "ilu.h")

STORED_F64, SURR_F64, SURR_F32, STORED_SGS = 0, 1, 2, 3
SCHED_AUTO, SCHED_PLANE, SCHED_DATAFLOW = 0, 1, 2
A_EXACT, A_SURROGATE = 0, 1
BOUNDARY_V2, BOUNDARY_V1 = 0, 1
OVERLAP_OFF, OVERLAP_ON, OVERLAP_FUSED = 0, 1, 2
COEFF_CONST, COEFF_SINPROD, COEFF_EXPSINCOS, COEFF_POLY = 0, 1, 2, 3


def library_path() -> str:
    return os.path.join(HERE, "libilu.so")


class ilu_tet_desc(ctypes.Structure):
    _fields_ = [("vertex", ctypes.c_double * 12), ("level", ctypes.c_int32), ("coeff_kind", ctypes.c_int32),
                ("coeff_param", ctypes.c_double * 4)]


class ilu_opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("degree", ctypes.c_int32 * 3), ("sample_stride", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("tile", ctypes.c_int32 * 2), ("a_mode", ctypes.c_int32),
                ("boundary", ctypes.c_int32)]


class ILUError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        detail = lib().ilu_last_error().decode() if code == -3 else ""
        super().__init__("%s: %s (%d)%s" % (what, lib().ilu_strerror(code).decode(), code,
                                            " [" + detail + "]" if detail else ""))


_lib = None


def lib():
    """Load libilu.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError("libilu.so is not built: run __graft_entry__.build() or "
                              "python paper_2210_15280_amd/build.py")
        L = ctypes.CDLL(path)
        P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.ilu_setup_surrogate.argtypes = [ctypes.POINTER(ilu_tet_desc), I32, ctypes.POINTER(ilu_opts), P,
                                          ctypes.POINTER(P)]
        L.ilu_smooth.argtypes = [P, P, P, I32, D, ctypes.POINTER(D), P]
        L.stencil_apply.argtypes = [P, P, P, P]
        L.ilu_pcg.argtypes = [P, P, P, I32, D, D, ctypes.POINTER(I32), ctypes.POINTER(D), P]
        L.ilu_contraction.argtypes = [P, P, I32, ctypes.POINTER(D), ctypes.POINTER(D), P]
        L.ilu_lfa_orientation.argtypes = [ctypes.POINTER(ilu_tet_desc), I32, I32, P, P, P]
        L.ilu_lfa_orientation_noalloc.argtypes = [ctypes.POINTER(ilu_tet_desc), I32, I32, P, P, P]
        L.ilu_layout.argtypes = [P, I32, ctypes.POINTER(I64), ctypes.POINTER(I64)]
        L.ilu_destroy.argtypes = [P]
        L.ilu_strerror.argtypes = [ctypes.c_int]
        L.ilu_strerror.restype = ctypes.c_char_p
        L.ilu_last_error.argtypes = []
        L.ilu_last_error.restype = ctypes.c_char_p
        L.ilu_get_stencil.argtypes = [P, I32, P, P]
        L.ilu_get_factors.argtypes = [P, I32, P, P, P]
        L.ilu_get_surrogate.argtypes = [P, I32, P]
        L.ilu_set_surrogate.argtypes = [P, I32, P, P]
        L.ilu_get_surrogate_a.argtypes = [P, I32, P]
        L.ilu_set_surrogate_a.argtypes = [P, I32, P, P]
        L.ilu_get_surrogate_values.argtypes = [P, I32, P, P, P]
        L.ilu_sample_stride.argtypes = [P, I32, ctypes.POINTER(I32)]
        L.ilu_tile.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.ilu_setup_memory.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.ilu_last_sweeps.argtypes = [P, ctypes.POINTER(I32)]
        L.ilu_last_timing.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(D)]
        L.ilu_set_kernel_timing.argtypes = [P, I32]
        L.ilu_set_graph.argtypes = [P, I32]
        L.ilu_set_overlap.argtypes = [P, I32]
        L.ilu_set_flow_grid.argtypes = [P, I32, ctypes.POINTER(I32)]
        L.ilu_set_residual_chunk.argtypes = [P, I32]
        L.ilu_get_residual_chunk.argtypes = [P, ctypes.POINTER(I32)]
        L.ilu_get_flow_grid.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
        L.ilu_get_overlap.argtypes = [P, ctypes.POINTER(I32)]
        L.ilu_check_layout.argtypes = [ctypes.POINTER(ilu_tet_desc), I32, ctypes.POINTER(ilu_opts),
                                       ctypes.POINTER(I64)]
        _lib = L
    return _lib


def header_symbols() -> list:
    """Function names declared in include/ilu.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)))


def exported_symbols() -> list:
    out = []
    L = lib()
    for name in header_symbols():
        try:
            getattr(L, name)
            out.append(name)
        except AttributeError:
            pass
    return out


def _tet_array(tets):
    arr = (ilu_tet_desc * len(tets))()
    for i, t in enumerate(tets):
        arr[i].vertex[:] = [float(c) for row in t.verts for c in row]
        arr[i].level = int(t.level)
        arr[i].coeff_kind = int(t.coeff_kind)
        arr[i].coeff_param[:] = [float(c) for c in t.coeff_params]
    return arr


def lfa_orientation(tets: Sequence, samples: int = 16, stream: int = 0):
    """LFA smoothing factors of the 24 vertex permutations of every tetrahedron
    (ilu_lfa_orientation).  Returns (mu as a list of 24-lists, best index per
    tetrahedron)."""
    n = len(tets)
    mu = (ctypes.c_double * (24 * n))()
    best = (ctypes.c_int32 * n)()
    _check(lib().ilu_lfa_orientation(_tet_array(tets), n, int(samples), mu, best, ctypes.c_void_p(stream)),
           "ilu_lfa_orientation")
    return [list(mu[24 * i:24 * i + 24]) for i in range(n)], list(best)


def lfa_orientation_noalloc(tets: Sequence, samples: int = 16, stream: int = 0):
    """lfa_orientation through ilu_lfa_orientation_noalloc (no device
    allocation; at most LFA_NOALLOC_MAX_TETS tetrahedra)."""
    n = len(tets)
    mu = (ctypes.c_double * (24 * n))()
    best = (ctypes.c_int32 * n)()
    _check(lib().ilu_lfa_orientation_noalloc(_tet_array(tets), n, int(samples), mu, best, ctypes.c_void_p(stream)),
           "ilu_lfa_orientation_noalloc")
    return [list(mu[24 * i:24 * i + 24]) for i in range(n)], list(best)


LFA_NOALLOC_MAX_TETS = 256


def _check(code: int, what: str):
    if code != 0:
        raise ILUError(code, what)


def _ptr(t) -> int:
    return ctypes.c_void_p(t.data_ptr())


class Smoother:
    """One libilu handle over a list of macro-tetrahedra.

    tets: objects with .verts (4x3), .level, .coeff_kind, .coeff_params (4).
    Vectors are float64 CUDA tensors holding every tetrahedron's interior points
    in lexicographic order, concatenated (see ``offsets``)."""

    def __init__(self, tets: Sequence, variant: int = STORED_F64, degree=4, stride: int = 4,
                 schedule: int = SCHED_AUTO, tile=(0, 0), a_mode: int = A_EXACT, boundary: int = BOUNDARY_V2,
                 stream=None):
        import torch
        self.torch = torch
        self.L = lib()
        self.ntets = len(tets)
        arr = _tet_array(tets)
        opts = ilu_opts()
        opts.variant = int(variant)
        dg = (degree,) * 3 if isinstance(degree, int) else tuple(degree)
        opts.degree[:] = [int(d) for d in dg]
        opts.sample_stride = int(stride)
        opts.schedule = int(schedule)
        opts.tile[:] = [int(tile[0]), int(tile[1])]
        opts.a_mode = int(a_mode)
        opts.boundary = int(boundary)
        self.variant = variant
        self.degree = dg
        self.h = ctypes.c_void_p()
        _check(self.L.ilu_setup_surrogate(arr, self.ntets, ctypes.byref(opts), self._stream(stream),
                                          ctypes.byref(self.h)), "ilu_setup_surrogate")
        self.offsets, self.counts = [], []
        for i in range(self.ntets):
            o, c = ctypes.c_int64(), ctypes.c_int64()
            _check(self.L.ilu_layout(self.h, i, ctypes.byref(o), ctypes.byref(c)), "ilu_layout")
            self.offsets.append(o.value)
            self.counts.append(c.value)
        self.n_total = sum(self.counts)

    def _stream(self, stream):
        if stream is None:
            return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(int(stream))

    def _vec(self, t):
        assert t.dtype == self.torch.float64 and t.is_cuda and t.is_contiguous() and t.numel() == self.n_total
        return _ptr(t)

    def smooth(self, x, b, nsweeps: int, rel_tol: float = 0.0, want_relres: bool = False, stream=None):
        rel = ctypes.c_double(-1.0)
        rc = self.L.ilu_smooth(self.h, self._vec(x), self._vec(b), int(nsweeps), float(rel_tol),
                               ctypes.byref(rel) if (want_relres or rel_tol > 0) else None, self._stream(stream))
        if rc == -7:  # ILU_ENOTCONV: report, not an error of the call itself
            return rel.value, False
        _check(rc, "ilu_smooth")
        return rel.value, True

    def pcg(self, x, b, maxit: int, rel_tol: float = 0.0, abs_tol: float = 0.0, stream=None):
        """CG on A x = b preconditioned by this smoother's C; x is the start and
        the result.  Returns (iterations, true residual norm, converged)."""
        it, res = ctypes.c_int32(0), ctypes.c_double(-1.0)
        rc = self.L.ilu_pcg(self.h, self._vec(x), self._vec(b), int(maxit), float(rel_tol), float(abs_tol),
                            ctypes.byref(it), ctypes.byref(res), self._stream(stream))
        if rc == -7:  # ILU_ENOTCONV
            return it.value, res.value, False
        _check(rc, "ilu_pcg")
        return it.value, res.value, True

    def contraction(self, x, nsteps: int = 20, stream=None):
        """Power-iteration contraction factor from start vector x (overwritten
        with the last normalised iterate).  Returns (rho, rho_res)."""
        rho, rr = ctypes.c_double(), ctypes.c_double()
        _check(self.L.ilu_contraction(self.h, self._vec(x), int(nsteps), ctypes.byref(rho), ctypes.byref(rr),
                                      self._stream(stream)), "ilu_contraction")
        return rho.value, rr.value

    def apply(self, x, stream=None):
        y = self.torch.empty_like(x)
        _check(self.L.stencil_apply(self.h, self._vec(x), _ptr(y), self._stream(stream)), "stencil_apply")
        return y

    def stencil(self, tet: int = 0):
        A = self.torch.zeros((self.counts[tet], 15), dtype=self.torch.float64, device="cuda")
        _check(self.L.ilu_get_stencil(self.h, tet, _ptr(A), self._stream(None)), "ilu_get_stencil")
        return A

    def factors(self, tet: int = 0):
        L = self.torch.zeros((self.counts[tet], 7), dtype=self.torch.float64, device="cuda")
        D = self.torch.zeros(self.counts[tet], dtype=self.torch.float64, device="cuda")
        _check(self.L.ilu_get_factors(self.h, tet, _ptr(L), _ptr(D), self._stream(None)), "ilu_get_factors")
        return L, D

    def ncoef(self) -> int:
        dx, dy, dz = self.degree
        return (dx + 1) * (dy + 1) * (dz + 1)

    def surrogate(self, tet: int = 0):
        import numpy as np
        c = np.zeros((8, self.ncoef()))
        _check(self.L.ilu_get_surrogate(self.h, tet, c.ctypes.data_as(ctypes.c_void_p)), "ilu_get_surrogate")
        return c

    def set_surrogate(self, tet: int, coeffs):
        import numpy as np
        c = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(8, self.ncoef())
        _check(self.L.ilu_set_surrogate(self.h, tet, c.ctypes.data_as(ctypes.c_void_p), self._stream(None)),
               "ilu_set_surrogate")

    def surrogate_a(self, tet: int = 0):
        import numpy as np
        c = np.zeros((8, self.ncoef()))
        _check(self.L.ilu_get_surrogate_a(self.h, tet, c.ctypes.data_as(ctypes.c_void_p)), "ilu_get_surrogate_a")
        return c

    def set_surrogate_a(self, tet: int, coeffs):
        import numpy as np
        c = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(8, self.ncoef())
        _check(self.L.ilu_set_surrogate_a(self.h, tet, c.ctypes.data_as(ctypes.c_void_p), self._stream(None)),
               "ilu_set_surrogate_a")

    def surrogate_values(self, tet: int = 0):
        L = self.torch.zeros((self.counts[tet], 7), dtype=self.torch.float64, device="cuda")
        D = self.torch.zeros(self.counts[tet], dtype=self.torch.float64, device="cuda")
        _check(self.L.ilu_get_surrogate_values(self.h, tet, _ptr(L), _ptr(D), self._stream(None)),
               "ilu_get_surrogate_values")
        return L, D

    def sample_stride(self, tet: int = 0) -> int:
        s = ctypes.c_int32()
        _check(self.L.ilu_sample_stride(self.h, tet, ctypes.byref(s)), "ilu_sample_stride")
        return s.value

    @property
    def last_sweeps(self) -> int:
        """Sweeps the last smooth call ran."""
        k = ctypes.c_int32()
        _check(self.L.ilu_last_sweeps(self.h, ctypes.byref(k)), "ilu_last_sweeps")
        return k.value

    @property
    def tile(self):
        """Block shape (BV, BW) of the sweep schedule in use."""
        bv, bw = ctypes.c_int32(), ctypes.c_int32()
        _check(self.L.ilu_tile(self.h, ctypes.byref(bv), ctypes.byref(bw)), "ilu_tile")
        return bv.value, bw.value

    @property
    def setup_memory(self):
        """(peak, resident) device bytes the library held during setup / holds after it."""
        pk, rs = ctypes.c_int64(), ctypes.c_int64()
        _check(self.L.ilu_setup_memory(self.h, ctypes.byref(pk), ctypes.byref(rs)), "ilu_setup_memory")
        return pk.value, rs.value

    def timing(self):
        """(sweep loop ms, forward ms, backward ms, residual ms) of the last smooth call."""
        a, f, b, r = (ctypes.c_double() for _ in range(4))
        _check(self.L.ilu_last_timing(self.h, ctypes.byref(a), ctypes.byref(f), ctypes.byref(b), ctypes.byref(r)),
               "ilu_last_timing")
        return a.value, f.value, b.value, r.value

    def set_kernel_timing(self, enable: bool):
        _check(self.L.ilu_set_kernel_timing(self.h, 1 if enable else 0), "ilu_set_kernel_timing")

    def set_overlap(self, mode: int):
        """OVERLAP_OFF (default), OVERLAP_ON or OVERLAP_FUSED (see ilu_set_overlap)."""
        _check(self.L.ilu_set_overlap(self.h, int(mode)), "ilu_set_overlap")

    def overlap(self) -> int:
        v = ctypes.c_int32()
        _check(self.L.ilu_get_overlap(self.h, ctypes.byref(v)), "ilu_get_overlap")
        return v.value

    def set_flow_grid(self, grid: int) -> int:
        """Cap the persistent sweep grid at `grid` workgroups (0: the resident
        maximum).  Returns the grid now in use."""
        g = ctypes.c_int32()
        _check(self.L.ilu_set_flow_grid(self.h, int(grid), ctypes.byref(g)), "ilu_set_flow_grid")
        return g.value

    def set_residual_chunk(self, hyperplanes: int):
        """Hyperplanes per workgroup of the residual run on its own: 64 or 128
        (see ilu_set_residual_chunk)."""
        _check(self.L.ilu_set_residual_chunk(self.h, int(hyperplanes)), "ilu_set_residual_chunk")

    @property
    def residual_chunk(self) -> int:
        v = ctypes.c_int32()
        _check(self.L.ilu_get_residual_chunk(self.h, ctypes.byref(v)), "ilu_get_residual_chunk")
        return v.value

    @property
    def flow_grid(self):
        """(grid in use, default grid) of the persistent sweeps."""
        g, m = ctypes.c_int32(), ctypes.c_int32()
        _check(self.L.ilu_get_flow_grid(self.h, ctypes.byref(g), ctypes.byref(m)), "ilu_get_flow_grid")
        return g.value, m.value

    def set_graph(self, enable: bool):
        """Replay fixed-count sweeps from a captured graph (default on)."""
        _check(self.L.ilu_set_graph(self.h, 1 if enable else 0), "ilu_set_graph")

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.L.ilu_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
