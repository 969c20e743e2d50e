"""ctypes binding of libmpsvlasov.so (include/mps_vlasov.h, include/mps_blocks.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device buffers and the current stream.  If the
library has not been built the import of any entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpsvlasov.so")

MPS_OK, MPS_EINVAL, MPS_ENOMEM, MPS_ENUMERIC, MPS_EDEVICE = 0, -1, -2, -3, -4
ORDER_SEQ, ORDER_INTERLEAVED = 0, 1
PREC_FP64, PREC_FP32_CONTRACT = 0, 1

_lib = None


class MpsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("status %d: %s" % (status, msg))
        self.status = status


class CProblem(ctypes.Structure):
    _fields_ = [
        ("Lx", ctypes.c_int32), ("Lv", ctypes.c_int32), ("order", ctypes.c_int32),
        ("x_min", ctypes.c_double), ("x_max", ctypes.c_double),
        ("v_min", ctypes.c_double), ("v_max", ctypes.c_double),
        ("qm", ctypes.c_double), ("dt", ctypes.c_double),
        ("chi_max", ctypes.c_int32), ("level", ctypes.c_int32),
        ("df_max", ctypes.c_int32), ("tol", ctypes.c_double),
        ("precision", ctypes.c_int32), ("x_scheme", ctypes.c_int32),
        ("cfl", ctypes.c_double), ("compression", ctypes.c_int32),
        ("nu", ctypes.c_double), ("nu_v0", ctypes.c_double), ("nu_vth", ctypes.c_double),
        ("coll_model", ctypes.c_int32), ("tall_apply", ctypes.c_int32),
    ]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PD = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "mps_init": [ctypes.POINTER(CProblem), _I32, _P, _P, _P, ctypes.POINTER(_P)],
    "mps_step": [_P, _I32, _P],
    "mps_moments": [_P, _P, _P, _PD, _P],
    "mps_to_dense": [_P, _P, _P],
    "mps_free": [_P],
    "mps_info": [_P, _PI32, _PI32, _PD, _PD, _PI64],
    "mps_get_cores": [_P, _PI32, _PI64, _P, _P],
    "mps_set_cores": [_P, _PI32, _P, _P],
    "mps_add_scaled": [_P, _D, _PI32, _P, _P],
    "mps_workspace_bound": [ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_size_t)],
    "mps_device_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "mps_entanglement": [_P, _PD, _P],
    "mps_step_batched": [ctypes.POINTER(_P), _I32, _I32, _P],
    "mps_last_error": [],
    "mpsb_gemm": [_I32, _I32, _I32, _D, _P, _I64, _P, _I64, _D, _P, _I64, _P],
    "mpsb_gemm_prec": [_I32, _I32, _I32, _D, _P, _I64, _P, _I64, _D, _P, _I64, _I32, _P],
    "mpsb_qr": [_I32, _I32, _P, _P, _P],
    "mpsb_qr_tall": [_I32, _I32, _P, _P, _I32, _P],
    "mpsb_gemm_strided": [_I32, _I32, _I32, _D, _P, _I64, _I64, _I64, _P, _I64, _I64, _I64,
                          _D, _P, _I64, _I64, _I64, _I32, _I32, _P],
    "mpsb_svd_truncate": [_I32, _I32, _P, _I32, _D, _P, _P, _P, _PI32, _PD, _P],
    "mpsb_svd_truncate_noalloc": [_I32, _I32, _P, _I32, _D, _P, _P, _P, _PI32, _PD, _P],
    "mpsb_compress": [_I32, _PI32, _P, _PI32, _P, _I32, _D, _PI32, _P, _I64, _PD, _P],
    "mps_plasma_init": [_I32, _P, _P, _P, _P, _P, _P, _P],
    "mps_plasma_step": [_P, _I32, _P],
    "mps_plasma_species": [_P, _I32],
    "mps_plasma_field": [_P, _P, _PD, _P],
    "mps_plasma_free": [_P],
    "mps_batch_init": [_I32, _P, _P, _P, _P, _P, _P],
    "mps_batch_set_cores": [_P, _PI32, _P, _P],
    "mps_batch_add_scaled": [_P, _PD, _PI32, _P, _P],
    "mps_batch_step": [_P, _I32, _P],
    "mps_batch_instance": [_P, _I32],
    "mps_batch_free": [_P],
    "mpsb_step_graph": [_P, _I32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "mpsb_batch_step_graph": [_P, _I32, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)],
    "mpsb_compress_centre": [_I32, _I32, _PI32, _P, _I32, _D, _PI32, _P, _I64, _PD, _P],
    "mpsb_add_compress": [_I32, _I32, _PD, _PI32, ctypes.POINTER(_P), _I32, _D,
                          _PI32, _P, _I64, _P],
    "mpsb_density_field": [_P, _P, _P, _P],
    "mpsb_operator": [_I32, _I32, _D, _D, _PI32, _PD, _PI64],
    "mpsb_stats": [_PI64, _PI64, _PI64],
    "mpsb_arena_bytes": [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)],
    "mpsb_set_jacobi_max_sweeps": [_I32],
    "mpsb_profile": [_I32],
    "mpsb_profile_read": [_I32, _PI64, _PD, _PD, _PD],
    "mpsb_profile_nested_flops": [_I32, _PD],
    "mpsb_tune_clear": [],
    "mpsb_tune_set": [_PI32, _I32],
    "mpsb_tune_get": [_PI32, _PI32, _PI32],
    "mpsb_tune_size": [_PI64],
    "mpsb_tune_load": [ctypes.c_char_p],
    "mpsb_tune_save": [ctypes.c_char_p],
    "mpsb_tune_record": [_I32],
    "mpsb_tune_records": [_PI32, _PI32, ctypes.POINTER(ctypes.c_uint32), _PI64, _PD, _I64,
                          _PI64],
}

EXPORTED = sorted(_SIGS)


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library %s is missing: run "
                               "`python -c 'import __graft_entry__ as g; g.build()'`"
                               % LIB_PATH)
        # torch first: its HIP runtime is then the one the library binds to,
        # so the process holds a single runtime whatever the import order
        _torch()
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = (ctypes.c_char_p if name == "mps_last_error" else
                         ctypes.c_void_p if name in ("mps_plasma_species", "mps_batch_instance")
                         else ctypes.c_int)
        _lib = L
    return _lib


def _check(st: int):
    if st != MPS_OK:
        raise MpsError(st, lib().mps_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def _dev(a, device="cuda"):
    torch = _torch()
    if isinstance(a, np.ndarray):
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return a.to(device=device, dtype=torch.float64).contiguous()


def make_problem(p) -> CProblem:
    """From any object with the fields of workloads.Problem."""
    c = CProblem()
    c.Lx, c.Lv, c.order = int(p.Lx), int(p.Lv), int(p.order)
    c.x_min, c.x_max = float(p.x_min), float(p.x_max)
    c.v_min, c.v_max = float(p.v_min), float(p.v_max)
    c.qm, c.dt = float(p.qm), float(p.dt)
    c.chi_max = int(p.chi_max) if p.chi_max else 0
    c.level, c.df_max = int(p.level), int(p.df_max)
    c.tol, c.precision = float(p.tol), int(getattr(p, "precision", 0))
    c.x_scheme = int(getattr(p, "x_scheme", 0))
    c.cfl = float(getattr(p, "cfl", 0.0))
    c.compression = int(getattr(p, "compression", 0))
    c.nu = float(getattr(p, "nu", 0.0))
    c.nu_v0 = float(getattr(p, "nu_v0", 0.0))
    c.nu_vth = float(getattr(p, "nu_vth", 1.0))
    c.coll_model = int(getattr(p, "coll_model", 0))
    c.tall_apply = int(getattr(p, "tall_apply", 0))
    return c


def pack_cores(cores: Sequence[np.ndarray]) -> Tuple[np.ndarray, np.ndarray]:
    """Host list of (l, 2, r) arrays -> (bonds int32[n+1], packed float64)."""
    bonds = [1] + [int(c.shape[2]) for c in cores]
    flat = np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in cores])
    return np.asarray(bonds, dtype=np.int32), flat


def unpack_cores(bonds, flat) -> List[np.ndarray]:
    out, off = [], 0
    for j in range(len(bonds) - 1):
        n = int(bonds[j]) * 2 * int(bonds[j + 1])
        out.append(np.asarray(flat[off:off + n]).reshape(int(bonds[j]), 2, int(bonds[j + 1])))
        off += n
    return out


class MpsState:
    """One solve: owns the device state created by mps_init."""

    def __init__(self, problem, ax, bv, stream=None):
        L = lib()
        self.problem = problem
        self.Nx, self.Nv = 2 ** int(problem.Lx), 2 ** int(problem.Lv)
        self._cp = make_problem(problem)
        axd = _dev(np.atleast_2d(ax))
        bvd = _dev(np.atleast_2d(bv))
        h = ctypes.c_void_p()
        _check(L.mps_init(ctypes.byref(self._cp), int(axd.shape[0]), _ptr(axd),
                          _ptr(bvd), _stream(stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def step(self, nsteps: int = 1, stream=None):
        _check(lib().mps_step(self._h, int(nsteps), _stream(stream)))

    def to_dense(self, out=None, stream=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.Nx * self.Nv, dtype=torch.float64, device="cuda")
        _check(lib().mps_to_dense(self._h, _ptr(out), _stream(stream)))
        return out.view(self.Nx, self.Nv)

    def moments(self, stream=None):
        torch = _torch()
        n = torch.empty(self.Nx, dtype=torch.float64, device="cuda")
        E = torch.empty(self.Nx, dtype=torch.float64, device="cuda")
        sc = (ctypes.c_double * 4)()
        _check(lib().mps_moments(self._h, _ptr(n), _ptr(E), sc, _stream(stream)))
        return n, E, {"mass": sc[0], "momentum": sc[1], "kinetic": sc[2],
                      "field_energy": sc[3]}

    def density_field(self, stream=None):
        torch = _torch()
        n = torch.empty(self.Nx, dtype=torch.float64, device="cuda")
        E = torch.empty(self.Nx, dtype=torch.float64, device="cuda")
        _check(lib().mpsb_density_field(self._h, _ptr(n), _ptr(E), _stream(stream)))
        return n, E

    def info(self):
        ns = ctypes.c_int32()
        _check(lib().mps_info(self._h, ctypes.byref(ns), None, None, None, None))
        n = ns.value
        bonds = (ctypes.c_int32 * (n + 1))()
        disc = (ctypes.c_double * max(n - 1, 1))()
        t = ctypes.c_double()
        st = ctypes.c_int64()
        _check(lib().mps_info(self._h, None, bonds, disc, ctypes.byref(t), ctypes.byref(st)))
        return {"n": n, "bonds": list(bonds), "discarded": list(disc)[:n - 1],
                "t": t.value, "steps": st.value}

    def entanglement(self, stream=None) -> List[float]:
        """Entanglement entropy (log2) at each of the n-1 bonds."""
        n = self.info()["n"]
        ee = (ctypes.c_double * max(n - 1, 1))()
        _check(lib().mps_entanglement(self._h, ee, _stream(stream)))
        return list(ee)[:n - 1]

    def step_graph(self, enable=None):
        """Turn captured step graphs on/off (None: unchanged); returns
        (captures, replays)."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        e = -1 if enable is None else int(bool(enable))
        _check(lib().mpsb_step_graph(self._h, e, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        _check(lib().mps_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def arena_bytes(self):
        """(reserved, peak) bytes of the state's seven arenas."""
        r = (ctypes.c_size_t * 7)()
        p = (ctypes.c_size_t * 7)()
        _check(lib().mpsb_arena_bytes(self._h, r, p))
        return list(r), list(p)

    def get_cores(self, stream=None):
        torch = _torch()
        n = self.info()["n"]
        bonds = (ctypes.c_int32 * (n + 1))()
        cnt = ctypes.c_int64()
        _check(lib().mps_get_cores(self._h, bonds, ctypes.byref(cnt), None, _stream(stream)))
        buf = torch.empty(cnt.value, dtype=torch.float64, device="cuda")
        _check(lib().mps_get_cores(self._h, bonds, ctypes.byref(cnt), _ptr(buf), _stream(stream)))
        return np.asarray(list(bonds), dtype=np.int32), buf

    def get_cores_host(self) -> List[np.ndarray]:
        b, buf = self.get_cores()
        return unpack_cores(b, buf.cpu().numpy())

    def set_cores(self, cores: Sequence[np.ndarray], stream=None):
        b, flat = pack_cores(cores)
        d = _dev(flat)
        _check(lib().mps_set_cores(self._h, b.ctypes.data_as(_PI32), _ptr(d), _stream(stream)))

    def add_scaled(self, alpha: float, cores: Sequence[np.ndarray], stream=None):
        b, flat = pack_cores(cores)
        d = _dev(flat)
        _check(lib().mps_add_scaled(self._h, float(alpha), b.ctypes.data_as(_PI32),
                                    _ptr(d), _stream(stream)))

    def free(self):
        if getattr(self, "_borrowed", False):
            self._h = ctypes.c_void_p()
            return
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().mps_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Lock-step instances of one problem shape (mps_batch_*): problems and
    (ax, bv) profiles per instance; each launch of a step covers them all."""

    def __init__(self, problems, profiles, stream=None):
        L = lib()
        n = len(problems)
        self.problems = list(problems)
        arr = (CProblem * n)(*[make_problem(p) for p in problems])
        self._dev = [(_dev(np.atleast_2d(a)), _dev(np.atleast_2d(b))) for a, b in profiles]
        ranks = (ctypes.c_int32 * n)(*[int(a.shape[0]) for a, _ in self._dev])
        axp = (ctypes.c_void_p * n)(*[a.data_ptr() for a, _ in self._dev])
        bvp = (ctypes.c_void_p * n)(*[b.data_ptr() for _, b in self._dev])
        h = ctypes.c_void_p()
        _check(L.mps_batch_init(n, ctypes.cast(arr, _P), ctypes.cast(ranks, _P),
                                ctypes.cast(axp, _P), ctypes.cast(bvp, _P),
                                _stream(stream), ctypes.byref(h)))
        self._h = h
        self.count = n

    def step(self, nsteps: int = 1, stream=None):
        _check(lib().mps_batch_step(self._h, int(nsteps), _stream(stream)))

    def _packed(self, cores_list):
        bonds, devs = None, []
        for cores in cores_list:
            b, flat = pack_cores(cores)
            if bonds is None:
                bonds = b
            assert np.array_equal(b, bonds), "instances need one set of bonds"
            devs.append(_dev(flat))
        ptrs = (ctypes.c_void_p * len(devs))(*[d.data_ptr() for d in devs])
        return bonds, devs, ptrs

    def set_cores(self, cores_list, stream=None):
        """Every instance's cores (host lists of (l, 2, r) arrays, one set of
        bonds)."""
        b, keep, ptrs = self._packed(cores_list)
        _check(lib().mps_batch_set_cores(self._h, b.ctypes.data_as(_PI32),
                                         ctypes.cast(ptrs, _P), _stream(stream)))

    def add_scaled(self, alphas, cores_list, stream=None):
        b, keep, ptrs = self._packed(cores_list)
        al = (ctypes.c_double * len(alphas))(*[float(a) for a in alphas])
        _check(lib().mps_batch_add_scaled(self._h, al, b.ctypes.data_as(_PI32),
                                          ctypes.cast(ptrs, _P), _stream(stream)))

    def step_graph(self, enable=None):
        """Turn captured step graphs of the batch on/off (None: unchanged);
        returns (captures, replays)."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        e = -1 if enable is None else int(bool(enable))
        _check(lib().mpsb_batch_step_graph(self._h, e, ctypes.byref(c), ctypes.byref(r)))
        return c.value, r.value

    def instance(self, i: int) -> "MpsState":
        """Instance i as a state owned by the batch (read-only: dense
        values, cores, moments, info)."""
        hp = lib().mps_batch_instance(self._h, int(i))
        if not hp:
            raise MpsError(MPS_EINVAL, "no instance %d" % i)
        st = MpsState.__new__(MpsState)
        p = self.problems[i]
        st.problem = p
        st.Nx, st.Nv = 2 ** int(p.Lx), 2 ** int(p.Lv)
        st._cp = make_problem(p)
        st._h = ctypes.c_void_p(hp)
        st._borrowed = True
        return st

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().mps_batch_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Plasma:
    """Several species sharing x and E (mps_plasma_*): problems, charges
    and (ax, bv) profiles per species."""

    def __init__(self, problems, charges, profiles, stream=None):
        L = lib()
        n = len(problems)
        self.problems = list(problems)
        arr = (CProblem * n)(*[make_problem(p) for p in problems])
        q = (ctypes.c_double * n)(*[float(c) for c in charges])
        self._dev = [(_dev(np.atleast_2d(a)), _dev(np.atleast_2d(b))) for a, b in profiles]
        ranks = (ctypes.c_int32 * n)(*[int(a.shape[0]) for a, _ in self._dev])
        axp = (ctypes.c_void_p * n)(*[a.data_ptr() for a, _ in self._dev])
        bvp = (ctypes.c_void_p * n)(*[b.data_ptr() for _, b in self._dev])
        h = ctypes.c_void_p()
        _check(L.mps_plasma_init(n, ctypes.cast(arr, _P), ctypes.cast(q, _P),
                                 ctypes.cast(ranks, _P), ctypes.cast(axp, _P),
                                 ctypes.cast(bvp, _P), _stream(stream), ctypes.byref(h)))
        self._h = h

    def step(self, nsteps: int = 1, stream=None):
        _check(lib().mps_plasma_step(self._h, int(nsteps), _stream(stream)))

    def species(self, s: int) -> "MpsState":
        """Species s as a state (owned by the plasma: not freed by it)."""
        hp = lib().mps_plasma_species(self._h, int(s))
        if not hp:
            raise MpsError("no species %d" % s)
        st = MpsState.__new__(MpsState)
        p = self.problems[s]
        st.problem = p
        st.Nx, st.Nv = 2 ** int(p.Lx), 2 ** int(p.Lv)
        st._cp = make_problem(p)
        st._h = ctypes.c_void_p(hp)
        st._borrowed = True
        return st

    def field(self, stream=None):
        torch = _torch()
        nx = 2 ** int(self.problems[0].Lx)
        E = torch.empty(nx, dtype=torch.float64, device="cuda")
        w = ctypes.c_double()
        _check(lib().mps_plasma_field(self._h, _ptr(E), ctypes.byref(w), _stream(stream)))
        return E, w.value

    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().mps_plasma_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def step_batched(states: Sequence[MpsState], nsteps: int = 1, stream=None):
    arr = (ctypes.c_void_p * len(states))(*[s.handle.value for s in states])
    _check(lib().mps_step_batched(arr, len(states), int(nsteps), _stream(stream)))


def workspace_bound(problem) -> int:
    c = make_problem(problem)
    b = ctypes.c_size_t()
    _check(lib().mps_workspace_bound(ctypes.byref(c), ctypes.byref(b)))
    return int(b.value)


# ------------------------------------------------------------- blocks

def gemm(A, B, alpha=1.0, beta=0.0, C=None, stream=None, precision=0):
    torch = _torch()
    A, B = _dev(A), _dev(B)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    if C is None:
        C = torch.zeros(M, N, dtype=torch.float64, device="cuda")
    _check(lib().mpsb_gemm_prec(M, N, K, alpha, _ptr(A), K, _ptr(B), N, beta, _ptr(C), N,
                                int(precision), _stream(stream)))
    return C


def gemm_strided(M, N, K, alpha, A, a_strides, B, b_strides, beta, C, c_strides,
                 batch=1, precision=0, stream=None):
    """mpsb_gemm_strided on device tensors; strides (row, col, batch) in
    elements."""
    _check(lib().mpsb_gemm_strided(M, N, K, float(alpha), _ptr(A), *a_strides, _ptr(B),
                                   *b_strides, float(beta), _ptr(C), *c_strides, int(batch),
                                   int(precision), _stream(stream)))
    return C


def qr(A, stream=None, tall_apply=None):
    """Returns (R upper-trapezoid k x n, Q thin m x k) as device tensors;
    tall_apply selects the reflector-application mode (mpsb_qr_tall)."""
    torch = _torch()
    A = _dev(A).clone()
    m, n = A.shape
    k = min(m, n)
    Q = torch.empty(m, k, dtype=torch.float64, device="cuda")
    if tall_apply is None:
        _check(lib().mpsb_qr(m, n, _ptr(A), _ptr(Q), _stream(stream)))
    else:
        _check(lib().mpsb_qr_tall(m, n, _ptr(A), _ptr(Q), int(tall_apply), _stream(stream)))
    return torch.triu(A[:k]), Q


def svd_truncate(X, cap=0, tol=0.0, stream=None):
    torch = _torch()
    X = _dev(X).clone()
    m, c = X.shape
    kmax = min(m, c, cap) if cap and cap > 0 else min(m, c)
    Vt = torch.empty(kmax * c, dtype=torch.float64, device="cuda")
    US = torch.empty(m * kmax, dtype=torch.float64, device="cuda")
    sig = torch.empty(min(m, c), dtype=torch.float64, device="cuda")
    D = ctypes.c_int32()
    disc = ctypes.c_double()
    _check(lib().mpsb_svd_truncate(m, c, _ptr(X), int(cap), float(tol), _ptr(Vt), _ptr(US),
                                   _ptr(sig), ctypes.byref(D), ctypes.byref(disc),
                                   _stream(stream)))
    d = D.value
    return Vt[:d * c].view(d, c), US[:m * d].view(m, d), sig, disc.value


def svd_truncate_noalloc(X, Vt, US, sig, cap=0, tol=0.0, stream=None):
    """mpsb_svd_truncate_noalloc on caller-allocated device buffers: X (m x c,
    overwritten), Vt (>= kmax * c), US (>= m * kmax), sig (>= min(m, c)) with
    kmax = min(m, c, cap); returns (D, discarded)."""
    m, c = X.shape
    D = ctypes.c_int32()
    disc = ctypes.c_double()
    _check(lib().mpsb_svd_truncate_noalloc(m, c, _ptr(X), int(cap), float(tol), _ptr(Vt),
                                           _ptr(US), _ptr(sig), ctypes.byref(D),
                                           ctypes.byref(disc), _stream(stream)))
    return D.value, disc.value


def compress(cores: Sequence[np.ndarray], cap=0, tol=0.0, mpo=None, stream=None):
    """Compress host MPS cores (optionally after applying a host MPO given as
    a list of (bl, 2, 2, br) arrays); returns (host cores, discarded)."""
    torch = _torch()
    n = len(cores)
    b, flat = pack_cores(cores)
    d = _dev(flat)
    if mpo is not None:
        wb = np.asarray([1] + [int(w.shape[3]) for w in mpo], dtype=np.int32)
        wd = _dev(np.concatenate([np.ascontiguousarray(w).ravel() for w in mpo]))
        wbp, wp = wb.ctypes.data_as(_PI32), _ptr(wd)
        wmax = int(max(wb))
    else:
        wbp, wp, wmax = None, ctypes.c_void_p(0), 1
    cap_eff = cap if cap and cap > 0 else 1 << 30
    capacity = sum(min(cap_eff, 2 ** min(j, n - j), int(b[j]) * wmax) * 2 *
                   min(cap_eff, 2 ** min(j + 1, n - j - 1), int(b[j + 1]) * wmax)
                   for j in range(n))
    out = torch.empty(capacity, dtype=torch.float64, device="cuda")
    ob = (ctypes.c_int32 * (n + 1))()
    disc = (ctypes.c_double * (n - 1))()
    _check(lib().mpsb_compress(n, wbp, wp, b.ctypes.data_as(_PI32), _ptr(d), int(cap),
                               float(tol), ob, _ptr(out), capacity, disc, _stream(stream)))
    return unpack_cores(list(ob), out.cpu().numpy()), list(disc)


def compress_centre(cores: Sequence[np.ndarray], centre: int, cap=0, tol=0.0,
                    stream=None):
    """Centre-first compression of host MPS cores cut at the bond
    centre-1 | centre; returns (host cores, discarded)."""
    torch = _torch()
    n = len(cores)
    b, flat = pack_cores(cores)
    d = _dev(flat)
    cap_eff = cap if cap and cap > 0 else 1 << 30
    capacity = sum(min(cap_eff, 2 ** min(j, n - j), int(b[j])) * 2 *
                   min(cap_eff, 2 ** min(j + 1, n - j - 1), int(b[j + 1]))
                   for j in range(n))
    out = torch.empty(capacity, dtype=torch.float64, device="cuda")
    ob = (ctypes.c_int32 * (n + 1))()
    disc = (ctypes.c_double * (n - 1))()
    _check(lib().mpsb_compress_centre(n, int(centre), b.ctypes.data_as(_PI32), _ptr(d),
                                      int(cap), float(tol), ob, _ptr(out), capacity,
                                      disc, _stream(stream)))
    return unpack_cores(list(ob), out.cpu().numpy()), list(disc)


def add_compress(terms: Sequence[Tuple[float, Sequence[np.ndarray]]], cap=0, tol=0.0,
                 stream=None):
    torch = _torch()
    n = len(terms[0][1])
    bonds_all, devs = [], []
    for _, cores in terms:
        b, flat = pack_cores(cores)
        bonds_all.append(b)
        devs.append(_dev(flat))
    bonds = np.concatenate(bonds_all).astype(np.int32)
    coef = (ctypes.c_double * len(terms))(*[float(c) for c, _ in terms])
    ptrs = (ctypes.c_void_p * len(terms))(*[t.data_ptr() for t in devs])
    tot = [sum(int(bb[j]) for bb in bonds_all) for j in range(n + 1)]
    tot[0] = tot[n] = 1
    capacity = sum(tot[j] * 2 * tot[j + 1] for j in range(n))
    out = torch.empty(capacity, dtype=torch.float64, device="cuda")
    ob = (ctypes.c_int32 * (n + 1))()
    _check(lib().mpsb_add_compress(n, len(terms), coef, bonds.ctypes.data_as(_PI32), ptrs,
                                   int(cap), float(tol), ob, _ptr(out), capacity,
                                   _stream(stream)))
    return unpack_cores(list(ob), out.cpu().numpy())


def operator(which: int, L: int, h0: float, h: float) -> List[np.ndarray]:
    cnt = ctypes.c_int64()
    bonds = (ctypes.c_int32 * (L + 1))()
    _check(lib().mpsb_operator(which, L, h0, h, bonds, None, ctypes.byref(cnt)))
    W = np.empty(cnt.value, dtype=np.float64)
    _check(lib().mpsb_operator(which, L, h0, h, bonds, W.ctypes.data_as(_PD),
                               ctypes.byref(cnt)))
    out, off = [], 0
    for j in range(L):
        n = bonds[j] * 4 * bonds[j + 1]
        out.append(W[off:off + n].reshape(bonds[j], 2, 2, bonds[j + 1]))
        off += n
    return out


def stats():
    q, s, j = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mpsb_stats(ctypes.byref(q), ctypes.byref(s), ctypes.byref(j)))
    return {"qr_calls": q.value, "svd_calls": s.value, "jacobi_sweeps": j.value}


def set_jacobi_max_sweeps(n: int):
    _check(lib().mpsb_set_jacobi_max_sweeps(int(n)))


KERNEL_CLASSES = ("gemm_f64", "qr_factor", "jacobi_svd", "other", "qr_apply", "qr_wy")


def profile(enable: bool):
    _check(lib().mpsb_profile(1 if enable else 0))


def profile_read():
    out = {}
    for c, name in enumerate(KERNEL_CLASSES):
        n, ms, fl, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().mpsb_profile_read(c, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl),
                                       ctypes.byref(by)))
        nf = ctypes.c_double()
        _check(lib().mpsb_profile_nested_flops(c, ctypes.byref(nf)))
        out[name] = {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value,
                     "nested_flops": nf.value}
    return out


# ---- launch-shape table (mpsb_tune_*)
TUNE_GEMM_TILE, TUNE_APPLY_COLS = 1, 2


def _key6(key):
    k = np.ascontiguousarray(np.asarray(key, dtype=np.int32))
    if k.shape != (6,):
        raise ValueError("a tuning key has six integers")
    return k


def tune_clear():
    _check(lib().mpsb_tune_clear())


def tune_set(key, value: int):
    k = _key6(key)
    _check(lib().mpsb_tune_set(k.ctypes.data_as(_PI32), int(value)))


def tune_get(key):
    k = _key6(key)
    v, f = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().mpsb_tune_get(k.ctypes.data_as(_PI32), ctypes.byref(v), ctypes.byref(f)))
    return v.value if f.value else None


def tune_size() -> int:
    n = ctypes.c_int64()
    _check(lib().mpsb_tune_size(ctypes.byref(n)))
    return n.value


def tune_load(path: str):
    _check(lib().mpsb_tune_load(os.fsencode(path)))


def tune_save(path: str):
    _check(lib().mpsb_tune_save(os.fsencode(path)))


def tune_record(on: bool):
    _check(lib().mpsb_tune_record(1 if on else 0))


def tune_records():
    """Records since tune_record(True): a list of dicts with the key (six
    ints), the value used, the allowed values, launches and summed ms."""
    n = ctypes.c_int64()
    _check(lib().mpsb_tune_records(None, None, None, None, None, 0, ctypes.byref(n)))
    cap = n.value
    keys = np.zeros((max(cap, 1), 6), dtype=np.int32)
    vals = np.zeros(max(cap, 1), dtype=np.int32)
    allowed = np.zeros(max(cap, 1), dtype=np.uint32)
    launches = np.zeros(max(cap, 1), dtype=np.int64)
    ms = np.zeros(max(cap, 1), dtype=np.float64)
    _check(lib().mpsb_tune_records(keys.ctypes.data_as(_PI32), vals.ctypes.data_as(_PI32),
                                   allowed.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                   launches.ctypes.data_as(_PI64), ms.ctypes.data_as(_PD),
                                   cap, ctypes.byref(n)))
    m = min(cap, n.value)
    return [{"key": tuple(int(x) for x in keys[i]), "value": int(vals[i]),
             "allowed": [b for b in range(32) if (int(allowed[i]) >> b) & 1],
             "launches": int(launches[i]), "ms": float(ms[i])} for i in range(m)]
