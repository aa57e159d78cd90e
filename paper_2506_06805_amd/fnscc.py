"""Thin ctypes binding of libfnscc (argument marshalling only).

Every step of the hot path runs inside the HIP library.  PyTorch supplies the device memory (its
caching allocator, through the allocator callbacks of fc_create) and the stream.  Loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import pathlib
import weakref

import numpy as np
# torch loads the HIP runtime first so that the library binds to the same one (loaded the other
# way round, the library's first hipSetDevice fails)
import torch  # noqa: F401

_LIB_PATH = pathlib.Path(__file__).resolve().parent / "libfnscc.so"
if not _LIB_PATH.exists():
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2506_06805_amd.build`")
lib = C.CDLL(str(_LIB_PATH))

FC_OK, FC_EARG, FC_EHIP, FC_ENOMEM, FC_ENOCONV, FC_ENUMERIC, FC_EUNSUPPORTED = range(7)
FC_C128, FC_C64 = 0, 1
FC_FP64, FC_SPLIT_BF16, FC_SPLIT_FP16, FC_FP32 = 0, 1, 2, 3
PRECISION = {"fp64": FC_FP64, "split-bf16": FC_SPLIT_BF16, "split-fp16": FC_SPLIT_FP16}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
ON_ITER_FN = C.CFUNCTYPE(None, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p)


class CcsdOpts(C.Structure):
    _fields_ = [("e_tol", C.c_double), ("r_tol", C.c_double), ("max_iter", C.c_int), ("diis_dim", C.c_int),
                ("learned", C.c_int), ("precision", C.c_int), ("t1_init", C.c_void_p), ("t2_init", C.c_void_p),
                ("mlp", C.c_void_p), ("stall_window", C.c_int), ("on_iter", ON_ITER_FN), ("user", C.c_void_p),
                ("diis_start", C.c_int), ("precond", C.c_int)]


class EomOpts(C.Structure):
    _fields_ = [("r_tol", C.c_double), ("w_tol", C.c_double), ("max_iter", C.c_int), ("max_subspace", C.c_int),
                ("guess_per_root", C.c_int), ("graph", C.c_int)]


P = C.c_void_p
_sig = {
    "fc_create": (C.c_int, [C.POINTER(P), C.c_int, P, ALLOC_FN, FREE_FN, P]),
    "fc_destroy": (None, [P]),
    "fc_last_error": (C.c_char_p, [P]),
    "fc_set_timing": (C.c_int, [P, C.c_int]),
    "fc_take_timings": (C.c_int, [P, C.c_char_p, C.c_size_t]),
    "fc_set_autotune": (C.c_int, [P, C.c_int]),
    "fc_set_gemm_config": (C.c_int, [P, C.c_int]),
    "fc_gemm_num_configs": (C.c_int, []),
    "fc_set_split_config": (C.c_int, [P, C.c_int]),
    "fc_split_num_configs": (C.c_int, []),
    "fc_autotune_save": (C.c_int, [P, C.c_char_p]),
    "fc_autotune_load": (C.c_int, [P, C.c_char_p]),
    "fc_autotune_size": (C.c_int, [P]),
    "cd_ao_pivoted": (C.c_int, [P, C.c_long, P, C.c_double, C.c_int, P, C.POINTER(C.c_int), P]),
    "ao_to_spinor": (C.c_int, [P, C.c_int, C.c_int, C.c_int, P, P, P]),
    "cd_integrals": (C.c_int, [P, C.c_int, C.c_int, C.c_int, P, P, C.c_int, C.c_int, C.c_int, C.POINTER(P)]),
    "fc_ints_info": (C.c_int, [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "fc_free_ints": (None, [P]),
    "fns_truncate": (C.c_int, [P, P, C.c_double, C.POINTER(P), C.POINTER(C.c_int), P, P]),
    "fc_ccsd_default_opts": (None, [C.POINTER(CcsdOpts)]),
    "ccsd_solve": (C.c_int, [P, C.c_int, C.POINTER(P), C.POINTER(CcsdOpts), C.POINTER(P), P, P]),
    "ccsd_residual": (C.c_int, [P, P, P, P, P, P, C.c_int]),
    "fc_ladder": (C.c_int, [P, P, P, P, P, C.c_int]),
    "fc_ladder_packed": (C.c_int, [P, P, P, P, P, C.c_int]),
    "fc_zgemm": (C.c_int, [P, C.c_char, C.c_char, C.c_long, C.c_long, C.c_long, P, P, C.c_long, P, C.c_long,
                           P, P, C.c_long, C.c_int]),
    "fc_zgemm_noalloc": (C.c_int, [P, C.c_char, C.c_char, C.c_long, C.c_long, C.c_long, P, P, C.c_long, P,
                                   C.c_long, P, P, C.c_long, C.c_int]),
    "fc_amps_create": (C.c_int, [P, P, P, P, C.POINTER(P)]),
    "fc_amps_read": (C.c_int, [P, P, P]),
    "fc_free_amps": (None, [P]),
    "ipeom_sigma": (C.c_int, [P, P, P, C.c_int, P, P]),
    "fc_eom_default_opts": (None, [C.POINTER(EomOpts)]),
    "ipeom_davidson": (C.c_int, [P, C.c_int, C.POINTER(P), C.POINTER(P), P, C.POINTER(EomOpts), P, P, P]),
    "ipeom_sigma_left": (C.c_int, [P, P, P, C.c_int, P, P]),
    "ipeom_left": (C.c_int, [P, C.c_int, C.POINTER(P), C.POINTER(P), P, C.POINTER(EomOpts), P, P, P, P, P]),
    "fc_mlp_create": (C.c_int, [P, P, C.c_ulonglong, C.POINTER(P)]),
    "fc_mlp_free": (None, [P]),
    "fc_mlp_num_params": (C.c_long, []),
    "fc_mlp_get_params": (C.c_int, [P, P, C.c_int]),
    "fc_mlp_grad": (C.c_int, [P, P, P, P, C.c_long, P, P]),
    "fc_mlp_train_step": (C.c_int, [P, P, P, P, C.c_long, C.c_float, P]),
    "fc_mlp_forward": (C.c_int, [P, P, C.c_long, P, C.c_int]),
    "fc_learned_step": (C.c_int, [P, P, P, P, P, P, P, P, P, P, P]),
    "fc_learn_samples": (C.c_int, [P, P, P, P, P, P, P, C.c_long, C.c_ulonglong, P, P, P]),
    "fc_host_zheev": (C.c_int, [C.c_int, P, P]),
    "fc_host_zgeev": (C.c_int, [C.c_int, P, P, P]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class FcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _require(t, name, dtypes, shape=None):
    """Refuse (ValueError) anything but a contiguous GPU tensor of one of `dtypes` and `shape`:
    the library takes raw device pointers and trusts their sizes, so a host tensor, a short
    tensor or the wrong element type must never reach it."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor on the GPU, got {type(t).__name__}")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: must be a GPU tensor (got device {t.device})")
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype} not accepted ({', '.join(map(str, dtypes))})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)} != {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t


_C128 = (torch.complex128,)


def _ptr(a):
    """Address of a numpy array or a torch tensor (contiguous)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags.c_contiguous
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


# ------------------------------------------------------------------------------ host utilities
def host_zheev(A):
    A = np.array(A, dtype=np.complex128, order="C")
    n = A.shape[0]
    w = np.zeros(n)
    rc = lib.fc_host_zheev(n, A.ctypes.data, w.ctypes.data)
    if rc:
        raise FcError(rc, "fc_host_zheev failed")
    return w, A


def host_zgeev(A):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    n = A.shape[0]
    w = np.zeros(n, dtype=np.complex128)
    V = np.zeros((n, n), dtype=np.complex128)
    rc = lib.fc_host_zgeev(n, A.ctypes.data, w.ctypes.data, V.ctypes.data)
    if rc:
        raise FcError(rc, "fc_host_zgeev failed")
    return w, V


# ------------------------------------------------------------------------------ device context
class Context:
    """fc_ctx bound to a torch device and its current stream; device memory from torch."""

    def __init__(self, device=0, stream=None, use_torch_allocator=True):
        import torch

        self.torch = torch
        self.device = device
        torch.cuda.set_device(device)   # initialise the device in torch before the library uses it
        self.stream = stream or torch.cuda.current_stream(device)
        self._children = weakref.WeakSet()   # handles that must be freed before the context
        if use_torch_allocator:
            def _alloc(nbytes, _stream, _user):
                try:
                    p = torch.cuda.caching_allocator_alloc(int(nbytes), device, self.stream)
                except Exception:  # out of memory: the library reports FC_ENOMEM
                    return None
                return p

            def _free(ptr, _nbytes, _stream, _user):
                torch.cuda.caching_allocator_delete(ptr)

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
        else:
            self._alloc_cb = ALLOC_FN()
            self._free_cb = FREE_FN()
        h = P()
        rc = lib.fc_create(C.byref(h), device, P(self.stream.cuda_stream), self._alloc_cb, self._free_cb, None)
        if rc:
            raise FcError(rc, "fc_create failed")
        self.h = h

    def check(self, rc, what):
        if rc not in (FC_OK,):
            raise FcError(rc, f"{what}: {lib.fc_last_error(self.h).decode()}")

    def adopt(self, child):
        self._children.add(child)
        return child

    def close(self):
        if getattr(self, "h", None):
            for child in list(self._children):
                child.free()
            lib.fc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on=True):
        lib.fc_set_timing(self.h, int(on))

    def set_autotune(self, on=True):
        self.check(lib.fc_set_autotune(self.h, int(on)), "fc_set_autotune")

    def autotune_save(self, path):
        self.check(lib.fc_autotune_save(self.h, str(path).encode()), "fc_autotune_save")

    def autotune_load(self, path):
        self.check(lib.fc_autotune_load(self.h, str(path).encode()), "fc_autotune_load")

    def autotune_size(self):
        return int(lib.fc_autotune_size(self.h))

    def set_gemm_config(self, cfg):
        """Force GEMM tile configuration `cfg` on every product it fits (-1: size heuristic)."""
        self.check(lib.fc_set_gemm_config(self.h, int(cfg)), "fc_set_gemm_config")

    @staticmethod
    def gemm_num_configs():
        return int(lib.fc_gemm_num_configs())

    def set_split_config(self, cfg):
        """Force the staging of the 128-wide split-precision tiles (0 registers, 1 four waves,
        2 direct-to-LDS; -1: default)."""
        self.check(lib.fc_set_split_config(self.h, int(cfg)), "fc_set_split_config")

    @staticmethod
    def split_num_configs():
        return int(lib.fc_split_num_configs())

    def take_timings(self):
        buf = C.create_string_buffer(1 << 16)
        lib.fc_take_timings(self.h, buf, len(buf))
        out = {}
        for kv in buf.value.decode().split(";"):
            if "=" in kv:
                k, v = kv.split("=")
                out[k] = float(v)
        return out


class _Handle:
    """Library handle owned by a context; freed before the context is destroyed."""

    _free_fn = None

    def free(self):
        if getattr(self, "h", None) and getattr(self.ctx, "h", None):
            type(self)._free_fn(self.h)
        self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Ints(_Handle):
    _free_fn = staticmethod(lambda h: lib.fc_free_ints(h))

    def __init__(self, ctx: Context, h, o, v, ncd):
        self.ctx, self.h, self.o, self.v, self.ncd = ctx, h, o, v, ncd
        ctx.adopt(self)

    @property
    def dim(self):
        return self.o + self.o * (self.o - 1) // 2 * self.v


class Amps(_Handle):
    _free_fn = staticmethod(lambda h: lib.fc_free_amps(h))

    def __init__(self, ctx: Context, ints: Ints, h):
        self.ctx, self.ints, self.h = ctx, ints, h
        ctx.adopt(self)

    def read(self):
        torch = self.ctx.torch
        o, v = self.ints.o, self.ints.v
        t1 = torch.empty((o, v), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        t2 = torch.empty((o, o, v, v), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        self.ctx.check(lib.fc_amps_read(self.h, t1.data_ptr(), t2.data_ptr()), "fc_amps_read")
        return t1, t2


def cd_ao_pivoted(ctx: Context, M, tau, max_vec, allow_cap=False):
    """Pivoted Cholesky of the symmetric PSD supermatrix M (m x m float64 device tensor), Eq. 21.

    Returns (L (nvec x m device tensor), pivots (numpy int32))."""
    torch = ctx.torch
    if M.dtype != torch.float64 or M.dim() != 2 or M.shape[0] != M.shape[1] or M.device.type != "cuda":
        raise ValueError("cd_ao_pivoted: M must be a square float64 GPU tensor")
    M = M.contiguous()
    m = M.shape[0]
    max_vec = int(min(max_vec, m))
    L = torch.empty((max_vec, m), dtype=torch.float64, device=M.device)
    nv = C.c_int()
    piv = np.zeros(max_vec, dtype=np.int32)
    rc = lib.cd_ao_pivoted(ctx.h, m, _ptr(M), float(tau), max_vec, _ptr(L), C.byref(nv), piv.ctypes.data)
    if rc == FC_ENOCONV and allow_cap:
        rc = FC_OK
    ctx.check(rc, "cd_ao_pivoted")
    return L[:nv.value], piv[:nv.value]


def ao_to_spinor(ctx: Context, Lao, Cspin, nao):
    """Spinor-basis vectors L^P_pq (nvec x n x n complex128) from real AO vectors (nvec x nao^2) and
    two-component coefficients Cspin (2 nao x n complex128), Eq. 22."""
    torch = ctx.torch
    Lao = Lao.contiguous()
    Cspin = Cspin.contiguous()
    nvec = Lao.shape[0]
    n = Cspin.shape[1]
    if Lao.dtype != torch.float64 or Lao.numel() != nvec * nao * nao:
        raise ValueError("ao_to_spinor: Lao must be nvec x nao^2 float64")
    if Cspin.dtype != torch.complex128 or Cspin.shape[0] != 2 * nao:
        raise ValueError("ao_to_spinor: C must be 2 nao x n complex128")
    out = torch.empty((nvec, n, n), dtype=torch.complex128, device=Lao.device)
    ctx.check(lib.ao_to_spinor(ctx.h, nvec, nao, n, _ptr(Lao), _ptr(Cspin), _ptr(out)), "ao_to_spinor")
    return out


def cd_integrals(ctx: Context, eps, L, o, precision="fp64"):
    """Stage Cholesky vectors L[P, p, q] (numpy host array or torch device tensor) and build integrals."""
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    if eps.ndim != 1:
        raise ValueError("cd_integrals: eps must be a vector of n spinor energies")
    n = eps.shape[0]
    v = n - o
    if L.ndim != 3 or L.shape[1] != n or L.shape[2] != n:
        raise ValueError(f"cd_integrals: L must be (ncd, {n}, {n}), got {tuple(L.shape)}")
    ncd = L.shape[0]
    if isinstance(L, np.ndarray):
        if L.dtype not in (np.complex128, np.complex64):
            raise ValueError(f"cd_integrals: L dtype {L.dtype} is neither complex128 nor complex64")
        L = np.ascontiguousarray(L)
        dt = FC_C128 if L.dtype == np.complex128 else FC_C64
        on_dev = 0
    else:
        _require(L, "cd_integrals: L", (torch.complex128, torch.complex64))
        dt = FC_C128 if L.dtype == torch.complex128 else FC_C64
        on_dev = 1
    h = P()
    rc = lib.cd_integrals(ctx.h, o, v, ncd, eps.ctypes.data, _ptr(L), dt, on_dev,
                          PRECISION.get(precision, precision), C.byref(h))
    ctx.check(rc, "cd_integrals")
    return Ints(ctx, h, o, v, ncd)


def fns_truncate(ctx: Context, ints: Ints, thresh):
    vk = C.c_int()
    occ = np.zeros(ints.v)
    h = P()
    rc = lib.fns_truncate(ctx.h, ints.h, float(thresh), C.byref(h), C.byref(vk), occ.ctypes.data, None)
    ctx.check(rc, "fns_truncate")
    return Ints(ctx, h, ints.o, vk.value, ints.ncd), occ


def ccsd_opts(**kw):
    op = CcsdOpts()
    lib.fc_ccsd_default_opts(C.byref(op))
    for k, val in kw.items():
        if k == "precision":
            val = PRECISION.get(val, val)
        elif k == "mlp":
            val = val.h if val is not None else None
            if val is not None:
                op.learned = 1
        elif k == "on_iter":
            val = ON_ITER_FN(val)
        elif k in ("t1_init", "t2_init"):   # contiguous device tensors (full layout) or None; the
            if val is not None:                # caller keeps them alive during the solve
                _require(val, k, _C128)
            val = _ptr(val)
        setattr(op, k, val)
    return op


def ccsd_solve(ctx: Context, ints, allow_noconv=False, **kw):
    """Returns (E_corr complex, iterations, Amps) for one handle or lists for several."""
    single = isinstance(ints, Ints)
    lst = [ints] if single else list(ints)
    nb = len(lst)
    arr = (P * nb)(*[x.h for x in lst])
    outs = (P * nb)()
    e = np.zeros(2 * nb)
    it = np.zeros(nb, dtype=np.int32)
    op = ccsd_opts(**kw)
    keep = op.on_iter  # the C callback must outlive the call
    rc = lib.ccsd_solve(ctx.h, nb, arr, C.byref(op), outs, e.ctypes.data, it.ctypes.data)
    del keep
    if rc == FC_ENOCONV and allow_noconv:
        rc = FC_OK
    amps = [Amps(ctx, x, P(outs[b])) for b, x in enumerate(lst)]
    ctx.check(rc, "ccsd_solve")
    E = e[0::2] + 1j * e[1::2]
    if single:
        return complex(E[0]), int(it[0]), amps[0]
    return E, it, amps


def _check_amplitudes(ints: Ints, t1, t2, what):
    o, v = ints.o, ints.v
    _require(t1, f"{what}: t1", _C128, (o, v))
    _require(t2, f"{what}: t2", _C128, (o, o, v, v))


def ccsd_residual(ctx: Context, ints: Ints, t1, t2, precision=-1):
    _check_amplitudes(ints, t1, t2, "ccsd_residual")
    r1 = torch.empty_like(t1)
    r2 = torch.empty_like(t2)
    ctx.check(lib.ccsd_residual(ctx.h, ints.h, _ptr(t1), _ptr(t2), _ptr(r1), _ptr(r2),
                                PRECISION.get(precision, precision)), "ccsd_residual")
    return r1, r2


def ladder(ctx: Context, ints: Ints, tau, t1=None, precision=-1, out=None):
    o, v = ints.o, ints.v
    _require(tau, "ladder: tau", _C128, (o, o, v, v))
    if t1 is not None:
        _require(t1, "ladder: t1", _C128, (o, v))
    if out is not None:
        _require(out, "ladder: out", _C128, (o, o, v, v))
    R = out if out is not None else torch.empty_like(tau)
    ctx.check(lib.fc_ladder(ctx.h, ints.h, _ptr(tau), _ptr(t1), _ptr(R), PRECISION.get(precision, precision)),
              "fc_ladder")
    return R


def ladder_packed(ctx: Context, ints: Ints, taup, t1=None, precision=-1, out=None):
    """The ladder on packed amplitudes: taup[pij][pef] (i<j, e<f) -> R[pij][pab] (i<j, a<b)."""
    o, v = ints.o, ints.v
    shape = (o * (o - 1) // 2, v * (v - 1) // 2)
    _require(taup, "ladder_packed: taup", _C128, shape)
    if t1 is not None:
        _require(t1, "ladder_packed: t1", _C128, (o, v))
    if out is not None:
        _require(out, "ladder_packed: out", _C128, shape)
    R = out if out is not None else torch.empty(shape, dtype=torch.complex128, device=taup.device)
    ctx.check(lib.fc_ladder_packed(ctx.h, ints.h, _ptr(taup), _ptr(t1), _ptr(R), PRECISION.get(precision, precision)),
              "fc_ladder_packed")
    return R


def zgemm(ctx: Context, opA, opB, A, B, alpha=1.0, beta=0.0, C=None, fp32=False, noalloc=False, precision=None):
    """C = alpha op(A) op(B) + beta C on the library's complex GEMM (2-D contiguous tensors);
    FP64 arithmetic, or FP32 arithmetic on the FP64 data with fp32=True, or the hi/lo split
    products with precision="split-bf16" / "split-fp16" (opA N or R, opB T or C).  noalloc=True
    calls fc_zgemm_noalloc (no device allocation inside the library; C must then be given)."""
    if opA not in "NTCR" or opB not in "NTCR" or len(opA) != 1 or len(opB) != 1:
        raise ValueError("zgemm: op must be one of N, T, C, R")
    if precision is None:
        prec = FC_FP32 if fp32 else FC_FP64
    else:
        prec = {"fp32": FC_FP32, **PRECISION}.get(precision, precision)
        if prec not in (FC_FP64, FC_FP32, FC_SPLIT_BF16, FC_SPLIT_FP16):
            raise ValueError(f"zgemm: unknown precision {precision!r}")
        if noalloc and prec in (FC_SPLIT_BF16, FC_SPLIT_FP16):
            raise ValueError("zgemm: the allocation-free product has no split precisions")
    _require(A, "zgemm: A", _C128)
    _require(B, "zgemm: B", _C128)
    if A.dim() != 2 or B.dim() != 2:
        raise ValueError("zgemm: A and B must be 2-D")
    tA, tB = opA in "TC", opB in "TC"
    M, K = (A.shape[1], A.shape[0]) if tA else (A.shape[0], A.shape[1])
    N = B.shape[0] if tB else B.shape[1]
    if (B.shape[1] if tB else B.shape[0]) != K:
        raise ValueError("zgemm: inner dimensions differ")
    if C is None:
        if noalloc:
            raise ValueError("zgemm: the allocation-free product writes into a given C")
        C = torch.zeros((M, N), dtype=torch.complex128, device=A.device)
    else:
        _require(C, "zgemm: C", _C128, (M, N))
    al = np.array([complex(alpha).real, complex(alpha).imag])
    be = np.array([complex(beta).real, complex(beta).imag])
    fn, name = (lib.fc_zgemm_noalloc, "fc_zgemm_noalloc") if noalloc else (lib.fc_zgemm, "fc_zgemm")
    ctx.check(fn(ctx.h, opA.encode(), opB.encode(), M, N, K, al.ctypes.data, _ptr(A), A.shape[1],
                 _ptr(B), B.shape[1], be.ctypes.data, _ptr(C), C.shape[1], prec), name)
    return C


def amps_create(ctx: Context, ints: Ints, t1, t2):
    _check_amplitudes(ints, t1, t2, "amps_create")
    h = P()
    ctx.check(lib.fc_amps_create(ctx.h, ints.h, _ptr(t1), _ptr(t2), C.byref(h)), "fc_amps_create")
    return Amps(ctx, ints, h)


def _check_ip_block(ints: Ints, R, what):
    if not isinstance(R, torch.Tensor):
        raise ValueError(f"{what}: expected a torch tensor on the GPU")
    R = R.contiguous()
    if R.dim() == 1:
        R = R[None]
    if R.dim() != 2:
        raise ValueError(f"{what}: vectors must be (nvec, dim)")
    return _require(R, what, _C128, (R.shape[0], ints.dim))


def ipeom_sigma(ctx: Context, ints: Ints, amps: Amps, R):
    R = _check_ip_block(ints, R, "ipeom_sigma: R")
    S = torch.empty_like(R)
    ctx.check(lib.ipeom_sigma(ctx.h, ints.h, amps.h, R.shape[0], _ptr(R), _ptr(S)), "ipeom_sigma")
    return S


def ipeom_sigma_left(ctx: Context, ints: Ints, amps: Amps, Y):
    """Rows of Y times the IP-EOM-CCSD matrix (the left product of Eq. 19-20)."""
    Y = _check_ip_block(ints, Y, "ipeom_sigma_left: Y")
    S = torch.empty_like(Y)
    ctx.check(lib.ipeom_sigma_left(ctx.h, ints.h, amps.h, Y.shape[0], _ptr(Y), _ptr(S)), "ipeom_sigma_left")
    return S


def eom_opts(**kw):
    op = EomOpts()
    lib.fc_eom_default_opts(C.byref(op))
    for k, val in kw.items():
        setattr(op, k, val)
    return op


def ipeom_davidson(ctx: Context, ints, amps, nroots, want_vectors=False, allow_noconv=False, **kw):
    """Lowest-nroots IPs (complex, ascending real part); optionally the right eigenvectors."""
    torch = ctx.torch
    single = isinstance(ints, Ints)
    il = [ints] if single else list(ints)
    al = [amps] if single else list(amps)
    nr = [nroots] * len(il) if isinstance(nroots, int) else list(nroots)
    nb = len(il)
    ai = (P * nb)(*[x.h for x in il])
    aa = (P * nb)(*[x.h for x in al])
    nra = np.array(nr, dtype=np.int32)
    om = np.zeros(2 * sum(nr))
    its = np.zeros(nb, dtype=np.int32)
    Rout = None
    if want_vectors:
        Rout = torch.empty(sum(k * x.dim for k, x in zip(nr, il)), dtype=torch.complex128,
                           device=f"cuda:{ctx.device}")
    op = eom_opts(**kw)
    rc = lib.ipeom_davidson(ctx.h, nb, ai, aa, nra.ctypes.data, C.byref(op), om.ctypes.data, _ptr(Rout),
                            its.ctypes.data)
    if rc == FC_ENOCONV and allow_noconv:
        rc = FC_OK
    ctx.check(rc, "ipeom_davidson")
    w = om[0::2] + 1j * om[1::2]
    if single:
        vecs = Rout.view(nr[0], il[0].dim) if want_vectors else None
        return (w, int(its[0]), vecs) if want_vectors else (w, int(its[0]))
    return (w, its, Rout) if want_vectors else (w, its)


def ipeom_left(ctx: Context, ints, amps, nroots, R, allow_noconv=False, **kw):
    """Left eigenvectors dual to the right eigenvectors R of ipeom_davidson (Eq. 19-20).

    Returns (omega_left, iters, L, weight): L has the layout of R with sum_x L_k[x] R_l[x] = delta_kl,
    weight[k] = sum_i l^i_k r_{k,i} (complex)."""
    torch = ctx.torch
    single = isinstance(ints, Ints)
    il = [ints] if single else list(ints)
    al = [amps] if single else list(amps)
    nr = [nroots] * len(il) if isinstance(nroots, int) else list(nroots)
    nb = len(il)
    total = sum(k * x.dim for k, x in zip(nr, il))
    R = R.contiguous().reshape(-1)
    if R.dtype != torch.complex128 or R.numel() != total or R.device.type != "cuda":
        raise ValueError(f"ipeom_left: R must be {total} complex128 entries on the GPU")
    ai = (P * nb)(*[x.h for x in il])
    aa = (P * nb)(*[x.h for x in al])
    nra = np.array(nr, dtype=np.int32)
    om = np.zeros(2 * sum(nr))
    wt = np.zeros(2 * sum(nr))
    its = np.zeros(nb, dtype=np.int32)
    L = torch.empty(total, dtype=torch.complex128, device=f"cuda:{ctx.device}")
    op = eom_opts(**kw)
    rc = lib.ipeom_left(ctx.h, nb, ai, aa, nra.ctypes.data, C.byref(op), _ptr(R), om.ctypes.data, _ptr(L),
                        wt.ctypes.data, its.ctypes.data)
    if rc == FC_ENOCONV and allow_noconv:
        rc = FC_OK
    ctx.check(rc, "ipeom_left")
    w = om[0::2] + 1j * om[1::2]
    weight = wt[0::2] + 1j * wt[1::2]
    if single:
        return w, int(its[0]), L.view(nr[0], il[0].dim), weight
    return w, its, L, weight


# ------------------------------------------------------------------------------ learned update
class Mlp(_Handle):
    """Handle of the learned T2-update network (FP32 master weights, BF16 copy for the solver)."""

    _free_fn = staticmethod(lambda h: lib.fc_mlp_free(h))

    def __init__(self, ctx: Context, params=None, seed=0):
        self.ctx = ctx
        h = P()
        arr = None
        if params is not None:
            arr = np.ascontiguousarray(params, dtype=np.float32)
            assert arr.size == lib.fc_mlp_num_params()
        rc = lib.fc_mlp_create(ctx.h, arr.ctypes.data if arr is not None else None, seed, C.byref(h))
        ctx.check(rc, "fc_mlp_create")
        self.h = h
        ctx.adopt(self)

    @staticmethod
    def num_params():
        return int(lib.fc_mlp_num_params())

    def params(self, bf16=False):
        out = np.zeros(self.num_params(), dtype=np.float32)
        self.ctx.check(lib.fc_mlp_get_params(self.h, out.ctypes.data, int(bf16)), "fc_mlp_get_params")
        return out

    def grad(self, X, q, r):
        g = np.zeros(self.num_params(), dtype=np.float32)
        loss = C.c_float()
        self.ctx.check(lib.fc_mlp_grad(self.h, _ptr(X), _ptr(q), _ptr(r), X.shape[0], g.ctypes.data, C.byref(loss)),
                       "fc_mlp_grad")
        return g, float(loss.value)

    def train_step(self, X, q, r, lr):
        loss = C.c_float()
        self.ctx.check(lib.fc_mlp_train_step(self.h, _ptr(X), _ptr(q), _ptr(r), X.shape[0], float(lr),
                                             C.byref(loss)), "fc_mlp_train_step")
        return float(loss.value)

    def forward(self, X, bf16=False):
        torch = self.ctx.torch
        Y = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
        self.ctx.check(lib.fc_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(Y), int(bf16)), "fc_mlp_forward")
        return Y


def learned_step(ctx: Context, ints: Ints, mlp: Mlp, t1, t2, r1, r2, r2prev, fdiag):
    """One learned amplitude update (device tensors, complex128); returns (t1_new, t2_new)."""
    o, v = ints.o, ints.v
    for name, x, shp in (("t1", t1, (o, v)), ("t2", t2, (o, o, v, v)), ("r1", r1, (o, v)),
                         ("r2", r2, (o, o, v, v)), ("fdiag", fdiag, (o + v,))):
        _require(x, f"learned_step: {name}", _C128, shp)
    if r2prev is not None:
        _require(r2prev, "learned_step: r2prev", _C128, (o, o, v, v))
    o1, o2 = torch.empty_like(t1), torch.empty_like(t2)
    ctx.check(lib.fc_learned_step(ctx.h, ints.h, mlp.h, _ptr(t1), _ptr(t2), _ptr(r1), _ptr(r2), _ptr(r2prev),
                                  _ptr(fdiag), _ptr(o1), _ptr(o2)), "fc_learned_step")
    return o1, o2


def learn_samples(ctx: Context, ints: Ints, t1_ptr, t2_ptr, t2_star, nsamp, seed, out=None, offset=0, prev=None):
    """Training samples at an iterate; t1_ptr/t2_ptr are device addresses or tensors, prev the
    previous iterate (t1, t2) tensors or None."""
    torch = ctx.torch
    if out is None:
        dev = f"cuda:{ctx.device}"
        out = (torch.empty((nsamp, 4), dtype=torch.float32, device=dev),
               torch.empty((nsamp, 2), dtype=torch.float32, device=dev),
               torch.empty((nsamp, 2), dtype=torch.float32, device=dev))
        offset = 0
    X, q, r = out
    a1 = t1_ptr if isinstance(t1_ptr, int) else _ptr(t1_ptr)
    a2 = t2_ptr if isinstance(t2_ptr, int) else _ptr(t2_ptr)
    p1, p2 = (None, None) if prev is None else (_ptr(prev[0]), _ptr(prev[1]))
    rc = lib.fc_learn_samples(ctx.h, ints.h, a1, a2, p1, p2, _ptr(t2_star), nsamp, seed,
                              X.data_ptr() + 16 * offset, q.data_ptr() + 8 * offset, r.data_ptr() + 8 * offset)
    ctx.check(rc, "fc_learn_samples")
    return out


def device_copy(ctx: Context, ptr, shape):
    """complex128 tensor copied from a device address (an iterate handed to a callback)."""
    torch = ctx.torch

    class _View:
        __cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<c16", "data": (int(ptr), False),
                                    "version": 2, "strides": None}

    return torch.as_tensor(_View(), device=f"cuda:{ctx.device}").clone()
