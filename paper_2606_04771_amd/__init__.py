"""MI355X (gfx950) two-site TDVP hot path for the U(1)xSU(2) Hubbard chain.

Thin ctypes binding of ``libtdvp.so`` (C ABI declared in include/tdvp.h).
It only marshals arguments: every step of the computation runs in the HIP
library.  Device buffers are passed as raw pointers (e.g. from torch
tensors); the binding allocates nothing on the device itself.

The library is loaded on first use (so that ``paper_2606_04771_amd.build``
imports in a fresh checkout); any call before it has been built
(``python -m paper_2606_04771_amd.build``) fails loudly: there is no fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdvp.so")

TDVP_OK = 0
ERRORS = {-1: "INVALID", -2: "SHAPE", -3: "SECTOR", -4: "NOMEM", -5: "HIP", -6: "NOCONV", -7: "NONFINITE"}
FP64, FP32, BF16X3 = 0, 1, 2


class TdvpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdvp error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class _Model(C.Structure):
    _fields_ = [("t", C.c_double), ("U", C.c_double), ("L", C.c_int32)]


class _Bond(C.Structure):
    _fields_ = [("n", C.c_int32), ("q", C.POINTER(C.c_int32)), ("tj", C.POINTER(C.c_int32)),
                ("dim", C.POINTER(C.c_int64))]


class _Blocks(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("keys", C.POINTER(C.c_int32)), ("offsets", C.POINTER(C.c_int64)),
                ("data", C.c_void_p), ("size", C.c_int64)]


class _KrylovInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("err_est", C.c_double),
                ("norm_in", C.c_double), ("alpha", C.c_double * 64), ("beta", C.c_double * 64),
                ("graph_iters", C.c_int32)]


class _Trunc(C.Structure):
    _fields_ = [("eps_tol", C.c_double), ("chi_cap", C.c_int64), ("keep_all", C.c_int32),
                ("krylov_tol", C.c_double), ("krylov_maxdim", C.c_int32)]


class _SweepInfo(C.Structure):
    _fields_ = [("max_discarded", C.c_double), ("sum_discarded", C.c_double), ("max_chi", C.c_int64),
                ("max_chi_su2", C.c_int64), ("krylov_iters", C.c_int32), ("krylov_max", C.c_int32),
                ("nonconverged", C.c_int32), ("heff_flops", C.c_double), ("env_flops", C.c_double),
                ("seconds", C.c_double), ("t_heff", C.c_double), ("t_lanczos", C.c_double),
                ("t_svd", C.c_double), ("t_env", C.c_double), ("graph_iters", C.c_int32),
                ("eig_fallbacks", C.c_int32)]


class _Term(C.Structure):
    _fields_ = [("kind", C.c_int32), ("out", C.c_int32), ("in_", C.c_int32), ("env", C.c_int32),
                ("coef", C.c_double)]


class _EnvTerm(C.Structure):
    _fields_ = [("kind", C.c_int32), ("out", C.c_int32), ("bra", C.c_int32), ("ket", C.c_int32),
                ("env", C.c_int32), ("coef", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_04771_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "tdvp_ctx_create": [C.POINTER(C.c_void_p), I32, P, I32, P, P, P],
        "tdvp_ctx_set_split": [P, D, I32],
        "tdvp_ctx_set_krylov_storage": [P, I32],
        "tdvp_ctx_set_host_staging": [P, I32],
        "tdvp_ctx_memory": [P, P, P, I32],
        "tdvp_split_sectors": [P, P, P, P, P, P, P],
        "tdvp_split": [P, P, P, P, I32, P, P, P, P],
        "tdvp_ctx_destroy": [P],
        "tdvp_ctx_set_precision": [P, I32],
        "tdvp_ctx_set_graphs": [P, I32],
        "tdvp_ctx_synchronize": [P],
        "tdvp_last_error": [P],
        "tdvp_center_layout": [P, P, I32, P, P, P, P],
        "tdvp_env_layout": [P, P, P, P, P],
        "tdvp_heff_apply": [P, P, I32, I32, P, P, P, P, P, P],
        "tdvp_heff_plan": [P, I32, I32, P, P, P, P, P, P, P, P],
        "tdvp_krylov_expm": [P, P, I32, I32, P, P, P, P, P, D, D, D, I32, P],
        "tdvp_tridiag_expm": [I32, P, P, D, D, D, P],
        "tdvp_env_update": [P, P, I32, I32, P, P, P, P, P],
        "tdvp_env_update_noalloc": [P, P, I32, I32, P, P, P, P, P],
        "tdvp_env_plan": [P, I32, I32, P, P, P, P, P, P, P, P],
        "tdvp_u1_center_layout": [P, P, I32, P, P, P, P],
        "tdvp_u1_env_layout": [P, P, P, P, P],
        "tdvp_u1_heff_plan": [P, I32, I32, P, P, P, P, P, P, P, P],
        "tdvp_u1_env_plan": [P, I32, I32, P, P, P, P, P, P, P, P],
        "tdvp_u1_heff_apply": [P, P, I32, I32, P, P, P, P, P, P],
        "tdvp_u1_krylov_expm": [P, P, I32, I32, P, P, P, P, P, D, D, D, I32, P],
        "tdvp_u1_env_update": [P, P, I32, I32, P, P, P, P, P],
        "tdvp_mps_create": [P, P, P, P, P],
        "tdvp_mps_create_neel": [P, P, I32, P],
        "tdvp_u1_mps_create": [P, P, P, P, P],
        "tdvp_u1_mps_create_neel": [P, P, I32, P],
        "tdvp_mps_destroy": [P],
        "tdvp_mps_bond": [P, I32, P, P, P, P],
        "tdvp_mps_site_layout": [P, I32, P, P, P, P],
        "tdvp_mps_site_read": [P, P, I32, P],
        "tdvp_sweep": [P, P, D, P, P],
        "tdvp_mps_measure": [P, P, P, P, P],
        "tdvp_mps_overlap": [P, P, P, P],
        "tdvp_sweep1": [P, P, D, P, P],
        "tdvp_step": [P, P, D, P, D, P, P],
    }
    for name, args in sig.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name == "tdvp_last_error" else (None if name.endswith("destroy") else C.c_int)
    return lib


class _LazyLib:
    """Loads libtdvp.so at the first attribute access and forwards to it."""

    def __init__(self):
        self._lib = None

    def __getattr__(self, name):
        if name.startswith("__"):
            raise AttributeError(name)
        if self._lib is None:
            self._lib = _load()
        return getattr(self._lib, name)


lib = _LazyLib()


def _check(rc, ctx=None):
    if rc != TDVP_OK:
        msg = lib.tdvp_last_error(ctx)
        raise TdvpError(rc, msg.decode() if msg else "")


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Model:
    def __init__(self, L, t=1.0, U=4.0):
        self.L, self.t, self.U = int(L), float(t), float(U)
        self._s = _Model(self.t, self.U, self.L)

    @property
    def ref(self):
        return C.byref(self._s)


class Bond:
    """A bond as sectors [(q, tj, d), ...]."""

    def __init__(self, sectors):
        self.sectors = [(int(q), int(tj), int(d)) for q, tj, d in sectors]
        n = len(self.sectors)
        self.q = np.array([s[0] for s in self.sectors], np.int32)
        self.tj = np.array([s[1] for s in self.sectors], np.int32)
        self.d = np.array([s[2] for s in self.sectors], np.int64)
        self._s = _Bond(n, self.q.ctypes.data_as(C.POINTER(C.c_int32)),
                        self.tj.ctypes.data_as(C.POINTER(C.c_int32)),
                        self.d.ctypes.data_as(C.POINTER(C.c_int64)))

    @property
    def ref(self):
        return C.byref(self._s)

    def __len__(self):
        return len(self.sectors)


class Blocks:
    """Block descriptor: keys (n x keylen int32), offsets (int64), device
    data pointer (int) and size in complex elements."""

    def __init__(self, keys, offsets, data_ptr=0, size=None, dims=None):
        self.keys = np.ascontiguousarray(np.asarray(keys, np.int32).reshape(len(offsets), -1))
        self.offsets = np.ascontiguousarray(np.asarray(offsets, np.int64))
        self.dims = dims
        if size is None:
            size = int(max((o + r * c for o, (r, c) in zip(self.offsets, dims)), default=0)) if dims else 0
        self.size = int(size)
        self.set_data(data_ptr)

    def set_data(self, data_ptr):
        self.data_ptr = int(data_ptr)
        self._s = _Blocks(len(self.offsets), self.keys.ctypes.data_as(C.POINTER(C.c_int32)),
                          self.offsets.ctypes.data_as(C.POINTER(C.c_int64)), C.c_void_p(self.data_ptr or None),
                          self.size)
        return self

    @property
    def ref(self):
        return C.byref(self._s)

    def __len__(self):
        return len(self.offsets)


def center_layout(left, right, nsites, abelian=False):
    """Canonical blocks of a centre tensor: (keys, offsets, total, dims).
    abelian: the U(1) x U(1) variant (bonds (2Sz, N, d); two-site keys
    (ia, s1, s2, ib))."""
    f = lib.tdvp_u1_center_layout if abelian else lib.tdvp_center_layout
    n = C.c_int32()
    tot = C.c_int64()
    _check(f(left.ref, right.ref, nsites, C.byref(n), None, None, C.byref(tot)))
    kl = (4 if abelian else 5) if nsites == 2 else 3
    keys = np.zeros((n.value, kl), np.int32)
    offs = np.zeros(n.value, np.int64)
    _check(f(left.ref, right.ref, nsites, C.byref(n), _ptr(keys), _ptr(offs), C.byref(tot)))
    dims = [(left.sectors[k[0]][2], right.sectors[k[-1]][2]) for k in keys]
    return keys, offs, tot.value, dims


def env_layout(bond, abelian=False):
    f = lib.tdvp_u1_env_layout if abelian else lib.tdvp_env_layout
    n = C.c_int32()
    tot = C.c_int64()
    _check(f(bond.ref, C.byref(n), None, None, C.byref(tot)))
    keys = np.zeros((n.value, 3), np.int32)
    offs = np.zeros(n.value, np.int64)
    _check(f(bond.ref, C.byref(n), _ptr(keys), _ptr(offs), C.byref(tot)))
    dims = [(bond.sectors[k[0]][2], bond.sectors[k[2]][2]) for k in keys]
    return keys, offs, tot.value, dims


def heff_plan(model, site, nsites, left, right, Lenv, Renv, x, abelian=False):
    """Host-side term list of one H_eff apply: structured array with fields
    kind, out, in_, env, coef; and the algorithmic flop count."""
    f = lib.tdvp_u1_heff_plan if abelian else lib.tdvp_heff_plan
    nt = C.c_int64(0)
    fl = C.c_double()
    _check(f(model.ref, site, nsites, left.ref, right.ref, Lenv.ref, Renv.ref, x.ref, C.byref(nt), None,
             C.byref(fl)))
    arr = (_Term * nt.value)()
    _check(f(model.ref, site, nsites, left.ref, right.ref, Lenv.ref, Renv.ref, x.ref, C.byref(nt), arr,
             C.byref(fl)))
    return [(t.kind, t.out, t.in_, t.env, t.coef) for t in arr], fl.value


def env_plan(model, site, direction, bond_in, bond_out, env_in, tensor, env_out, abelian=False):
    f = lib.tdvp_u1_env_plan if abelian else lib.tdvp_env_plan
    nt = C.c_int64(0)
    fl = C.c_double()
    _check(f(model.ref, site, direction, bond_in.ref, bond_out.ref, env_in.ref, tensor.ref, env_out.ref,
             C.byref(nt), None, C.byref(fl)))
    arr = (_EnvTerm * nt.value)()
    _check(f(model.ref, site, direction, bond_in.ref, bond_out.ref, env_in.ref, tensor.ref, env_out.ref,
             C.byref(nt), arr, C.byref(fl)))
    return [(t.kind, t.out, t.bra, t.ket, t.env, t.coef) for t in arr], fl.value


def split_sectors(left, right):
    """Coupled sectors of the bond between two sites: [(q, tj, rows, cols)]."""
    n = C.c_int32()
    _check(lib.tdvp_split_sectors(left.ref, right.ref, C.byref(n), None, None, None, None))
    q = np.zeros(n.value, np.int32)
    tj = np.zeros(n.value, np.int32)
    r = np.zeros(n.value, np.int64)
    c = np.zeros(n.value, np.int64)
    _check(lib.tdvp_split_sectors(left.ref, right.ref, C.byref(n), _ptr(q), _ptr(tj), _ptr(r), _ptr(c)))
    return [(int(a), int(b), int(x), int(y)) for a, b, x, y in zip(q, tj, r, c)]


def tridiag_expm(alpha, beta, tau, nrm=1.0):
    a = np.ascontiguousarray(alpha, np.float64)
    b = np.ascontiguousarray(beta if len(beta) else [0.0], np.float64)
    y = np.zeros(2 * len(a))
    _check(lib.tdvp_tridiag_expm(len(a), _ptr(a), _ptr(b), float(np.real(tau)), float(np.imag(tau)),
                                 float(nrm), _ptr(y)))
    return y[0::2] + 1j * y[1::2]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


def torch_allocator(device, stream):
    """(dev_alloc, dev_free) callbacks on torch's caching allocator, bound to
    the raw stream handle the context runs on (stream-ordered reuse)."""
    import torch

    def alloc(n, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(n), device, int(stream))
        except Exception:
            return None

    def free(p, user):
        torch.cuda.caching_allocator_delete(int(p))

    return _ALLOC_FN(alloc), _FREE_FN(free)


class Context:
    """A library context on one HIP device and stream.

    allocator: "torch" (default when a stream is given: device memory from
    torch's caching allocator on that stream), None (hipMalloc), or a pair of
    ctypes callbacks (dev_alloc(bytes, user) -> ptr, dev_free(ptr, user))."""

    def __init__(self, device=0, stream=None, precision=FP64, allocator="torch"):
        if allocator == "torch":
            allocator = torch_allocator(int(device), stream) if stream else None
        self._alloc = allocator
        a, f = allocator if allocator else (None, None)
        h = C.c_void_p()
        _check(lib.tdvp_ctx_create(C.byref(h), int(device), C.c_void_p(stream), int(precision),
                                   C.cast(a, C.c_void_p) if a else None,
                                   C.cast(f, C.c_void_p) if f else None, None))
        self.h = h

    def close(self):
        if self.h:
            lib.tdvp_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, p):
        _check(lib.tdvp_ctx_set_precision(self.h, int(p)), self.h)

    def set_graphs(self, enable):
        _check(lib.tdvp_ctx_set_graphs(self.h, int(bool(enable))), self.h)

    def set_krylov_storage(self, precision):
        """Krylov basis storage: FP64 (default) or FP32 (complex64 basis vectors)."""
        _check(lib.tdvp_ctx_set_krylov_storage(self.h, int(precision)), self.h)

    def set_host_staging(self, enable):
        """Sweeps keep inactive MPS tensors and environments in pinned host memory."""
        _check(lib.tdvp_ctx_set_host_staging(self.h, int(bool(enable))), self.h)

    def memory(self, reset_peak=False):
        """(live, peak) device bytes held through the context's allocator."""
        live, peak = C.c_int64(), C.c_int64()
        _check(lib.tdvp_ctx_memory(self.h, C.byref(live), C.byref(peak), int(bool(reset_peak))), self.h)
        return live.value, peak.value

    def set_split(self, alpha=-1.0, kmin=128):
        """K-chain splitting of effective-Hamiltonian launches (alpha < 0: size rule)."""
        _check(lib.tdvp_ctx_set_split(self.h, float(alpha), int(kmin)), self.h)

    def split(self, left, right, theta, direction, eps_tol=1e-4, chi_cap=4096, keep_all=False):
        """Two-site split of theta (Blocks on the device).  Returns (MPS of two
        sites holding the result, {(q, tj): reduced singular values}, discarded)."""
        sec = split_sectors(left, right)
        n = sum(min(r, c) for _, _, r, c in sec)
        sv = np.zeros(max(n, 1))
        disc = C.c_double()
        tr = _Trunc(float(eps_tol), int(chi_cap), int(bool(keep_all)), 1e-12, 40)
        h = C.c_void_p()
        _check(lib.tdvp_split(self.h, left.ref, right.ref, theta.ref, int(direction), C.byref(tr), C.byref(h),
                              _ptr(sv), C.byref(disc)), self.h)
        out, o = {}, 0
        for q, tj, r, c in sec:
            k = min(r, c)
            out[(q, tj)] = sv[o:o + k].copy()
            o += k
        return MPS(self, h, Model(2, 0.0, 0.0)), out, disc.value

    def synchronize(self):
        _check(lib.tdvp_ctx_synchronize(self.h), self.h)

    def heff_apply(self, model, site, nsites, left, right, Lenv, Renv, x, y, abelian=False):
        f = lib.tdvp_u1_heff_apply if abelian else lib.tdvp_heff_apply
        _check(f(self.h, model.ref, site, nsites, left.ref, right.ref, Lenv.ref, Renv.ref, x.ref, y.ref), self.h)

    def krylov_expm(self, model, site, nsites, left, right, Lenv, Renv, x, tau, tol=1e-12, maxdim=40,
                    check=True, abelian=False):
        info = _KrylovInfo()
        f = lib.tdvp_u1_krylov_expm if abelian else lib.tdvp_krylov_expm
        rc = f(self.h, model.ref, site, nsites, left.ref, right.ref, Lenv.ref, Renv.ref, x.ref,
               float(np.real(tau)), float(np.imag(tau)), float(tol), int(maxdim), C.byref(info))
        if check:
            _check(rc, self.h)
        return rc, {"iters": info.iters, "converged": bool(info.converged), "err": info.err_est,
                    "norm": info.norm_in, "alpha": list(info.alpha[:info.iters]),
                    "beta": list(info.beta[:info.iters]), "graph_iters": info.graph_iters}

    def env_update(self, model, site, direction, bond_in, bond_out, env_in, tensor, env_out, abelian=False):
        f = lib.tdvp_u1_env_update if abelian else lib.tdvp_env_update
        _check(f(self.h, model.ref, site, direction, bond_in.ref, bond_out.ref, env_in.ref, tensor.ref,
                 env_out.ref), self.h)

    def env_update_noalloc(self, model, site, direction, bond_in, bond_out, env_in, tensor, env_out):
        _check(lib.tdvp_env_update_noalloc(self.h, model.ref, site, direction, bond_in.ref, bond_out.ref,
                                           env_in.ref, tensor.ref, env_out.ref), self.h)


class MPS:
    """Library-owned MPS (right-canonical, centre on site 1), U(1)xSU(2) or,
    with abelian=True at creation, U(1)xU(1)."""

    def __init__(self, ctx, handle, model, abelian=False):
        self.ctx, self.h, self.model, self.abelian = ctx, handle, model, abelian

    @classmethod
    def neel(cls, ctx, model, complete=False, abelian=False):
        h = C.c_void_p()
        f = lib.tdvp_u1_mps_create_neel if abelian else lib.tdvp_mps_create_neel
        _check(f(ctx.h, model.ref, int(bool(complete)), C.byref(h)), ctx.h)
        return cls(ctx, h, model, abelian)

    @classmethod
    def from_blocks(cls, ctx, model, bonds, sites, abelian=False):
        """bonds: L+1 Bond objects; sites: L Blocks (device data, keys (ia, s, ib))."""
        barr = (_Bond * len(bonds))(*[b._s for b in bonds])
        sarr = (_Blocks * len(sites))(*[s._s for s in sites])
        h = C.c_void_p()
        f = lib.tdvp_u1_mps_create if abelian else lib.tdvp_mps_create
        _check(f(ctx.h, model.ref, barr, sarr, C.byref(h)), ctx.h)
        return cls(ctx, h, model, abelian)

    def close(self):
        if self.h:
            lib.tdvp_mps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bond(self, k):
        n = C.c_int32()
        _check(lib.tdvp_mps_bond(self.h, k, C.byref(n), None, None, None))
        q = np.zeros(n.value, np.int32)
        tj = np.zeros(n.value, np.int32)
        d = np.zeros(n.value, np.int64)
        _check(lib.tdvp_mps_bond(self.h, k, C.byref(n), _ptr(q), _ptr(tj), _ptr(d)))
        return [(int(a), int(b), int(c)) for a, b, c in zip(q, tj, d)]

    def site(self, k):
        """(keys, offsets, host complex data) of site tensor k (1-based)."""
        n = C.c_int32()
        tot = C.c_int64()
        _check(lib.tdvp_mps_site_layout(self.h, k, C.byref(n), None, None, C.byref(tot)))
        keys = np.zeros((n.value, 3), np.int32)
        offs = np.zeros(n.value, np.int64)
        _check(lib.tdvp_mps_site_layout(self.h, k, C.byref(n), _ptr(keys), _ptr(offs), C.byref(tot)))
        data = np.zeros(max(tot.value, 1), np.complex128)
        _check(lib.tdvp_mps_site_read(self.ctx.h, self.h, k, _ptr(data)), self.ctx.h)
        return keys, offs, data[:tot.value]

    def sweep(self, dt, eps_tol=1e-4, chi_cap=4096, keep_all=False, krylov_tol=1e-12, krylov_maxdim=40):
        tr = _Trunc(float(eps_tol), int(chi_cap), int(bool(keep_all)), float(krylov_tol), int(krylov_maxdim))
        info = _SweepInfo()
        _check(lib.tdvp_sweep(self.ctx.h, self.h, float(dt), C.byref(tr), C.byref(info)), self.ctx.h)
        return {f: getattr(info, f) for f, _ in _SweepInfo._fields_}

    def step(self, dt, mode, eps_tol=1e-4, chi_cap=4096, krylov_tol=1e-12, krylov_maxdim=40, switch=0.97):
        """One time step of the adaptive scheme: mode 0 = two-site sweep (then
        1 once the largest bond reaches switch x chi_cap), 1 = one-site sweep.
        Returns (info, new mode)."""
        tr = _Trunc(float(eps_tol), int(chi_cap), 0, float(krylov_tol), int(krylov_maxdim))
        info = _SweepInfo()
        m = C.c_int32(int(mode))
        _check(lib.tdvp_step(self.ctx.h, self.h, float(dt), C.byref(tr), float(switch), C.byref(m), C.byref(info)),
               self.ctx.h)
        return {f: getattr(info, f) for f, _ in _SweepInfo._fields_}, m.value

    def sweep1(self, dt, krylov_tol=1e-12, krylov_maxdim=40):
        """One time step of one-site TDVP (bond dimensions fixed)."""
        tr = _Trunc(0.0, 0, 1, float(krylov_tol), int(krylov_maxdim))
        info = _SweepInfo()
        _check(lib.tdvp_sweep1(self.ctx.h, self.h, float(dt), C.byref(tr), C.byref(info)), self.ctx.h)
        return {f: getattr(info, f) for f, _ in _SweepInfo._fields_}

    def overlap(self, ket):
        """<self|ket> as a complex number."""
        out = np.zeros(2)
        _check(lib.tdvp_mps_overlap(self.ctx.h, self.h, ket.h, _ptr(out)), self.ctx.h)
        return complex(out[0], out[1])

    def measure(self):
        """Site-resolved <S^z_k> and <n_k,up n_k,down> (arrays of L) and the norm^2."""
        sz = np.zeros(self.model.L)
        docc = np.zeros(self.model.L)
        n2 = C.c_double()
        _check(lib.tdvp_mps_measure(self.ctx.h, self.h, _ptr(sz), _ptr(docc), C.byref(n2)), self.ctx.h)
        return sz, docc, n2.value
