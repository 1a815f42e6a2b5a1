"""Python binding of libgf (the C ABI in include/gf.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream, every computation runs in the library's HIP kernels. Importing this
module raises if ``libgf.so`` has not been built; there is no CPU fallback.

Field tensors in the internal layout have shape (2, nb, 4, nelem, 64, 2):
[parity][block of 64 sites][mu][matrix element e = 3*row + col][site in
block][re, im], nb = ceil(V / 128), nelem = 9 (18-real storage) or 6 (12-real
storage), dtype float32 or float64.
Canonical fields are complex tensors of shape (nt, nz, ny, nx, 4, 3, 3).
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED = -1, -2, -3, -4, -5
LANDAU, COULOMB = 0, 1
F64, F32 = 0, 1
STORE_18, STORE_12, STORE_8 = 0, 1, 2

_ERRNAMES = {EINVAL: "GF_EINVAL", ENOMEM: "GF_ENOMEM", EDEVICE: "GF_EDEVICE",
             ENONFINITE: "GF_ENONFINITE", EUNSUPPORTED: "GF_EUNSUPPORTED"}


class GFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("check_every", ctypes.c_int),
        ("reunit_every", ctypes.c_int),
        ("start_sweep", ctypes.c_longlong),
        ("storage", ctypes.c_int),
        ("lanes_per_site", ctypes.c_int),
        ("block_threads", ctypes.c_int),
        ("nontemporal", ctypes.c_int),
        ("use_graph", ctypes.c_int),
        ("timing", ctypes.c_int),
        ("log_path", ctypes.c_char_p),
        ("tile_order", ctypes.c_int),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; call __graft_entry__.build() or "
                          "python -m paper_1412_1498_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    PP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "gf_params_default": (None, [ctypes.POINTER(Params), I]),
        "gf_create": (I, [PP, P, I, I, I, P, ctypes.POINTER(Params)]),
        "gf_batch_create": (I, [PP, I, P, P, I, P, ctypes.POINTER(Params)]),
        "gf_destroy": (I, [P]),
        "gf_batch_destroy": (I, [P]),
        "gf_quality_slices": (I, [P, P, P, P]),
        "gf_quality_noalloc": (I, [P, P, I, I, I, P, P]),
        "gf_last_error": (ctypes.c_char_p, [P]),
        "gf_field_bytes": (ctypes.c_size_t, [P, I]),
        "gf_pack": (I, [P, P, P]),
        "gf_unpack": (I, [P, P, P]),
        "gf_sweep": (I, [P, P, I, D]),
        "gf_sweeps": (I, [P, P, D, I]),
        "gf_reunit": (I, [P, P]),
        "gf_quality": (I, [P, P, P, P]),
        "gf_fix": (I, [P, P, D, D, I, P, P, P]),
        "gf_batch_fix": (I, [P, P, P, D, I, P, P, P]),
        "gf_batch_quality": (I, [P, P, P, P]),
        "gf_autotune": (I, [P, P, D, ctypes.c_char_p]),
        "gf_get_schedule": (I, [P, P, P, P, P]),
        "gf_timing": (I, [P, P, P]),
        "gf_set_sweep_count": (I, [P, LL]),
        "gf_get_sweep_count": (LL, [P]),
        "gf_pack_alg": (I, [P, P, P]),
        "gf_unpack_alg": (I, [P, P, P]),
        "gf_functional": (I, [P, P, P, P]),
        "gf_functional_grad": (I, [P, P, P, D, P]),
        "gf_gauge_transform": (I, [P, P, P]),
        "gf_sd_step": (I, [P, P, D]),
        "gf_sd_fix": (I, [P, P, D, D, I, P, P, P]),
        "gf_host_su2_step": (None, [P, D, P]),
        "gf_host_trig": (None, [D, D, P]),
        "gf_host_link8": (I, [I, P, P, P]),
        "gf_site_links": (I, [P, I, LL, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def default_params(prec=F32, **kw) -> Params:
    p = Params()
    lib.gf_params_default(ctypes.byref(p), prec)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown gf_params field {k}")
        if k == "log_path":
            p.log_path = None if v is None else os.fsencode(v)
        else:
            setattr(p, k, int(v))
    return p


def _dims_arr(dims):
    d = [int(x) for x in dims]
    if len(d) != 4:
        raise ValueError("dims must be (nx, ny, nz, nt)")
    return (ctypes.c_int * 4)(*d)


def _ptr(t: torch.Tensor) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """A libgf context: one lattice, or an ensemble of lattices (n > 1)."""

    def __init__(self, dims, gauge=LANDAU, prec=F32, stream=None, params: Params | None = None,
                 ensemble=None, nc=3):
        """nc: number of colours of a single lattice (3, or 2 / 4 for the SU(N)
        kernels); ensembles are SU(3)."""
        self.prec = prec
        self.nc = int(nc)
        self.rdtype = torch.float64 if prec == F64 else torch.float32
        self.cdtype = torch.complex128 if prec == F64 else torch.complex64
        p = params if params is not None else default_params(prec)
        self.storage = p.storage
        self.nelem = {STORE_12: 6, STORE_8: 4}.get(p.storage, 9) if self.nc == 3 else self.nc * self.nc
        self._h = ctypes.c_void_p()
        sh = _stream_handle(stream)
        if ensemble is None:
            self.members = [(tuple(int(x) for x in dims), int(gauge))]
            rc = lib.gf_create(ctypes.byref(self._h), _dims_arr(dims), self.nc, int(gauge), prec, sh,
                               ctypes.byref(p))
        else:
            if self.nc != 3:
                raise ValueError("ensembles are SU(3) only")
            self.members = [(tuple(int(x) for x in d), int(g)) for d, g in ensemble]
            n = len(self.members)
            dd = (ctypes.c_int * (4 * n))(*[x for d, _ in self.members for x in d])
            gg = (ctypes.c_int * n)(*[g for _, g in self.members])
            rc = lib.gf_batch_create(ctypes.byref(self._h), n, dd, gg, prec, sh, ctypes.byref(p))
        if rc != OK:
            raise GFError(rc, "context creation failed (invalid dims, gauge or precision?)")

    # -- lifetime -------------------------------------------------------------
    def close(self):
        if self._h:
            (lib.gf_batch_destroy if self.n > 1 else lib.gf_destroy)(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc, allow=(OK,)):
        if rc not in allow:
            msg = lib.gf_last_error(self._h)
            raise GFError(rc, msg.decode() if msg else "")
        return rc

    # -- fields ---------------------------------------------------------------
    @property
    def n(self):
        return len(self.members)

    def volume(self, i=0):
        d = self.members[i][0]
        return d[0] * d[1] * d[2] * d[3]

    def field_bytes(self, i=0) -> int:
        return int(lib.gf_field_bytes(self._h, i))

    BLOCK = 64

    def blocks(self, i=0):
        return (self.volume(i) // 2 + self.BLOCK - 1) // self.BLOCK

    def empty_field(self, i=0, device="cuda") -> torch.Tensor:
        # zero-filled, so the padding of the last block is deterministic
        return torch.zeros((2, self.blocks(i), 4, self.nelem, self.BLOCK, 2), dtype=self.rdtype,
                           device=device)

    def _check_field(self, U, i=0):
        n = 2 * self.blocks(i) * 4 * self.nelem * self.BLOCK * 2
        if U.dtype != self.rdtype or U.numel() != n:
            raise ValueError(f"field must be {self.rdtype} with {n} elements")
        return _ptr(U)

    def _canonical_shape(self, i=0):
        d = self.members[i][0]
        return (d[3], d[2], d[1], d[0], 4, self.nc, self.nc)

    def pack(self, U_aos: torch.Tensor, U: torch.Tensor | None = None) -> torch.Tensor:
        """Canonical complex (nt, nz, ny, nx, 4, N, N) -> internal layout."""
        if U_aos.dtype != self.cdtype:
            raise ValueError(f"canonical field must be {self.cdtype}")
        if tuple(U_aos.shape) != self._canonical_shape():
            raise ValueError(f"canonical field must have shape {self._canonical_shape()}")
        if U is None:
            U = self.empty_field(device=U_aos.device)
        self._check(lib.gf_pack(self._h, ctypes.c_void_p(_ptr(U_aos)),
                                ctypes.c_void_p(self._check_field(U))))
        return U

    def unpack(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self._canonical_shape(), dtype=self.cdtype, device=U.device)
        elif tuple(out.shape) != self._canonical_shape() or out.dtype != self.cdtype:
            raise ValueError(f"out must be {self.cdtype} with shape {self._canonical_shape()}")
        self._check(lib.gf_unpack(self._h, ctypes.c_void_p(self._check_field(U)),
                                  ctypes.c_void_p(_ptr(out))))
        return out

    # -- Alg. 1 -----------------------------------------------------------------
    def sweep(self, U, parity, omega):
        self._check(lib.gf_sweep(self._h, ctypes.c_void_p(self._check_field(U)), int(parity), float(omega)))

    def sweeps(self, U, omega, n):
        self._check(lib.gf_sweeps(self._h, ctypes.c_void_p(self._check_field(U)), float(omega), int(n)))

    def reunit(self, U):
        self._check(lib.gf_reunit(self._h, ctypes.c_void_p(self._check_field(U))))

    def quality(self, U):
        F, th = ctypes.c_double(), ctypes.c_double()
        self._check(lib.gf_quality(self._h, ctypes.c_void_p(self._check_field(U)),
                                   ctypes.byref(F), ctypes.byref(th)))
        return F.value, th.value

    def quality_slices(self, U):
        """(F_t, theta_t) per time slice t of member 0, as lists of nt floats."""
        nt = self.members[0][0][3]
        Ft, tht = (ctypes.c_double * nt)(), (ctypes.c_double * nt)()
        self._check(lib.gf_quality_slices(self._h, ctypes.c_void_p(self._check_field(U)), Ft, tht))
        return list(Ft), list(tht)

    def fix(self, U, omega, eps, max_iter):
        it, F, th = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        rc = self._check(lib.gf_fix(self._h, ctypes.c_void_p(self._check_field(U)), float(omega),
                                    float(eps), int(max_iter), ctypes.byref(it), ctypes.byref(F),
                                    ctypes.byref(th)), allow=(OK, NOT_CONVERGED))
        return dict(converged=rc == OK, iters=it.value, F=F.value, theta=th.value)

    def _ptr_array(self, Us):
        if len(Us) != self.n:
            raise ValueError(f"expected {self.n} fields")
        return (ctypes.c_void_p * self.n)(*[self._check_field(u, i) for i, u in enumerate(Us)])

    def batch_fix(self, Us, omega, eps, max_iter):
        n = self.n
        om = omega if hasattr(omega, "__len__") else [omega] * n
        oo = (ctypes.c_double * n)(*[float(x) for x in om])
        it = (ctypes.c_int * n)()
        F = (ctypes.c_double * n)()
        th = (ctypes.c_double * n)()
        rc = self._check(lib.gf_batch_fix(self._h, self._ptr_array(Us), oo, float(eps), int(max_iter),
                                          it, F, th), allow=(OK, NOT_CONVERGED))
        return dict(converged=rc == OK, iters=list(it), F=list(F), theta=list(th))

    def batch_quality(self, Us):
        n = self.n
        F = (ctypes.c_double * n)()
        th = (ctypes.c_double * n)()
        self._check(lib.gf_batch_quality(self._h, self._ptr_array(Us), F, th))
        return list(F), list(th)

    # -- steepest descent with Fourier acceleration (Alg. 2) --------------------
    def sd_step(self, U, alpha=0.08):
        self._check(lib.gf_sd_step(self._h, ctypes.c_void_p(self._check_field(U)), float(alpha)))

    def sd_fix(self, U, alpha, eps, max_iter):
        it, F, th = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        rc = self._check(lib.gf_sd_fix(self._h, ctypes.c_void_p(self._check_field(U)), float(alpha),
                                       float(eps), int(max_iter), ctypes.byref(it), ctypes.byref(F),
                                       ctypes.byref(th)), allow=(OK, NOT_CONVERGED))
        return dict(converged=rc == OK, iters=it.value, F=F.value, theta=th.value)

    # -- schedule, timing -------------------------------------------------------
    def autotune(self, Us, omega, cache_path=None):
        if isinstance(Us, torch.Tensor):
            Us = [Us]
        cp = cache_path.encode() if cache_path else None
        self._check(lib.gf_autotune(self._h, self._ptr_array(Us), float(omega), cp))
        return self.schedule()

    def schedule(self):
        v = [ctypes.c_int() for _ in range(4)]
        self._check(lib.gf_get_schedule(self._h, *[ctypes.byref(x) for x in v]))
        return dict(lanes_per_site=v[0].value, block_threads=v[1].value, nontemporal=v[2].value,
                    tile_order=v[3].value)

    def timing(self):
        ms, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(lib.gf_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    @property
    def sweep_count(self):
        return int(lib.gf_get_sweep_count(self._h))

    @sweep_count.setter
    def sweep_count(self, v):
        self._check(lib.gf_set_sweep_count(self._h, int(v)))

    # -- differentiation ---------------------------------------------------------
    def empty_alg(self, device="cuda"):
        """An algebra field in the internal layout, shape (2, nb, 8, 64):
        [parity][block of 64 sites][component a][site in block]; the padding
        of the last block is zero (the kernels never write it)."""
        return torch.zeros((2, self.blocks(), 8, 64), dtype=self.rdtype, device=device)

    def _check_alg(self, s):
        n = 2 * self.blocks() * 8 * 64
        if s.dtype != self.rdtype or s.numel() != n:
            raise ValueError(f"algebra field must be {self.rdtype} with {n} elements (2 x nb x 8 x 64)")
        return _ptr(s)

    def pack_alg(self, s_aos):
        s = self.empty_alg(device=s_aos.device)
        if s_aos.dtype != self.rdtype or s_aos.numel() != 8 * self.volume():
            raise ValueError("canonical algebra field must be (nt, nz, ny, nx, 8) of the context dtype")
        self._check(lib.gf_pack_alg(self._h, ctypes.c_void_p(_ptr(s_aos)), ctypes.c_void_p(self._check_alg(s))))
        return s

    def unpack_alg(self, s):
        d = self.members[0][0]
        out = torch.empty((d[3], d[2], d[1], d[0], 8), dtype=self.rdtype, device=s.device)
        self._check(lib.gf_unpack_alg(self._h, ctypes.c_void_p(self._check_alg(s)), ctypes.c_void_p(_ptr(out))))
        return out

    def functional(self, U, s):
        F = ctypes.c_double()
        self._check(lib.gf_functional(self._h, ctypes.c_void_p(self._check_field(U)),
                                      ctypes.c_void_p(self._check_alg(s)), ctypes.byref(F)))
        return F.value

    def functional_grad(self, U, s, dF=1.0, out=None):
        if out is None:
            out = torch.zeros_like(s)
        self._check(lib.gf_functional_grad(self._h, ctypes.c_void_p(self._check_field(U)),
                                           ctypes.c_void_p(self._check_alg(s)), float(dF),
                                           ctypes.c_void_p(self._check_alg(out))))
        return out

    def gauge_transform(self, U, s):
        self._check(lib.gf_gauge_transform(self._h, ctypes.c_void_p(self._check_field(U)),
                                           ctypes.c_void_p(self._check_alg(s))))


class GaugeFunctional(torch.autograd.Function):
    """F_U[g] for g = exp(i s_a lambda_a / 2) with a hand-written backward
    kernel: forward -> gf_functional, backward -> gf_functional_grad."""

    @staticmethod
    def forward(actx, s, U, ctx: Context):
        actx.save_for_backward(s, U)
        actx.gf = ctx
        return torch.tensor(ctx.functional(U, s), dtype=torch.float64, device=s.device)

    @staticmethod
    def backward(actx, dF):
        s, U = actx.saved_tensors
        grad = actx.gf.functional_grad(U, s, float(dF))
        return grad, None, None


# -- host-only helpers (no device use) ------------------------------------------

def host_su2_step(b, omega):
    bb = (ctypes.c_double * 4)(*[float(x) for x in b])
    r = (ctypes.c_double * 4)()
    lib.gf_host_su2_step(bb, float(omega), r)
    return list(r)


def host_trig(x, y):
    out = (ctypes.c_double * 3)()
    lib.gf_host_trig(float(x), float(y), out)
    return tuple(out)


def host_link8(prec, U):
    """8-real round trip of one 3x3 complex matrix with the kernels' code:
    returns (the 8 stored reals, the reconstructed 3x3 complex matrix)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(U, dtype=np.complex128).reshape(9))
    inp = (ctypes.c_double * 18)(*[v for z in a for v in (z.real, z.imag)])
    st = (ctypes.c_double * 8)()
    out = (ctypes.c_double * 18)()
    rc = lib.gf_host_link8(int(prec), inp, st, out)
    if rc != OK:
        raise GFError(rc, "host_link8")
    o = np.array(out[:])
    return np.array(st[:]), (o[0::2] + 1j * o[1::2]).reshape(3, 3)


def site_links(dims, parity, h):
    out = (ctypes.c_longlong * 8)()
    rc = lib.gf_site_links(_dims_arr(dims), int(parity), int(h), out)
    if rc != OK:
        raise GFError(rc, "bad arguments")
    return list(out)
