"""ctypes binding of liblbmrv.so (the HIP library).  Argument marshalling only.

Every call goes to the C ABI declared in include/lbmrv.h; the arithmetic of the
scheme runs in the library's HIP kernels.  PyTorch supplies device memory and
the current stream.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbmrv.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NONFINITE, ERR_ALIGNMENT = 0, -1, -2, -4, -5, -6
LATTICES = {"d2q9": 0, "d3q19": 1, "d3q27": 2}
BASES = {"default": 0, "geier": 1}
STORAGES = {"f64": 0, "f32": 1, "f32dev": 2, "f16dev": 3}
MODES = {"zero": 0, "fluid": 1, "field": 2}
STREAMING = {"pull": 0, "push": 1, "aa": 2}
EQUILIBRIA = {"polynomial": 0, "maxwellian": 1}
BLOCK_ORDERS = {"auto": 0, "natural": 1, "xcd": 2}
QD = {"d2q9": (9, 2), "d3q19": (19, 3), "d3q27": (27, 3)}

_c_void_p = ctypes.c_void_p
_c_int = ctypes.c_int
_c_double = ctypes.c_double
_c_int64 = ctypes.c_int64

class PolyBasis(ctypes.Structure):
    """lbmrv_poly_basis: q polynomials in xi = X / lambda as a list of terms."""
    _fields_ = [("nterms", ctypes.c_int32), ("poly_of_term", ctypes.POINTER(ctypes.c_int32)),
                ("exps", ctypes.POINTER(ctypes.c_int32)), ("coef", ctypes.POINTER(_c_double))]


_SIGS = {
    "lbmrv_create": (_c_int, [ctypes.POINTER(_c_void_p), _c_int, _c_int, _c_double, ctypes.POINTER(_c_double),
                              ctypes.POINTER(_c_int64), _c_int, _c_double]),
    "lbmrv_create_custom": (_c_int, [ctypes.POINTER(_c_void_p), _c_int, ctypes.POINTER(PolyBasis), _c_double,
                                     ctypes.POINTER(_c_double), ctypes.POINTER(_c_int64), _c_int, _c_double]),
    "lbmrv_set_rates": (_c_int, [_c_void_p, ctypes.POINTER(_c_double)]),
    "lbmrv_set_streaming": (_c_int, [_c_void_p, _c_int]),
    "lbmrv_set_walls": (_c_int, [_c_void_p, ctypes.c_uint32, ctypes.POINTER(_c_double), _c_double]),
    "lbmrv_set_equilibrium": (_c_int, [_c_void_p, _c_int]),
    "lbmrv_set_block_order": (_c_int, [_c_void_p, _c_int]),
    "lbmrv_info": (_c_int, [_c_void_p] + [ctypes.POINTER(_c_int64)] * 4),
    "lbmrv_step": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int, _c_double, _c_void_p, _c_int64, _c_void_p]),
    "lbmrv_collide": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_int, _c_double, _c_void_p, _c_void_p]),
    "lbmrv_transport": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "lbmrv_moments": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "lbmrv_conservation": (_c_int, [_c_void_p, _c_void_p, ctypes.POINTER(_c_double), _c_void_p]),
    "lbmrv_conservation_noalloc": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "lbmrv_init_equilibrium": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_double, _c_void_p,
                                        _c_void_p]),
    "lbmrv_import": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "lbmrv_export": (_c_int, [_c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "lbmrv_lattice_tables": (_c_int, [_c_int, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_c_double)]),
    "lbmrv_adjoint_workspace_bytes": (ctypes.c_size_t, [_c_void_p, _c_int64, _c_int64]),
    "lbmrv_adjoint": (_c_int, [_c_void_p, _c_void_p, _c_int, _c_double, _c_void_p, _c_int64, _c_int64, _c_void_p,
                               _c_void_p, ctypes.c_size_t, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "lbmrv_deviation_norm": (_c_int, [_c_void_p, _c_void_p, ctypes.POINTER(_c_double), ctypes.POINTER(_c_double),
                                      _c_void_p]),
    "lbmrv_deviation_scale": (_c_int, [_c_void_p, _c_void_p, ctypes.POINTER(_c_double), _c_double, _c_void_p]),
    "lbmrv_destroy": (None, [_c_void_p]),
    "lbmrv_strerror": (ctypes.c_char_p, [_c_int]),
}

_lib = None


def library():
    """Load liblbmrv.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("liblbmrv.so not built: run python paper_1312_3297_amd/build.py first")
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LbmrvError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        msg = library().lbmrv_strerror(code).decode()
        super().__init__("%s failed: %s (%d)" % (what, msg, code))


def _check(code, what):
    if code != OK:
        raise LbmrvError(code, what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def lattice_tables(lattice):
    """Integer directions c [q, 3] and weights w [q] as the library defines them."""
    q, _ = QD[lattice]
    c = (ctypes.c_int32 * (3 * q))()
    w = (_c_double * q)()
    _check(library().lbmrv_lattice_tables(LATTICES[lattice], c, w), "lbmrv_lattice_tables")
    return np.array(c[:], dtype=np.int64).reshape(q, 3), np.array(w[:])


def poly_basis(polys):
    """Marshal q polynomials, each a list of (coef, (ex, ey, ez)) terms, into a
    PolyBasis; the ctypes arrays are kept alive on the returned object."""
    pot, exps, coef = [], [], []
    for k, terms in enumerate(polys):
        for c, e in terms:
            e = tuple(int(x) for x in e) + (0,) * (3 - len(e))
            pot.append(k)
            exps.extend(e)
            coef.append(float(c))
    n = len(pot)
    arrs = ((ctypes.c_int32 * max(n, 1))(*pot), (ctypes.c_int32 * max(3 * n, 1))(*exps),
            (_c_double * max(n, 1))(*coef))
    pb = PolyBasis(n, ctypes.cast(arrs[0], ctypes.POINTER(ctypes.c_int32)),
                   ctypes.cast(arrs[1], ctypes.POINTER(ctypes.c_int32)), ctypes.cast(arrs[2], ctypes.POINTER(_c_double)))
    pb._keep = arrs
    return pb


class Lbmrv:
    """One context: lattice, basis, lambda, rates, grid (nx, ny[, nz]) and storage.

    basis is "default", "geier" (D2Q9) or a run-time basis: a sequence of q
    polynomials in xi = X / lambda, each a list of (coef, (ex, ey, ez)) terms
    (see lbmrv_create_custom for the requirements)."""

    def __init__(self, lattice, s, dims, storage="f32", basis="default", lam=1.0, rho0=1.0):
        self.lattice, self.basis, self.storage = lattice, basis, storage
        self.q, self.d = QD[lattice]
        self.dims = tuple(int(x) for x in dims)
        if len(self.dims) != self.d:
            raise ValueError("dims must have %d entries" % self.d)
        self.lam = float(lam)
        self.rho0 = float(rho0)
        rates = (_c_double * self.q)(*[float(x) for x in s])
        dd = (_c_int64 * 3)(*(list(self.dims) + [1] * (3 - self.d)))
        h = _c_void_p()
        if isinstance(basis, str):
            _check(library().lbmrv_create(ctypes.byref(h), LATTICES[lattice], BASES[basis], self.lam, rates, dd,
                                          STORAGES[storage], self.rho0), "lbmrv_create")
        else:
            pb = poly_basis(basis)
            _check(library().lbmrv_create_custom(ctypes.byref(h), LATTICES[lattice], ctypes.byref(pb), self.lam,
                                                 rates, dd, STORAGES[storage], self.rho0), "lbmrv_create_custom")
        self._h = h
        self.N = int(np.prod(self.dims))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().lbmrv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes and dtypes
    @property
    def grid_shape(self):
        """Array shape of one population field: (ny, nx) or (nz, ny, nx)."""
        return tuple(reversed(self.dims))

    @property
    def torch_dtype(self):
        import torch
        return {"f64": torch.float64, "f32": torch.float32, "f32dev": torch.float32,
                "f16dev": torch.float16}[self.storage]

    @property
    def out_dtype(self):
        import torch
        return torch.float64 if self.storage == "f64" else torch.float32

    def empty(self, device="cuda"):
        import torch
        return torch.empty((self.q,) + self.grid_shape, dtype=self.torch_dtype, device=device)

    # calls
    def set_rates(self, s):
        rates = (_c_double * self.q)(*[float(x) for x in s])
        _check(library().lbmrv_set_rates(self._h, rates), "lbmrv_set_rates")

    def set_streaming(self, kind):
        _check(library().lbmrv_set_streaming(self._h, STREAMING[kind]), "lbmrv_set_streaming")

    def set_block_order(self, order):
        _check(library().lbmrv_set_block_order(self._h, BLOCK_ORDERS[order]), "lbmrv_set_block_order")

    def set_equilibrium(self, kind):
        _check(library().lbmrv_set_equilibrium(self._h, EQUILIBRIA[kind]), "lbmrv_set_equilibrium")

    def set_walls(self, mask, wall_u=None, rho_w=1.0):
        """Half-way bounce-back faces: bit 2a+side of mask; wall_u [6][3] or None."""
        wu = None
        if wall_u is not None:
            flat = [float(v) for row in wall_u for v in row]
            wu = (_c_double * 18)(*flat)
        _check(library().lbmrv_set_walls(self._h, int(mask), wu, float(rho_w)), "lbmrv_set_walls")

    def step(self, f_in, f_out, mode="zero", alpha=1.0, field=None, nsteps=1, stream=None):
        _check(library().lbmrv_step(self._h, _ptr(f_in), _ptr(f_out), MODES[mode], float(alpha), _ptr(field),
                                    int(nsteps), _stream(stream)), "lbmrv_step")

    def collide(self, f_in, f_out, mode="zero", alpha=1.0, field=None, stream=None):
        _check(library().lbmrv_collide(self._h, _ptr(f_in), _ptr(f_out), MODES[mode], float(alpha), _ptr(field),
                                       _stream(stream)), "lbmrv_collide")

    def transport(self, f_in, f_out, stream=None):
        _check(library().lbmrv_transport(self._h, _ptr(f_in), _ptr(f_out), _stream(stream)), "lbmrv_transport")

    def moments(self, f, with_m0=False, stream=None):
        import torch
        rho = torch.empty(self.grid_shape, dtype=self.out_dtype, device=f.device)
        u = torch.empty((self.d,) + self.grid_shape, dtype=self.out_dtype, device=f.device)
        m0 = torch.empty((self.q,) + self.grid_shape, dtype=self.out_dtype, device=f.device) if with_m0 else None
        _check(library().lbmrv_moments(self._h, _ptr(f), _ptr(rho), _ptr(u), _ptr(m0), _stream(stream)),
               "lbmrv_moments")
        return rho, u, m0

    def conservation(self, f, stream=None):
        """(mass, momentum[d]) in FP64 and whether every population is finite."""
        out = (_c_double * 4)()
        rc = library().lbmrv_conservation(self._h, _ptr(f), out, _stream(stream))
        if rc not in (OK, ERR_NONFINITE):
            _check(rc, "lbmrv_conservation")
        return out[0], list(out[1:1 + self.d]), rc == OK

    def conservation_noalloc(self, f, out, stream=None):
        """The same sums into the device tensor `out` (5 doubles: mass,
        momentum[3], count of non-finite values), asynchronously and without
        any allocation (lbmrv_conservation_noalloc)."""
        _check(library().lbmrv_conservation_noalloc(self._h, _ptr(f), _ptr(out), _stream(stream)),
               "lbmrv_conservation_noalloc")
        return out

    def init_equilibrium(self, rho, u, noise=None, amp=0.0, out=None, stream=None):
        out = self.empty(rho.device) if out is None else out
        _check(library().lbmrv_init_equilibrium(self._h, _ptr(rho), _ptr(u), _ptr(noise), float(amp), _ptr(out),
                                                _stream(stream)), "lbmrv_init_equilibrium")
        return out

    @property
    def compute_dtype(self):
        import torch
        return torch.float64 if self.storage == "f64" else torch.float32

    def adjoint_workspace_bytes(self, nsteps, K):
        return int(library().lbmrv_adjoint_workspace_bytes(self._h, int(nsteps), int(K)))

    def adjoint(self, f0, cot_fN, nsteps, K=100, mode="zero", field=None, want_fN=False, workspace=None,
                stream=None, alpha=1.0):
        """Discrete adjoint of nsteps steps: (f_N or None, dJ/df0, dJ/ds [FP64], dJ/du~ [FP64] or None)."""
        import torch
        dev = f0.device
        nbytes = self.adjoint_workspace_bytes(nsteps, K)
        if workspace is None or workspace.numel() < nbytes:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        grad_f0 = torch.empty((self.q,) + self.grid_shape, dtype=self.compute_dtype, device=dev)
        grad_s = torch.empty(self.q, dtype=torch.float64, device=dev)
        grad_ut = torch.empty((self.d,) + self.grid_shape, dtype=torch.float64, device=dev) \
            if mode == "field" else None
        fN = self.empty(dev) if want_fN else None
        _check(library().lbmrv_adjoint(self._h, _ptr(f0), MODES[mode], float(alpha), _ptr(field), int(nsteps), int(K),
                                       _ptr(cot_fN), _ptr(workspace), nbytes, _ptr(fN), _ptr(grad_f0),
                                       _ptr(grad_s), _ptr(grad_ut), _stream(stream)), "lbmrv_adjoint")
        return fN, grad_f0, grad_s, grad_ut

    def deviation_norm2(self, f, f_ref, stream=None):
        """sum over nodes and j of (f_j - f_ref_j)^2 (FP64) and whether f is finite."""
        ref = (_c_double * self.q)(*[float(x) for x in f_ref])
        out = (_c_double * 1)()
        rc = library().lbmrv_deviation_norm(self._h, _ptr(f), ref, out, _stream(stream))
        if rc not in (OK, ERR_NONFINITE):
            _check(rc, "lbmrv_deviation_norm")
        return out[0], rc == OK

    def deviation_scale(self, f, f_ref, factor, stream=None):
        ref = (_c_double * self.q)(*[float(x) for x in f_ref])
        _check(library().lbmrv_deviation_scale(self._h, _ptr(f), ref, float(factor), _stream(stream)),
               "lbmrv_deviation_scale")

    def import_f64(self, f, out=None, stream=None):
        out = self.empty(f.device) if out is None else out
        _check(library().lbmrv_import(self._h, _ptr(f), _ptr(out), _stream(stream)), "lbmrv_import")
        return out

    def export_f64(self, f, out=None, stream=None):
        import torch
        out = torch.empty((self.q,) + self.grid_shape, dtype=torch.float64, device=f.device) if out is None else out
        _check(library().lbmrv_export(self._h, _ptr(f), _ptr(out), _stream(stream)), "lbmrv_export")
        return out


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
def _steps_function():
    import torch

    class Steps(torch.autograd.Function):
        """f_N = N steps of the scheme from f0 with rates s and relative velocity
        u~ = field (if given), alpha * u (if alpha is given) or 0.  backward()
        runs the library's discrete adjoint (lbmrv_adjoint) and returns dJ/df0,
        dJ/ds (FP64) and dJ/du~ (field case)."""

        @staticmethod
        def forward(ctx, f0, s, field, lb, nsteps, K, alpha):
            lb.set_rates([float(x) for x in s.detach().cpu()])
            mode = "field" if field is not None else ("fluid" if alpha is not None else "zero")
            fin = f0.detach().clone()
            fout = torch.empty_like(fin)
            fld = None if field is None else field.detach().contiguous()
            a = 1.0 if alpha is None else float(alpha)
            lb.step(fin, fout, mode, a, fld, nsteps)
            ctx.save_for_backward(f0, s, field if field is not None else torch.empty(0))
            ctx.lb, ctx.nsteps, ctx.K, ctx.mode, ctx.alpha = lb, nsteps, K, mode, a
            return fout

        @staticmethod
        def backward(ctx, grad_fN):
            f0, s, field = ctx.saved_tensors
            lb = ctx.lb
            lb.set_rates([float(x) for x in s.detach().cpu()])
            cot = grad_fN.detach().to(lb.compute_dtype).contiguous()
            fld = field.detach().contiguous() if ctx.mode == "field" else None
            _, gf, gs, gu = lb.adjoint(f0.detach().contiguous(), cot, ctx.nsteps, ctx.K, ctx.mode, fld,
                                       alpha=ctx.alpha)
            g_field = gu.to(field.dtype) if ctx.mode == "field" else None
            return gf.to(f0.dtype), gs.to(device=s.device, dtype=s.dtype), g_field, None, None, None, None

    return Steps


_STEPS = None


def steps(f0, s, field, lb, nsteps, K=100, alpha=None):
    """Differentiable N-step map (see Steps)."""
    global _STEPS
    if _STEPS is None:
        _STEPS = _steps_function()
    return _STEPS.apply(f0, s, field, lb, nsteps, K, alpha)


def kinetic_energy(lb, f):
    """J = 1/2 sum_x |q|^2 / rho of a population tensor in the context's storage
    (torch ops, differentiable): the objective of the adjoint workload."""
    import torch
    c, w = lattice_tables(lb.lattice)
    ff = f.to(torch.float64)
    if lb.storage in ("f32dev", "f16dev"):
        ff = ff + torch.tensor(w * lb.rho0, dtype=torch.float64, device=f.device).reshape((-1,) + (1,) * lb.d)
    rho = ff.sum(0)
    v = torch.tensor(lb.lam * c[:, : lb.d], dtype=torch.float64, device=f.device)
    qm = torch.einsum("ja,j...->a...", v, ff)
    return 0.5 * ((qm * qm).sum(0) / rho).sum()
