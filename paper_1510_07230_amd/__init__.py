"""Python binding of libpou.so, the MI355X library for the parallel
orbital-updating optimisation of Kohn-Sham DFT (arXiv 1510.07230).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in include/pou.h.  PyTorch supplies device memory
and the stream.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpou.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pou.h")

POU_OK = 0
STATUS = {0: "POU_OK", -1: "POU_ERR_ARG", -2: "POU_ERR_STATE", -3: "POU_ERR_HIP",
          -4: "POU_ERR_OOM", -5: "POU_ERR_NOT_SPD", -6: "POU_ERR_CG_NO_CONV",
          -7: "POU_ERR_NONFINITE"}
FP64, MIXED = 0, 1
TERM_KIN, TERM_EXT, TERM_HARTREE, TERM_XC, TERM_ALL = 1, 2, 4, 8, 15
TERM_CORR = 16  # LDA correlation, opt in
TERM_NLOC = 32  # nonlocal projectors, switched on by set_projectors
GRAM_ACCURATE, GRAM_BF16 = 0, 1


class PouError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("L", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [("rho1", ctypes.c_double), ("delta", ctypes.c_double), ("eta", ctypes.c_double),
                ("bb_mode", ctypes.c_int), ("tau_init", ctypes.c_double), ("s_max", ctypes.c_int),
                ("orth_passes", ctypes.c_int), ("cg_rtol", ctypes.c_double),
                ("cg_maxit", ctypes.c_int), ("cg_precond", ctypes.c_int),
                ("terms", ctypes.c_uint), ("n_org", ctypes.c_int), ("n_diag", ctypes.c_int)]


class EnergyTerms(ctypes.Structure):
    _fields_ = [("E", ctypes.c_double), ("E_kin", ctypes.c_double), ("E_ext", ctypes.c_double),
                ("E_H", ctypes.c_double), ("E_x", ctypes.c_double), ("cg_iters", ctypes.c_int),
                ("E_c", ctypes.c_double), ("E_nl", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("l", ctypes.c_int), ("s", ctypes.c_int), ("accepted", ctypes.c_int),
                ("cg_iters", ctypes.c_int), ("E", ctypes.c_double), ("tau_bb", ctypes.c_double),
                ("tau", ctypes.c_double), ("zz", ctypes.c_double), ("df", ctypes.c_double),
                ("C", ctypes.c_double), ("Q", ctypes.c_double), ("gram_dev", ctypes.c_double),
                ("orthonormalized", ctypes.c_int), ("rotated", ctypes.c_int)]


_LIB = None
_vp, _dp, _i, _d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double

_SIGNATURES = {
    "pou_default_params": (None, [ctypes.POINTER(Params)]),
    "pou_create": (_i, [ctypes.POINTER(_vp), _i, _vp]),
    "pou_destroy": (_i, [_vp]),
    "pou_last_error": (ctypes.c_char_p, [_vp]),
    "pou_set_system": (_i, [_vp, ctypes.POINTER(Grid), _i, _dp, _dp, _dp, _i, _dp, _i,
                            ctypes.POINTER(Params)]),
    "pou_energy": (_i, [_vp, _vp, ctypes.POINTER(EnergyTerms)]),
    "pou_set_projectors": (_i, [_vp, _dp]),
    "pou_residual": (_i, [_vp, _vp, _dp, _dp]),
    "pou_orthonormalize": (_i, [_vp, _vp, _dp]),
    "pou_orbital_update_step": (_i, [_vp, _vp, ctypes.POINTER(StepInfo)]),
    "pou_energy_backward": (_i, [_vp, _vp, _d, _vp, _vp, _vp]),
    "pou_hamiltonian_apply": (_i, [_vp, _vp, _vp, _dp]),
    "pou_get_fields": (_i, [_vp, _vp, _vp, _vp, _vp]),
    "pou_gram": (_i, [_vp, _vp, _i, _dp]),
    "pou_trial_point": (_i, [_vp, _vp, _d, _vp, _dp]),
    "pou_gram_static": (_i, [_vp, _i, _i, _i, ctypes.c_longlong, _d, _vp, _vp]),
    "pou_convert": (_i, [_vp, _vp, _i, _vp, _i, ctypes.c_longlong]),
    "pou_reset_history": (_i, [_vp]),
    "pou_profile_enable": (_i, [_vp, ctypes.c_uint]),
    "pou_profile_read": (_i, [_vp, _i, _dp, ctypes.POINTER(ctypes.c_longlong)]),
}

KERNEL_GROUPS = ["hamiltonian", "density", "xc", "poisson", "gram", "cholesky", "apply",
                 "trial", "commit", "other", "apply_gram"]


def header_symbols(path=HEADER):
    """Names of the functions declared in include/pou.h."""
    txt = open(path).read()
    return sorted(set(re.findall(r"\b(pou_[a-z_]+)\s*\(", txt)))


def lib():
    """Load libpou.so (built by paper_1510_07230_amd.build); raise if missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1510_07230_amd.build")
        # Load torch's HIP runtime first: libpou then binds to that same copy
        # (matching soname) instead of pulling in a second runtime.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def default_params(**overrides) -> Params:
    p = Params()
    lib().pou_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _dptr(a):
    return a.ctypes.data_as(_dp)


class System:
    """One context: grid, ions, occupations, precision and parameters.

    Orbital blocks are torch tensors on the context's device, shape
    [N, n, n, n], float64 (precision "fp64") or float32 ("mixed").
    """

    def __init__(self, n, L, R, Z, sigma, occ, precision="fp64", params=None, device=0,
                 stream=None, proj=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.n, self.L = int(n), float(L)
        self.N = len(occ)
        self.M = len(Z)
        self.prec = FP64 if precision in ("fp64", FP64) else MIXED
        self.dtype = torch.float64 if self.prec == FP64 else torch.float32
        self.params = params if params is not None else default_params()
        self._stream = stream
        h = ctypes.c_void_p()
        st = self._stream_handle()
        rc = lib().pou_create(ctypes.byref(h), int(device), st)
        if rc != POU_OK:
            raise PouError(rc, "pou_create failed")
        self._h = h
        self.proj = None if proj is None else np.ascontiguousarray(np.asarray(proj, np.float64))
        self.set_system(R, Z, sigma, occ)

    def _stream_handle(self):
        torch = self.torch
        s = self._stream if self._stream is not None else torch.cuda.current_stream(self.device)
        return ctypes.c_void_p(s.cuda_stream)

    def _check(self, rc):
        if rc != POU_OK:
            msg = lib().pou_last_error(self._h)
            raise PouError(rc, msg.decode() if msg else "")

    def set_system(self, R, Z, sigma, occ):
        R = np.ascontiguousarray(np.asarray(R, dtype=np.float64).reshape(-1, 3))
        Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64))
        sigma = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
        occ = np.ascontiguousarray(np.asarray(occ, dtype=np.float64))
        self.R, self.Z, self.sigma, self.occ = R, Z, sigma, occ
        self.M = len(Z)
        self.N = len(occ)
        g = Grid(self.n, self.L)
        self._check(lib().pou_set_system(self._h, ctypes.byref(g), self.M, _dptr(R), _dptr(Z),
                                         _dptr(sigma), self.N, _dptr(occ), self.prec,
                                         ctypes.byref(self.params)))
        if getattr(self, "proj", None) is not None:
            self.set_projectors(self.proj)

    def set_projectors(self, proj):
        """Nonlocal projectors (section 2.1): proj [M, 3] = (rc, b_s, b_p) per
        ion, or None to remove them.  Kept across set_system calls."""
        self.proj = None if proj is None else np.ascontiguousarray(np.asarray(proj, np.float64))
        if self.proj is not None and self.proj.shape != (self.M, 3):
            raise ValueError("proj must be [natoms, 3]")
        ptr = _dptr(self.proj) if self.proj is not None else None
        self._check(lib().pou_set_projectors(self._h, ptr))

    def close(self):
        if getattr(self, "_h", None):
            lib().pou_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_block(self, data=None):
        """Device block [N, n, n, n] of this system's dtype (copy of `data` if given)."""
        torch = self.torch
        shape = (self.N, self.n, self.n, self.n)
        if data is None:
            return torch.zeros(shape, dtype=self.dtype, device=self.device)
        t = torch.as_tensor(np.asarray(data)).to(self.device, self.dtype)
        if tuple(t.shape) != shape:
            t = t.reshape(shape)
        return t.contiguous()

    def _block(self, U):
        if U.device != self.device or U.dtype != self.dtype or not U.is_contiguous():
            raise ValueError(f"block must be contiguous {self.dtype} on {self.device}")
        if U.numel() != self.N * self.n ** 3:
            raise ValueError("block has the wrong number of elements")
        return ctypes.c_void_p(U.data_ptr())

    def energy(self, U):
        t = EnergyTerms()
        self._check(lib().pou_energy(self._h, self._block(U), ctypes.byref(t)))
        return {"E": t.E, "E_kin": t.E_kin, "E_ext": t.E_ext, "E_H": t.E_H, "E_x": t.E_x,
                "E_c": t.E_c, "E_nl": t.E_nl, "cg_iters": t.cg_iters}

    @staticmethod
    def _written(t):
        """Tell autograd that the library wrote t in place (ctypes bypasses
        torch's version counter), so a graph that saved t refuses to use it."""
        from torch.autograd.graph import increment_version
        increment_version(t)

    def orthonormalize_(self, U):
        err = ctypes.c_double(0.0)
        try:
            self._check(lib().pou_orthonormalize(self._h, self._block(U), ctypes.byref(err)))
        finally:
            self._written(U)
        return err.value

    def step_(self, U):
        info = StepInfo()
        try:
            self._check(lib().pou_orbital_update_step(self._h, self._block(U),
                                                      ctypes.byref(info)))
        finally:
            self._written(U)
        return {k: getattr(info, k) for k, _ in StepInfo._fields_}

    def residual(self, U):
        """(||H U - U Sigma||, Sigma) with Sigma = <(H U)^T U> (eq. "gra")."""
        r = ctypes.c_double(0.0)
        S = np.zeros((self.N, self.N))
        self._check(lib().pou_residual(self._h, self._block(U), ctypes.byref(r), _dptr(S)))
        return r.value, S

    def hamiltonian(self, U):
        HU = self.torch.empty_like(U)
        sig = np.zeros(self.N)
        self._check(lib().pou_hamiltonian_apply(self._h, self._block(U), self._block(HU),
                                                _dptr(sig)))
        return HU, sig

    def fields(self):
        torch = self.torch
        out = {k: torch.empty((self.n,) * 3, dtype=torch.float64, device=self.device)
               for k in ("rho", "vh", "veff", "vext")}
        self._check(lib().pou_get_fields(self._h, *[ctypes.c_void_p(out[k].data_ptr())
                                                    for k in ("rho", "vh", "veff", "vext")]))
        return out

    def gram(self, U, bf16=False):
        """<U^T U> (FP64 host array); bf16=True: the mixed form's first-pass
        BF16 Gram (FP32 blocks only)."""
        G = np.zeros((self.N, self.N))
        mode = GRAM_BF16 if bf16 else GRAM_ACCURATE
        self._check(lib().pou_gram(self._h, self._block(U), mode, _dptr(G)))
        return G

    def trial_point(self, U, tau):
        """(W~ = U - tau Z as a device block, its Gram as the step's first pass
        forms it) for Z = H(rho(U)) U - U diag(sigma)."""
        Wt = self.torch.empty_like(U)
        G = np.zeros((self.N, self.N))
        self._check(lib().pou_trial_point(self._h, self._block(U), float(tau),
                                          ctypes.c_void_p(Wt.data_ptr()), _dptr(G)))
        return Wt, G

    def backward(self, U, gE=1.0, want_dU=True, want_forces=True):
        torch = self.torch
        dU = torch.empty_like(U) if want_dU else None
        dR = torch.empty((self.M, 3), dtype=torch.float64, device=self.device) if want_forces else None
        ds = torch.empty((self.M,), dtype=torch.float64, device=self.device) if want_forces else None
        p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
        self._check(lib().pou_energy_backward(self._h, self._block(U), float(gE), p(dU), p(dR),
                                              p(ds)))
        return dU, dR, ds

    def convert(self, src, dst):
        pr = lambda t: FP64 if t.dtype == self.torch.float64 else MIXED
        if src.numel() != dst.numel():
            raise ValueError("size mismatch")
        try:
            self._check(lib().pou_convert(self._h, ctypes.c_void_p(src.data_ptr()), pr(src),
                                          ctypes.c_void_p(dst.data_ptr()), pr(dst), src.numel()))
        finally:
            self._written(dst)
        return dst

    def reset_history(self):
        self._check(lib().pou_reset_history(self._h))

    def profile(self, enable=True, groups=None):
        """Turn per-kernel-group HIP event timing on/off (on clears the totals).

        groups: names from KERNEL_GROUPS to time (default: all of them).  Each
        timed launch adds event records to the stream, so time only the groups
        being measured when the step time matters."""
        mask = 0
        if enable:
            names = KERNEL_GROUPS if groups is None else groups
            for name in names:
                mask |= 1 << KERNEL_GROUPS.index(name)
        self._check(lib().pou_profile_enable(self._h, mask))

    def profile_read(self):
        """{group: (total_ms, launches)} since profiling was enabled."""
        out = {}
        for k, name in enumerate(KERNEL_GROUPS):
            ms = ctypes.c_double(0.0)
            n = ctypes.c_longlong(0)
            self._check(lib().pou_profile_read(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out


def gram_static(U, dv, bf16=False, out=None, stream=None):
    """pou_gram_static: dv * U U^T of a device block U ([N, ...], float64 or
    float32, N <= 128) into a device [N, N] float64 tensor, with no context
    and no allocation inside the library (out is allocated here if None)."""
    import torch
    if not U.is_cuda or not U.is_contiguous() or U.dtype not in (torch.float64, torch.float32):
        raise ValueError("U must be a contiguous float64/float32 device tensor")
    N = U.shape[0]
    ng = U.numel() // N
    if out is None:
        out = torch.empty((N, N), dtype=torch.float64, device=U.device)
    s = stream if stream is not None else torch.cuda.current_stream(U.device)
    prec = FP64 if U.dtype == torch.float64 else MIXED
    rc = lib().pou_gram_static(ctypes.c_void_p(U.data_ptr()), prec,
                               GRAM_BF16 if bf16 else GRAM_ACCURATE, N, ng, float(dv),
                               ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream))
    if rc != POU_OK:
        raise PouError(rc, "pou_gram_static failed")
    return out


def _energy_fn():
    import torch

    class EnergyFn(torch.autograd.Function):
        """E(U; R, sigma) with gradients dE/dU = 2 f_i h^3 H u_i and the forces
        dE/dR, dE/dsigma from pou_energy_backward."""

        @staticmethod
        def forward(ctx, U, R, sigma, system):
            Rn = np.array(R.detach().cpu().numpy(), dtype=np.float64).reshape(-1, 3)
            sn = np.array(sigma.detach().cpu().numpy(), dtype=np.float64)
            if not (np.array_equal(Rn, system.R) and np.array_equal(sn, system.sigma)):
                system.set_system(Rn, system.Z, sn, system.occ)
            e = system.energy(U.detach())
            ctx.system = system
            # the ions of this evaluation: another forward may move the shared
            # context's ions before this graph's backward runs
            ctx.R, ctx.sigma = Rn, sn
            ctx.rdev = (R.device, R.dtype, sigma.device, sigma.dtype)
            ctx.save_for_backward(U)
            return torch.tensor(e["E"], dtype=torch.float64, device=U.device)

        @staticmethod
        def backward(ctx, g):
            (U,) = ctx.saved_tensors
            system = ctx.system
            if not (np.array_equal(ctx.R, system.R) and np.array_equal(ctx.sigma, system.sigma)):
                system.set_system(ctx.R, system.Z, ctx.sigma, system.occ)
            # evaluate U afresh at these ions: the context's cached evaluation may
            # belong to another block or to other ions
            system.energy(U.detach())
            dU, dR, ds = system.backward(U.detach(), float(g.item()),
                                         want_dU=ctx.needs_input_grad[0],
                                         want_forces=(ctx.needs_input_grad[1]
                                                      or ctx.needs_input_grad[2]))
            if dR is not None:
                dR = dR.to(ctx.rdev[0], ctx.rdev[1])
                ds = ds.to(ctx.rdev[2], ctx.rdev[3])
            return dU, dR, ds, None

    return EnergyFn


def __getattr__(name):
    if name == "EnergyFn":
        return _energy_fn()
    raise AttributeError(name)
