"""Thin Python binding of ``libmgcccs.so`` (C ABI in ``include/mgcccs.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (fields, workspace) and the HIP stream.  The
library must be built (``__graft_entry__.build()``); importing this module
without it raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgcccs.so")

MGC_OK, MGC_EINVAL, MGC_ENOMEM, MGC_EHIP, MGC_ENOCONV, MGC_ESTATE, MGC_ENUMERIC = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "MGC_OK", -1: "MGC_EINVAL", -2: "MGC_ENOMEM", -3: "MGC_EHIP", -4: "MGC_ENOCONV",
                -5: "MGC_ESTATE", -6: "MGC_ENUMERIC"}
FP64, FP32 = 0, 1
SWEEP_MAX = 256                      # MGC_SWEEP_MAX
STATIONARY, IR, FGMRES, BICGSTAB = 0, 1, 2, 3
SMOOTH_JACOBI, SMOOTH_GMRES3 = 0, 1
PC_MG_CCCS, PC_DEFLATION = 0, 1

EXPORTED = ["mgc_create_grid", "mgc_workspace_bytes", "mgc_bind_workspace", "mgc_field_pitch",
            "mgc_set_potential", "mgc_set_energy", "mgc_build_rhs_tp", "mgc_residual", "mgc_vcycle",
            "mgc_cccs", "mgc_solve", "mgc_solve_transpose", "mgc_cross_section",
            "mgc_cross_section_sweep", "mgc_cross_section_grad", "mgc_set_kernel_timer", "mgc_read_kernel_timer",
            "mgc_batch_create", "mgc_batch_solve", "mgc_batch_destroy",
            "mgc_set_schedule", "mgc_get_schedule", "mgc_cccs_noalloc", "mgc_single_ionization",
            "mgc_total_double_ionization", "mgc_batch_cross_sections", "mgc_set_potential_exp",
            "mgc_channel_energies", "mgc_destroy_grid", "mgc_last_error"]

# kernel classes of mgc_set_kernel_timer
(KT_NONE, KT_APPLY_DOT, KT_AXPY, KT_S1, KT_S2, KT_CCCS_PROJECT, KT_CCCS_CHAIN, KT_S1_FINE, KT_S2_FINE,
 KT_CCCS_EXPAND) = range(10)


class GridDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("L", ctypes.c_double), ("R0", ctypes.c_double),
                ("theta", ctypes.c_double), ("levels", ctypes.c_int), ("M", ctypes.c_int),
                ("Lch", ctypes.c_int), ("omega", ctypes.c_double), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("pc_gamma", ctypes.c_double), ("pc_first_level", ctypes.c_int),
                ("max_restart", ctypes.c_int), ("precisions", ctypes.c_int), ("pc_gamma0", ctypes.c_double),
                ("gamma", ctypes.c_double), ("smoother", ctypes.c_int), ("pc_order", ctypes.c_int),
                ("pot_tables", ctypes.c_int), ("gs_from", ctypes.c_int)]


class Schedule(ctypes.Structure):
    """Launch schedule of the zero-guess cycle (mgc_schedule)."""
    _fields_ = [("small_tiles", ctypes.c_int), ("level_pairs", ctypes.c_int), ("coarse_tail", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int), ("inner", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_it", ctypes.c_int), ("inner_cycles", ctypes.c_int), ("tol", ctypes.c_double)]


class KernelTiming(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("launches", ctypes.c_longlong),
                ("bytes", ctypes.c_double), ("floor_ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("vcycles", ctypes.c_int), ("relres", ctypes.c_double),
                ("hist", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int),
                ("hist_len", ctypes.c_int), ("t_setup_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "mgc_create_grid": [ctypes.POINTER(GridDesc), vp, ctypes.POINTER(vp)],
        "mgc_workspace_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "mgc_bind_workspace": [vp, vp, ctypes.c_size_t],
        "mgc_field_pitch": [vp, i, ctypes.POINTER(i)],
        "mgc_set_potential": [vp, d, d, d],
        "mgc_set_potential_exp": [vp, d, d, d, d, d, d],
        "mgc_channel_energies": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
        "mgc_set_energy": [vp, d],
        "mgc_build_rhs_tp": [vp, vp, i],
        "mgc_residual": [vp, vp, vp, vp, ctypes.POINTER(d), i],
        "mgc_vcycle": [vp, vp, vp, i],
        "mgc_cccs": [vp, vp, vp, i],
        "mgc_cccs_noalloc": [vp, vp, vp, i],
        "mgc_solve": [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(Stats)],
        "mgc_solve_transpose": [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(Stats)],
        "mgc_cross_section": [vp, vp, vp, d, d, ctypes.POINTER(d), ctypes.POINTER(d)],
        "mgc_cross_section_sweep": [vp, vp, vp, i, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d),
                                    ctypes.POINTER(d)],
        "mgc_cross_section_grad": [vp, vp, vp, d, d, ctypes.POINTER(SolveOpts), vp,
                                   ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d),
                                   ctypes.POINTER(Stats)],
        "mgc_set_kernel_timer": [vp, i],
        "mgc_read_kernel_timer": [vp, ctypes.POINTER(KernelTiming)],
        "mgc_batch_create": [ctypes.POINTER(vp), i, ctypes.POINTER(vp)],
        "mgc_batch_solve": [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(SolveOpts),
                            ctypes.POINTER(Stats)],
        "mgc_batch_destroy": [vp],
        "mgc_single_ionization": [vp, vp, vp, i, ctypes.POINTER(d), ctypes.POINTER(d)],
        "mgc_total_double_ionization": [vp, vp, vp, i, ctypes.POINTER(d), ctypes.POINTER(d)],
        "mgc_batch_cross_sections": [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i, i, ctypes.POINTER(d),
                                     ctypes.POINTER(d)],
        "mgc_set_schedule": [vp, ctypes.POINTER(Schedule)],
        "mgc_get_schedule": [vp, ctypes.POINTER(Schedule)],
        "mgc_destroy_grid": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.mgc_last_error.argtypes = []
    lib.mgc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


class MGCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(rc: int, allow=()):
    if rc != MGC_OK and rc not in allow:
        raise MGCError(rc, load_library().mgc_last_error().decode())
    return rc


@dataclasses.dataclass
class SolveResult:
    status: int
    iters: int
    vcycles: int
    relres: float
    history: list
    t_setup_ms: float
    t_solve_ms: float


class Grid:
    """One MG-CCCS handle with a torch-allocated workspace on a CUDA device."""

    def __init__(self, n, L, R0, theta, levels, M, Lch=None, omega=2.0 / 3.0, nu1=1, nu2=1,
                 pc_gamma=0.0, pc_first_level=0, max_restart=16, fp32=True, device="cuda:0",
                 pc_gamma0=0.0, gamma=0.0, smoother=0, pc_order=0, pot_tables=0, gs_from=0):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        Lch = M if Lch is None else Lch
        self.desc = GridDesc(n, L, R0, theta, levels, M, Lch, omega, nu1, nu2, pc_gamma,
                             pc_first_level, max_restart, 1 | (2 if fp32 else 0), pc_gamma0, gamma, smoother,
                             pc_order, pot_tables, gs_from)
        self.n, self.levels, self.M, self.Lch = n, levels, M, Lch
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            _check(self.lib.mgc_create_grid(ctypes.byref(self.desc), ctypes.c_void_p(self.stream.cuda_stream),
                                            ctypes.byref(h)))
            self.h = h
            nb = ctypes.c_size_t()
            _check(self.lib.mgc_workspace_bytes(self.h, ctypes.byref(nb)))
            self.workspace_bytes = nb.value
            self._ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            off = (-base) % 256
            _check(self.lib.mgc_bind_workspace(self.h, ctypes.c_void_p(base + off), nb.value))
        p = ctypes.c_int()
        _check(self.lib.mgc_field_pitch(self.h, 0, ctypes.byref(p)))
        self.pitch = p.value

    @classmethod
    def from_workload(cls, w, **kw):
        kw.setdefault("pc_gamma", w.pc_gamma)
        kw.setdefault("pc_first_level", w.pc_first_level)
        kw.setdefault("pc_gamma0", w.pc_gamma0)
        return cls(w.n, w.L, w.R0, w.theta, w.levels, w.M, omega=w.omega, nu1=w.nu1, nu2=w.nu2, **kw)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.mgc_destroy_grid(h)
            self.h = None

    # ---- fields --------------------------------------------------------------
    def field(self, fp32: bool = False):
        """Zero level-0 field: an (n+1) x (n+1) view of an (n+1) x pitch buffer."""
        t = self.torch
        buf = t.zeros((self.n + 1, self.pitch), dtype=t.complex64 if fp32 else t.complex128,
                      device=self.device)
        return buf[:, : self.n + 1]

    def from_numpy(self, a, fp32: bool = False):
        out = self.field(fp32)
        out.copy_(self.torch.from_numpy(a).to(out.dtype))
        return out

    def _ptr(self, x, prec=FP64):
        """Device pointer of a level-0 field after checking that the kernels'
        indexing (element (k, j) at k * pitch + j, k, j <= n) stays inside it:
        a tensor on this handle's device, complex128 (FP64) or complex64
        (FP32), shape (n+1, n+1), strides (pitch, 1) and storage for
        (n+1) * pitch elements from its first element.  MGCError(MGC_EINVAL)
        otherwise; nothing reaches the library."""
        t = self.torch
        want = t.complex128 if prec == FP64 else t.complex64
        bad = None
        if not isinstance(x, t.Tensor):
            bad = f"expected a torch tensor, got {type(x).__name__}"
        elif x.device != self.device:
            bad = f"field on {x.device}, handle on {self.device}"
        elif x.dtype != want:
            bad = f"field dtype {x.dtype}, this call needs {want}"
        elif tuple(x.shape) != (self.n + 1, self.n + 1):
            bad = f"field shape {tuple(x.shape)}, expected {(self.n + 1, self.n + 1)}"
        elif tuple(x.stride()) != (self.pitch, 1):
            bad = f"field strides {tuple(x.stride())}, expected {(self.pitch, 1)} (use Grid.field())"
        else:
            avail = x.untyped_storage().nbytes() - x.storage_offset() * x.element_size()
            if avail < (self.n + 1) * self.pitch * x.element_size():
                bad = f"field storage holds {avail} bytes, needs {(self.n + 1) * self.pitch * x.element_size()}"
        if bad is not None:
            raise MGCError(MGC_EINVAL, bad)
        return ctypes.c_void_p(x.data_ptr())

    def _prec(self, x):
        """Precision of the call from the first field's dtype (the other
        fields must match it: _ptr checks them against it)."""
        if getattr(x, "dtype", None) == self.torch.complex64:
            return FP32
        return FP64

    # ---- entry points (same names as the C ABI) -------------------------------
    def set_potential(self, Z1, Z2, lam):
        _check(self.lib.mgc_set_potential(self.h, Z1, Z2, lam))

    def set_potential_exp(self, a1=4.5, b1=1.0, a2=4.5, b2=1.0, c12=2.0, d12=0.1):
        """Exponential model; defaults are the values of Sec. 6.1 (needs
        pot_tables=1 at construction)."""
        _check(self.lib.mgc_set_potential_exp(self.h, a1, b1, a2, b2, c12, d12))

    def channel_energies(self):
        """(lambda_i of H1 for i < M, lambda_l of H2 for l < Lch) as complex arrays."""
        import numpy as np
        a = (ctypes.c_double * (2 * max(self.M, 1)))()
        b = (ctypes.c_double * (2 * max(self.Lch, 1)))()
        _check(self.lib.mgc_channel_energies(self.h, a, b))
        la = np.array(a[:2 * self.M]).view(complex) if self.M else np.zeros(0, complex)
        lb = np.array(b[:2 * self.Lch]).view(complex) if self.Lch else np.zeros(0, complex)
        return la, lb

    def set_energy(self, E):
        _check(self.lib.mgc_set_energy(self.h, E))

    def build_rhs_tp(self, chi):
        _check(self.lib.mgc_build_rhs_tp(self.h, self._ptr(chi), FP64))
        return chi

    def residual(self, u, f, r, want_relres=True):
        rel = ctypes.c_double()
        p = self._prec(u)
        _check(self.lib.mgc_residual(self.h, self._ptr(u, p), self._ptr(f, p), self._ptr(r, p),
                                     ctypes.byref(rel) if want_relres else None, p))
        return rel.value if want_relres else None

    def vcycle(self, u, f):
        p = self._prec(u)
        _check(self.lib.mgc_vcycle(self.h, self._ptr(u, p), self._ptr(f, p), p))

    def cccs(self, u, f):
        p = self._prec(u)
        _check(self.lib.mgc_cccs(self.h, self._ptr(u, p), self._ptr(f, p), p))

    def cccs_noalloc(self, u, f):
        """mgc_cccs with its scratch in the library's static device array."""
        p = self._prec(u)
        _check(self.lib.mgc_cccs_noalloc(self.h, self._ptr(u, p), self._ptr(f, p), p))

    def _solve(self, fn, u, f, outer, inner, restart, max_it, inner_cycles, tol, hist_cap):
        opts = SolveOpts(outer, inner, restart, max_it, inner_cycles, tol)
        hist = (ctypes.c_double * hist_cap)()
        st = Stats(0, 0, 0.0, ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), hist_cap, 0,
                   0.0, 0.0)
        rc = _check(fn(self.h, self._ptr(u), self._ptr(f), ctypes.byref(opts), ctypes.byref(st)),
                    allow=(MGC_ENOCONV, MGC_ENUMERIC))
        hv = [hist[i] for i in range(st.hist_len)]
        return SolveResult(rc, st.iters, st.vcycles, st.relres, hv, st.t_setup_ms, st.t_solve_ms)

    def solve(self, u, f, outer=FGMRES, inner=FP64, restart=10, max_it=1000, inner_cycles=2,
              tol=1e-10, hist_cap=4096):
        return self._solve(self.lib.mgc_solve, u, f, outer, inner, restart, max_it, inner_cycles,
                           tol, hist_cap)

    def solve_transpose(self, v, g, outer=FGMRES, inner=FP64, restart=10, max_it=1000,
                        inner_cycles=2, tol=1e-10, hist_cap=4096):
        return self._solve(self.lib.mgc_solve_transpose, v, g, outer, inner, restart, max_it,
                           inner_cycles, tol, hist_cap)

    def cross_section_grad(self, u, chi, k1, k2, v, outer=FGMRES, inner=FP64, restart=10,
                           max_it=5000, tol=1e-13, hist_cap=4096):
        """(d sigma / d(Z1, Z2, lambda), zeta, sigma, adjoint SolveResult); v holds
        the adjoint initial guess on entry and the adjoint solution on exit."""
        opts = SolveOpts(outer, inner, restart, max_it, 2, tol)
        hist = (ctypes.c_double * hist_cap)()
        st = Stats(0, 0, 0.0, ctypes.cast(hist, ctypes.POINTER(ctypes.c_double)), hist_cap, 0,
                   0.0, 0.0)
        ds = (ctypes.c_double * 3)()
        z = (ctypes.c_double * 2)()
        sig = ctypes.c_double()
        rc = _check(self.lib.mgc_cross_section_grad(self.h, self._ptr(u), self._ptr(chi), k1, k2,
                                                    ctypes.byref(opts), self._ptr(v), ds, z,
                                                    ctypes.byref(sig), ctypes.byref(st)),
                    allow=(MGC_ENOCONV,))
        res = SolveResult(rc, st.iters, st.vcycles, st.relres,
                          [hist[i] for i in range(st.hist_len)], st.t_setup_ms, st.t_solve_ms)
        return [ds[0], ds[1], ds[2]], complex(z[0], z[1]), sig.value, res

    def set_schedule(self, small_tiles=-1, level_pairs=1, coarse_tail=1):
        """Launch schedule of the zero-guess cycle (same results either way)."""
        _check(self.lib.mgc_set_schedule(self.h, ctypes.byref(Schedule(small_tiles, level_pairs, coarse_tail))))

    def get_schedule(self):
        s = Schedule()
        _check(self.lib.mgc_get_schedule(self.h, ctypes.byref(s)))
        return s.small_tiles, s.level_pairs, s.coarse_tail

    def set_kernel_timer(self, kernel_class: int):
        """Time every launch of one kernel class inside FGMRES solves (KT_*)."""
        _check(self.lib.mgc_set_kernel_timer(self.h, kernel_class))

    def read_kernel_timer(self):
        """(total ms, launches, algorithmic bytes, empty-pair ms) since the last
        read; clears."""
        t = KernelTiming()
        _check(self.lib.mgc_read_kernel_timer(self.h, ctypes.byref(t)))
        return t.total_ms, t.launches, t.bytes, t.floor_ms

    def cross_section(self, u, chi, k1, k2):
        z = (ctypes.c_double * 2)()
        sig = ctypes.c_double()
        _check(self.lib.mgc_cross_section(self.h, self._ptr(u), self._ptr(chi), k1, k2, z,
                                          ctypes.byref(sig)))
        return complex(z[0], z[1]), sig.value


    def cross_section_sweep(self, u, chi, k1s, k2s):
        """zeta and sigma for every pair (k1s[a], k2s[a]) in one pass (at most
        SWEEP_MAX pairs); returns (list of complex zeta, list of sigma)."""
        npairs = len(k1s)
        assert len(k2s) == npairs
        a1 = (ctypes.c_double * npairs)(*[float(k) for k in k1s])
        a2 = (ctypes.c_double * npairs)(*[float(k) for k in k2s])
        z = (ctypes.c_double * (2 * npairs))()
        sig = (ctypes.c_double * npairs)()
        _check(self.lib.mgc_cross_section_sweep(self.h, self._ptr(u), self._ptr(chi), npairs, a1, a2, z, sig))
        return [complex(z[2 * a], z[2 * a + 1]) for a in range(npairs)], [sig[a] for a in range(npairs)]

    def single_ionization(self, u, chi, nstates):
        """(s_n for n = 1..nstates, k_n): single-ionisation amplitudes (Sec. 3.3)."""
        s = (ctypes.c_double * (2 * nstates))()
        kn = (ctypes.c_double * nstates)()
        _check(self.lib.mgc_single_ionization(self.h, self._ptr(u), self._ptr(chi), nstates, s, kn))
        return [complex(s[2 * q], s[2 * q + 1]) for q in range(nstates)], [kn[q] for q in range(nstates)]

    def total_double_ionization(self, u, chi, nodes=32):
        """(sigma_tot, zeta at the Gauss-Legendre angles, ascending) (Sec. 3.3)."""
        sig = ctypes.c_double()
        z = (ctypes.c_double * (2 * nodes))()
        _check(self.lib.mgc_total_double_ionization(self.h, self._ptr(u), self._ptr(chi), nodes,
                                                    ctypes.byref(sig), z))
        return sig.value, [complex(z[2 * q], z[2 * q + 1]) for q in range(nodes)]


def sharing_momenta(E_excess: float, alphas):
    """Momentum pairs k1 = K cos a, k2 = K sin a of an energy-sharing sweep,
    K^2 / 2 = E_excess (Sec. 3.3)."""
    K = math.sqrt(2.0 * E_excess)
    return [K * math.cos(a) for a in alphas], [K * math.sin(a) for a in alphas]


def k0_of(E: float, Z1: float = 1.0) -> float:
    """Incoming momentum sqrt(2(E + Z1^2/2)) of the 1s target."""
    return math.sqrt(2.0 * (E + 0.5 * Z1 * Z1))


class Batch:
    """Handles solved together (mgc_batch_*): per restart round, one graph per
    unfinished solve, launched over the batch's streams, and one
    synchronisation for all of them."""

    def __init__(self, grids):
        self.lib = load_library()
        self.grids = list(grids)             # keep the handles alive
        arr = (ctypes.c_void_p * len(self.grids))(*[g.h.value for g in self.grids])
        h = ctypes.c_void_p()
        _check(self.lib.mgc_batch_create(arr, len(self.grids), ctypes.byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.mgc_batch_destroy(h)
            self.h = None

    def cross_sections(self, us, chis, nodes=32, nstates=0):
        """(sigma_tot per solve or None, s_n per solve or None) for every
        handle of the batch in one call (mgc_batch_cross_sections)."""
        nb = len(self.grids)
        up = (ctypes.c_void_p * nb)(*[g._ptr(x).value for g, x in zip(self.grids, us)])
        cp = (ctypes.c_void_p * nb)(*[g._ptr(x).value for g, x in zip(self.grids, chis)])
        sig = (ctypes.c_double * max(nb, 1))()
        s = (ctypes.c_double * max(2 * nstates * nb, 1))()
        _check(self.lib.mgc_batch_cross_sections(self.h, up, cp, nodes, nstates, sig, s))
        sigs = [sig[i] for i in range(nb)] if nodes > 0 else None
        ss = ([[complex(s[2 * nstates * i + 2 * q], s[2 * nstates * i + 2 * q + 1]) for q in range(nstates)]
               for i in range(nb)] if nstates > 0 else None)
        return sigs, ss

    def solve(self, us, fs, inner=FP32, restart=10, max_it=20000, tol=1e-10, hist_cap=4096):
        """Solve grids[i] u_i = f_i for all i; returns one SolveResult each."""
        nb = len(self.grids)
        assert len(us) == nb and len(fs) == nb
        opts = SolveOpts(FGMRES, inner, restart, max_it, 1, tol)
        hists = [(ctypes.c_double * hist_cap)() for _ in range(nb)]
        st = (Stats * nb)()
        for i in range(nb):
            st[i] = Stats(0, 0, 0.0, ctypes.cast(hists[i], ctypes.POINTER(ctypes.c_double)), hist_cap, 0,
                          0.0, 0.0)
        up = (ctypes.c_void_p * nb)(*[g._ptr(x).value for g, x in zip(self.grids, us)])
        fp = (ctypes.c_void_p * nb)(*[g._ptr(x).value for g, x in zip(self.grids, fs)])
        _check(self.lib.mgc_batch_solve(self.h, up, fp, ctypes.byref(opts), st),
               allow=(MGC_ENOCONV, MGC_ENUMERIC))
        out = []
        for i in range(nb):
            s = st[i]
            status = MGC_OK
            if not math.isfinite(s.relres):
                status = MGC_ENUMERIC
            elif s.relres > tol:
                status = MGC_ENOCONV
            out.append(SolveResult(status, s.iters, s.vcycles, s.relres,
                                   [hists[i][k] for k in range(s.hist_len)], s.t_setup_ms, s.t_solve_ms))
        return out
