"""ctypes binding of the C ABI in include/pnp_cdft.h (argument marshalling only).

PyTorch provides device memory (outputs, workspaces) and the current HIP
stream; every step of the evaluation runs in the HIP library.  There is no
fallback: a missing library raises PnpError.
"""
import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

TERM_HS, TERM_EC, TERM_SW, TERM_ALL, TERM_HS_WB = 1, 2, 4, 7, 8
FP64, MIXED = 0, 1
FLAG_ASYNC = 1
FLAG_APERIODIC = 2  # non-periodic domain: zero extension onto the doubled grid
FLAG_CUBIC = 4  # sphere quadrature: tricubic instead of trilinear interpolation

STATUS_NAMES = {
    0: "PNP_OK", -1: "PNP_E_ARG", -2: "PNP_E_UNSUPPORTED_SIZE", -3: "PNP_E_NOMEM",
    -4: "PNP_E_PACKING", -5: "PNP_E_OVERFLOW", -6: "PNP_E_NONFINITE", -7: "PNP_E_DEVICE",
    -8: "PNP_E_BUDGET",
}

EXPORTED = [
    "pnp_create", "pnp_destroy", "pnp_last_error", "pnp_supported_size", "pnp_workspace_bytes",
    "pnp_cdft_mu_ex", "pnp_weighted_densities", "pnp_batch_mu_ex", "pnp_read_status",
    "pnp_relax_densities", "pnp_debug_rfft3", "pnp_debug_copy", "pnp_profile_enable",
    "pnp_profile_select", "pnp_profile_read", "pnp_free_energy", "pnp_equilibrium", "pnp_bulk_mu_ex", "pnp_session_bytes", "pnp_pool_create", "pnp_pool_destroy",
    "pnp_pool_usage", "pnp_session_open", "pnp_session_step", "pnp_session_view", "pnp_session_close",
    "pnp_plan_create", "pnp_plan_launch", "pnp_plan_status", "pnp_plan_destroy", "pnp_pool_graphs",
    "pnp_autotune", "pnp_tune_export", "pnp_tune_import", "pnp_sphere_quadrature", "pnp_cdft_mu_ex_noalloc",
]

PASS_NAMES = ["tables", "z_fwd_rho", "y_fwd_rho", "x_fwd_weights", "y_inv_n", "z_deriv",
              "y_fwd_dphi", "x_back_pairs", "y_inv_mu", "z_inv_final"]


class PnpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double)]


class SpeciesC(ctypes.Structure):
    _fields_ = [("d", ctypes.c_double), ("q", ctypes.c_double), ("rho_bulk", ctypes.c_double),
                ("mu_el_bulk", ctypes.c_double), ("mobile", ctypes.c_int32)]


class ParamsC(ctypes.Structure):
    _fields_ = [("terms", ctypes.c_uint32), ("precision", ctypes.c_int32),
                ("per_term", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("eps_r", ctypes.c_double), ("sw_eps", ctypes.POINTER(ctypes.c_double)),
                ("sw_rout", ctypes.POINTER(ctypes.c_double)), ("sw_gamma", ctypes.c_double),
                ("sw_prefactor", ctypes.c_double)]


class RequestC(ctypes.Structure):
    _fields_ = [("grid", Grid), ("S", ctypes.c_int32), ("species", ctypes.POINTER(SpeciesC)),
                ("rho", ctypes.c_void_p), ("T", ctypes.c_double),
                ("params", ctypes.POINTER(ParamsC)), ("mu_ex", ctypes.c_void_p),
                ("slotboom", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("status", ctypes.c_int32)]


class RelaxSpecC(ctypes.Structure):
    _fields_ = [("mu_bulk", ctypes.POINTER(ctypes.c_double)), ("lambda_", ctypes.c_double),
                ("clip", ctypes.c_double)]


_LIB = None


def lib_path() -> str:
    return os.environ.get("PNP_CDFT_LIB", os.path.join(HERE, "libpnpcdft.so"))


def load_library():
    """Load libpnpcdft.so (built in-tree by paper_1407_0674_amd.build)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise PnpError(-7, f"HIP library not built: {path} (run python -m paper_1407_0674_amd.build)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.pnp_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
    lib.pnp_destroy.argtypes = [P]
    lib.pnp_destroy.restype = None
    lib.pnp_last_error.argtypes = [P]
    lib.pnp_last_error.restype = ctypes.c_char_p
    lib.pnp_supported_size.argtypes = [ctypes.c_int32]
    lib.pnp_workspace_bytes.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32,
                                        ctypes.POINTER(ParamsC), ctypes.POINTER(ctypes.c_size_t)]
    lib.pnp_cdft_mu_ex.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(SpeciesC),
                                   P, ctypes.c_double, ctypes.POINTER(ParamsC), P, P, P,
                                   ctypes.c_size_t, P]
    lib.pnp_cdft_mu_ex_noalloc.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(SpeciesC),
                                           P, ctypes.c_double, ctypes.POINTER(ParamsC), P, P, P]
    lib.pnp_weighted_densities.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32,
                                           ctypes.POINTER(SpeciesC), P, ctypes.POINTER(ParamsC), P,
                                           P, ctypes.c_size_t, P]
    lib.pnp_batch_mu_ex.argtypes = [P, ctypes.c_int32, ctypes.POINTER(RequestC), P]
    lib.pnp_sphere_quadrature.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, P,
                                          ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_uint32, P, P]
    lib.pnp_equilibrium.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(SpeciesC),
                                    ctypes.c_double, ctypes.POINTER(ParamsC), P, P, P, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double), P, ctypes.c_size_t, P]
    lib.pnp_free_energy.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(SpeciesC), P,
                                    ctypes.c_double, ctypes.POINTER(ParamsC), ctypes.POINTER(ctypes.c_double),
                                    P, P, ctypes.c_size_t, P]
    lib.pnp_read_status.argtypes = [P, P, P]
    lib.pnp_relax_densities.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32,
                                        ctypes.POINTER(SpeciesC), P, P,
                                        ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double, P]
    lib.pnp_debug_rfft3.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
    lib.pnp_debug_copy.argtypes = [P, P, P, ctypes.c_size_t, P]
    lib.pnp_bulk_mu_ex.argtypes = [P, ctypes.c_int32, ctypes.POINTER(SpeciesC), ctypes.c_double,
                                   ctypes.POINTER(ParamsC), ctypes.POINTER(ctypes.c_double)]
    lib.pnp_session_bytes.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(ParamsC),
                                      ctypes.POINTER(ctypes.c_size_t)]
    lib.pnp_pool_create.argtypes = [P, P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.pnp_pool_destroy.argtypes = [P]
    lib.pnp_pool_destroy.restype = None
    lib.pnp_pool_usage.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.pnp_session_open.argtypes = [P, ctypes.POINTER(Grid), ctypes.c_int32, ctypes.POINTER(SpeciesC),
                                     ctypes.c_double, ctypes.POINTER(ParamsC), P,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_double, P,
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.pnp_session_step.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32), P]
    lib.pnp_session_view.argtypes = [P, ctypes.c_int64, ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64)]
    lib.pnp_session_close.argtypes = [P, ctypes.c_int64]
    lib.pnp_plan_create.argtypes = [P, ctypes.c_int32, ctypes.POINTER(RequestC), ctypes.POINTER(RelaxSpecC),
                                    ctypes.POINTER(P)]
    lib.pnp_plan_launch.argtypes = [P, P]
    lib.pnp_plan_status.argtypes = [P, P, ctypes.POINTER(ctypes.c_int32)]
    lib.pnp_plan_destroy.argtypes = [P]
    lib.pnp_plan_destroy.restype = None
    lib.pnp_pool_graphs.argtypes = [P, ctypes.c_int32]
    lib.pnp_autotune.argtypes = [P, ctypes.c_int32, ctypes.POINTER(RequestC), ctypes.c_int32, P]
    lib.pnp_tune_export.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
    lib.pnp_tune_import.argtypes = [P, ctypes.c_char_p]
    lib.pnp_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.pnp_profile_select.argtypes = [P, ctypes.c_uint32]
    lib.pnp_profile_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.c_int32, ctypes.c_int32]
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("pnp_destroy", "pnp_last_error", "pnp_pool_destroy", "pnp_plan_destroy"):
            f.restype = ctypes.c_int
    _LIB = lib
    return lib


class _Marshal:
    """Host-side C records of one problem description (kept alive for a call)."""

    def __init__(self, problem, per_term=False, flags=0, precision=None):
        S = len(problem.species)
        self.grid = Grid(problem.n, problem.n, problem.n, float(problem.h))
        self.species = (SpeciesC * S)(*[SpeciesC(s.d, s.q, s.rho_bulk, s.mu_el_bulk,
                                                  int(bool(getattr(s, "mobile", True))))
                                         for s in problem.species])
        self._eps = None if problem.sw_eps is None else np.ascontiguousarray(problem.sw_eps, dtype=np.float64)
        self._rout = None if problem.sw_rout is None else np.ascontiguousarray(problem.sw_rout, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        self.params = ParamsC(
            int(problem.terms), int(problem.precision if precision is None else precision),
            int(bool(per_term)), int(flags), float(problem.eps_r),
            self._eps.ctypes.data_as(dp) if self._eps is not None else dp(),
            self._rout.ctypes.data_as(dp) if self._rout is not None else dp(),
            float(problem.sw_gamma), float(problem.sw_prefactor))
        self.S = S
        self.T = float(problem.T)


def _torch():
    import torch
    return torch


class Evaluator:
    """One library context on one GPU."""

    def __init__(self, device: Optional[int] = None):
        torch = _torch()
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else int(device)
        ctx = ctypes.c_void_p()
        st = self.lib.pnp_create(self.device, ctypes.byref(ctx))
        if st != 0:
            raise PnpError(st, "pnp_create failed")
        self.ctx = ctx
        self._ws = {}
        cache = os.environ.get("PNP_TUNE_CACHE")
        if cache and os.path.exists(cache):
            with open(cache) as f:
                self.tune_import(f.read())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pnp_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def _check(self, st):
        if st != 0:
            raise PnpError(st, self.lib.pnp_last_error(self.ctx).decode())

    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)

    def workspace_bytes(self, problem, per_term=False, precision=None, flags=0) -> int:
        return self._ws_bytes(_Marshal(problem, per_term, flags, precision=precision))

    def _ws_bytes(self, m) -> int:
        out = ctypes.c_size_t()
        self._check(self.lib.pnp_workspace_bytes(self.ctx, ctypes.byref(m.grid), m.S,
                                                 ctypes.byref(m.params), ctypes.byref(out)))
        return int(out.value)

    def workspace(self, nbytes: int, key="default"):
        """A cached uint8 device buffer of at least nbytes (torch allocations
        are 256-byte aligned)."""
        torch = _torch()
        buf = self._ws.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws[key] = buf
        return buf

    @staticmethod
    def _dev(t, name):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise PnpError(-1, f"{name} must be a contiguous float64 CUDA tensor")
        return ctypes.c_void_p(t.data_ptr())

    # -- the C ABI calls ------------------------------------------------------
    def mu_ex(self, problem, rho, per_term=False, slotboom=True, out=None, slot=None,
              workspace=None, flags=0, precision=None):
        torch = _torch()
        m = _Marshal(problem, per_term, flags, precision)
        n3 = problem.n ** 3
        if tuple(rho.shape) != (m.S, problem.n, problem.n, problem.n):
            raise PnpError(-1, f"rho has shape {tuple(rho.shape)}")
        if out is None:
            shape = (3, m.S, problem.n, problem.n, problem.n) if per_term else (m.S, problem.n, problem.n, problem.n)
            out = torch.empty(shape, dtype=torch.float64, device=rho.device)
        if slotboom and slot is None:
            slot = torch.empty((m.S, problem.n, problem.n, problem.n), dtype=torch.float64, device=rho.device)
        ws = self.workspace(self._ws_bytes(m)) if workspace is None else workspace
        st = self.lib.pnp_cdft_mu_ex(
            self.ctx, ctypes.byref(m.grid), m.S, m.species, self._dev(rho, "rho"), m.T,
            ctypes.byref(m.params), self._dev(out, "mu_ex"),
            self._dev(slot, "slotboom") if slotboom else ctypes.c_void_p(0),
            ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()), self._stream())
        self._check(st)
        return out, (slot if slotboom else None)

    def mu_ex_noalloc(self, problem, rho, out, slot=None, per_term=False, flags=0, precision=None):
        """pnp_cdft_mu_ex_noalloc: the evaluation into caller-given outputs with
        the library's static scratch array as workspace (no allocation here or
        in the library)."""
        m = _Marshal(problem, per_term, flags, precision)
        st = self.lib.pnp_cdft_mu_ex_noalloc(
            self.ctx, ctypes.byref(m.grid), m.S, m.species, self._dev(rho, "rho"), m.T, ctypes.byref(m.params),
            self._dev(out, "mu_ex"), self._dev(slot, "slotboom") if slot is not None else ctypes.c_void_p(0),
            self._stream())
        self._check(st)
        return out, slot

    def free_energy(self, problem, rho, precision=None):
        """{"hs", "el", "sh", "total"} excess free energies [k_B T] and the
        per-term beta mu_ex [3][S][n][n][n] they came from."""
        torch = _torch()
        m = _Marshal(problem, True, 0, precision)
        mu3 = torch.empty((3, m.S, problem.n, problem.n, problem.n), dtype=torch.float64, device=rho.device)
        nb = self.workspace_bytes(problem, True, precision)
        ws = self.workspace(nb)
        out = (ctypes.c_double * 4)()
        self._check(self.lib.pnp_free_energy(self.ctx, ctypes.byref(m.grid), m.S, m.species,
                                             self._dev(rho, "rho"), m.T, ctypes.byref(m.params), out,
                                             self._dev(mu3, "mu3"), ctypes.c_void_p(ws.data_ptr()),
                                             ctypes.c_size_t(ws.numel()), self._stream()))
        return {"hs": out[0], "el": out[1], "sh": out[2], "total": out[3]}, mu3

    def equilibrium(self, problem, rho, beta_v=None, lam=0.1, tol=1e-10, max_iter=200, precision=None):
        """Picard solve of the grand-ensemble equilibrium in place on `rho`;
        returns (mu_ex of the last evaluated densities, iterations, residual)."""
        torch = _torch()
        m = _Marshal(problem, False, 0, precision)
        mu = torch.empty_like(rho)
        nb = self.workspace_bytes(problem, False, precision)
        ws = self.workspace(nb)
        it = ctypes.c_int32()
        res = ctypes.c_double()
        self._check(self.lib.pnp_equilibrium(
            self.ctx, ctypes.byref(m.grid), m.S, m.species, m.T, ctypes.byref(m.params),
            self._dev(beta_v, "beta_v") if beta_v is not None else ctypes.c_void_p(0),
            self._dev(rho, "rho"), self._dev(mu, "mu_ex"), float(lam), float(tol), int(max_iter),
            ctypes.byref(it), ctypes.byref(res), ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
            self._stream()))
        return mu, int(it.value), float(res.value)

    def weighted_densities(self, problem, rho, precision=None):
        torch = _torch()
        m = _Marshal(problem, False, 0, precision)
        out = torch.empty((10, problem.n, problem.n, problem.n), dtype=torch.float64, device=rho.device)
        q = problem.with_(terms=TERM_HS) if hasattr(problem, "with_") else problem
        nb = self.workspace_bytes(q, False, precision)
        ws = self.workspace(nb)
        st = self.lib.pnp_weighted_densities(
            self.ctx, ctypes.byref(m.grid), m.S, m.species, self._dev(rho, "rho"),
            ctypes.byref(m.params), self._dev(out, "n_out"), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_size_t(ws.numel()), self._stream())
        self._check(st)
        return out

    def sphere_quadrature(self, f, radius, h, order=8, precision=MIXED, flags=0, out=None):
        """Sphere integrals (I, I_x, I_y, I_z) of each field by the product rule of
        Sec. 3.5; f is [F, nx, ny, nz] float64 on the device, radius F values [nm].
        Returns out [F, 4, nx, ny, nz]."""
        torch = _torch()
        if f.dim() != 4:
            raise PnpError(-1, f"f has shape {tuple(f.shape)}, expected [F, nx, ny, nz]")
        F, nx, ny, nz = (int(v) for v in f.shape)
        radii = [float(r) for r in radius]
        if len(radii) != F:
            raise PnpError(-1, f"{len(radii)} radii for {F} fields")
        if out is None:
            out = torch.empty((F, 4, nx, ny, nz), dtype=torch.float64, device=f.device)
        elif tuple(out.shape) != (F, 4, nx, ny, nz):
            raise PnpError(-1, f"out has shape {tuple(out.shape)}")
        g = Grid(nx, ny, nz, float(h))
        r = (ctypes.c_double * F)(*radii)
        st = self.lib.pnp_sphere_quadrature(self.ctx, ctypes.byref(g), F, self._dev(f, "f"), r, int(order),
                                            int(precision), int(flags), self._dev(out, "out"), self._stream())
        self._check(st)
        return out

    def _requests(self, problems, rhos, slotboom, workspaces, outs, slots):
        """C request records for `problems` with their output and workspace
        tensors; returns (reqs, keep-alive list, mu list, slot list)."""
        torch = _torch()
        count = len(problems)
        ms = [_Marshal(p) for p in problems]
        reqs = (RequestC * count)()
        keep = [ms]
        mus, sls = [], []
        for r, (p, m, rho) in enumerate(zip(problems, ms, rhos)):
            mu = outs[r] if outs is not None else torch.empty(tuple(rho.shape), dtype=torch.float64, device=rho.device)
            sl = None
            if slotboom:
                sl = slots[r] if slots is not None else torch.empty(tuple(rho.shape), dtype=torch.float64, device=rho.device)
            if workspaces is not None:
                ws = workspaces[r]
            else:
                ws = torch.empty(self.workspace_bytes(p), dtype=torch.uint8, device=rho.device)
            keep.append(ws)
            reqs[r].grid = m.grid
            reqs[r].S = m.S
            reqs[r].species = ctypes.cast(m.species, ctypes.POINTER(SpeciesC))
            reqs[r].rho = self._dev(rho, "rho").value
            reqs[r].T = m.T
            reqs[r].params = ctypes.pointer(m.params)
            reqs[r].mu_ex = mu.data_ptr()
            reqs[r].slotboom = sl.data_ptr() if sl is not None else None
            reqs[r].workspace = ws.data_ptr()
            reqs[r].workspace_bytes = ws.numel()
            mus.append(mu)
            sls.append(sl)
        return reqs, keep, mus, sls

    def batch(self, problems: Sequence, rhos: Sequence, slotboom=True, workspaces=None,
              outs=None, slots=None):
        """Evaluate independent problems in shared launches.  Returns
        (mu list, slot list, status list)."""
        count = len(problems)
        reqs, keep, mus, sls = self._requests(problems, rhos, slotboom, workspaces, outs, slots)
        st = self.lib.pnp_batch_mu_ex(self.ctx, count, reqs, self._stream())
        self._check(st)
        return mus, sls, [int(reqs[r].status) for r in range(count)]

    def autotune(self, problems: Sequence, rhos: Sequence, reps: int = 3):
        """Time both FFT schedules and both tile shapes of every pass on these
        problems (evaluated as one batch), keep the faster per pass, and keep
        that choice in this context only if it beats the size's default end
        to end (schedule per precision and size, tile shape also per
        instance-count class); returns the statuses.  Saved to
        $PNP_TUNE_CACHE when that is set."""
        count = len(problems)
        reqs, keep, _, _ = self._requests(problems, rhos, True, None, None, None)
        self._check(self.lib.pnp_autotune(self.ctx, count, reqs, int(reps), self._stream()))
        cache = os.environ.get("PNP_TUNE_CACHE")
        if cache:
            with open(cache, "w") as f:
                f.write(self.tune_export())
        return [int(reqs[r].status) for r in range(count)]

    def tune_export(self) -> str:
        n = ctypes.c_size_t()
        self._check(self.lib.pnp_tune_export(self.ctx, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value + 1)
        self._check(self.lib.pnp_tune_export(self.ctx, buf, n.value + 1, ctypes.byref(n)))
        return buf.value.decode()

    def tune_import(self, text: str):
        self._check(self.lib.pnp_tune_import(self.ctx, text.encode()))

    def plan(self, problems: Sequence, rhos: Sequence, slotboom=True, workspaces=None, outs=None,
             slots=None, relax=None):
        """Capture the evaluation of these buffers in a HIP graph (see Plan)."""
        return Plan(self, problems, rhos, slotboom, workspaces, outs, slots, relax)

    def profile(self, enable: bool = True, passes=None):
        """Pass timing on/off; `passes`: names of the passes that record
        events (default all)."""
        mask = 0xFFFFFFFF if passes is None else sum(1 << PASS_NAMES.index(p) for p in passes)
        self._check(self.lib.pnp_profile_select(self.ctx, mask))
        self._check(self.lib.pnp_profile_enable(self.ctx, int(bool(enable))))

    def profile_read(self, reset: bool = True):
        """{pass name: (total ms, launches)} since the last reset."""
        ms = (ctypes.c_double * 10)()
        cnt = (ctypes.c_int32 * 10)()
        self._check(self.lib.pnp_profile_read(self.ctx, ms, cnt, 10, int(bool(reset))))
        return {PASS_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(10)}

    def read_status(self, workspace=None):
        ws = self._ws["default"] if workspace is None else workspace
        self._check(self.lib.pnp_read_status(self.ctx, ctypes.c_void_p(ws.data_ptr()), self._stream()))

    def relax(self, problem, rho, mu, mu_bulk, lam=0.1, clip=0.0):
        m = _Marshal(problem)
        mb = (ctypes.c_double * m.S)(*[float(x) for x in mu_bulk])
        self._check(self.lib.pnp_relax_densities(self.ctx, ctypes.byref(m.grid), m.S, m.species,
                                                 self._dev(rho, "rho"), self._dev(mu, "mu"), mb,
                                                 float(lam), float(clip), self._stream()))

    def _fft_workspace(self, n, count, precision):
        g = Grid(n, n, n, 1.0)
        prm = ParamsC(0, int(precision), 0, 0, 1.0, ctypes.POINTER(ctypes.c_double)(),
                      ctypes.POINTER(ctypes.c_double)(), 1.2, 0.5)
        nb = ctypes.c_size_t()
        self._check(self.lib.pnp_workspace_bytes(self.ctx, ctypes.byref(g), count, ctypes.byref(prm),
                                                 ctypes.byref(nb)))
        return self.workspace(int(nb.value), "fft")

    def rfft3(self, x, precision=FP64):
        """Forward 3D real DFT through the library's passes, numpy layout."""
        torch = _torch()
        count, n = x.shape[0], x.shape[1]
        out = torch.empty((count, n, n, n // 2 + 1, 2), dtype=torch.float64, device=x.device)
        g = Grid(n, n, n, 1.0)
        ws = self._fft_workspace(n, count, precision)
        self._check(self.lib.pnp_debug_rfft3(self.ctx, ctypes.byref(g), precision, count, 0,
                                             self._dev(x, "in"), self._dev(out, "out"),
                                             ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                             self._stream()))
        return torch.view_as_complex(out)

    def irfft3(self, X, precision=FP64):
        """Unnormalised inverse (numpy irfftn times n^3) from numpy layout."""
        torch = _torch()
        count, n = X.shape[0], X.shape[1]
        Xr = torch.view_as_real(X.contiguous()).contiguous()
        out = torch.empty((count, n, n, n), dtype=torch.float64, device=X.device)
        g = Grid(n, n, n, 1.0)
        ws = self._fft_workspace(n, count, precision)
        self._check(self.lib.pnp_debug_rfft3(self.ctx, ctypes.byref(g), precision, count, 1,
                                             self._dev(Xr, "in"), self._dev(out, "out"),
                                             ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
                                             self._stream()))
        return out

    def copy(self, src, dst):
        """Device copy through the library's calibration kernel (asynchronous)."""
        torch = _torch()
        for t, nm in ((src, "src"), (dst, "dst")):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
                raise PnpError(-1, f"{nm} must be a contiguous CUDA tensor")
        nbytes = src.numel() * src.element_size()
        if dst.numel() * dst.element_size() != nbytes:
            raise PnpError(-1, "copy: size mismatch")
        self._check(self.lib.pnp_debug_copy(self.ctx, ctypes.c_void_p(src.data_ptr()),
                                            ctypes.c_void_p(dst.data_ptr()), ctypes.c_size_t(nbytes),
                                            self._stream()))


class Plan:
    """A captured evaluation (pnp_plan_* in the header): the requests' buffers
    are bound at creation; launch() replays every kernel as one graph launch
    on the current stream, status() waits and returns each request's status.
    relax: None, or one (mu_bulk, lam, clip) per request: each replay then
    also relaxes that request's rho in place after its evaluation."""

    def __init__(self, ev, problems, rhos, slotboom=True, workspaces=None, outs=None, slots=None, relax=None):
        self.ev = ev
        self.lib = ev.lib
        self.count = len(problems)
        reqs, keep, self.mu, self.slot = ev._requests(problems, rhos, slotboom, workspaces, outs, slots)
        self._keep = [keep, list(rhos)]
        rspec = None
        if relax is not None:
            rspec = (RelaxSpecC * self.count)()
            for r, (mb, lam, clip) in enumerate(relax):
                arr = (ctypes.c_double * len(mb))(*[float(x) for x in mb])
                self._keep.append(arr)
                rspec[r] = RelaxSpecC(ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)), float(lam), float(clip))
        plan = ctypes.c_void_p()
        ev._check(self.lib.pnp_plan_create(ev.ctx, self.count, reqs, rspec, ctypes.byref(plan)))
        self.plan = plan
        self.created_status = [int(reqs[r].status) for r in range(self.count)]

    def launch(self):
        self.ev._check(self.lib.pnp_plan_launch(self.plan, self.ev._stream()))

    def status(self):
        out = (ctypes.c_int32 * self.count)()
        self.ev._check(self.lib.pnp_plan_status(self.plan, self.ev._stream(), out))
        return [int(x) for x in out]

    def close(self):
        if getattr(self, "plan", None):
            self.lib.pnp_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bulk_mu_ex(problem):
    """beta mu_ex of the uniform bulk state of `problem` (host arithmetic in
    the library; no device needed).  Returns a list of S floats."""
    lib = load_library()
    m = _Marshal(problem)
    out = (ctypes.c_double * m.S)()
    st = lib.pnp_bulk_mu_ex(None, m.S, m.species, m.T, ctypes.byref(m.params), out)
    if st != 0:
        raise PnpError(st, "pnp_bulk_mu_ex failed")
    return [float(x) for x in out]


class Pool:
    """Resident sessions in one device pool (see pnp_session_* in the header).

    The pool's memory is one uint8 CUDA tensor of `nbytes` owned by this
    object; sessions are sub-allocated from it by the library."""

    def __init__(self, ev: "Evaluator", nbytes: int):
        torch = _torch()
        self.ev = ev
        self.lib = ev.lib
        self.arena = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{ev.device}")
        pool = ctypes.c_void_p()
        ev._check(self.lib.pnp_pool_create(ev.ctx, ctypes.c_void_p(self.arena.data_ptr()),
                                           ctypes.c_size_t(self.arena.numel()), ctypes.byref(pool)))
        self.pool = pool
        self._marshal = {}

    def close(self):
        if getattr(self, "pool", None):
            _torch().cuda.synchronize()
            self.lib.pnp_pool_destroy(self.pool)
            self.pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def session_bytes(self, problem) -> int:
        m = _Marshal(problem)
        out = ctypes.c_size_t()
        self.ev._check(self.lib.pnp_session_bytes(self.ev.ctx, ctypes.byref(m.grid), m.S,
                                                  ctypes.byref(m.params), ctypes.byref(out)))
        return int(out.value)

    def graphs(self, max_plans: int):
        """Replay steps from captured graphs (up to max_plans id lists); 0: off."""
        self.ev._check(self.lib.pnp_pool_graphs(self.pool, int(max_plans)))

    def usage(self):
        used, big, n = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int32()
        self.ev._check(self.lib.pnp_pool_usage(self.pool, ctypes.byref(used), ctypes.byref(big), ctypes.byref(n)))
        return int(used.value), int(big.value), int(n.value)

    def open(self, problem, rho0, mu_bulk=None, lam=0.1, clip=1.0):
        """Admit a session; returns its id, or None when it does not fit now."""
        m = _Marshal(problem)
        mb = None if mu_bulk is None else (ctypes.c_double * m.S)(*[float(x) for x in mu_bulk])
        sid = ctypes.c_int64()
        st = self.lib.pnp_session_open(self.pool, ctypes.byref(m.grid), m.S, m.species, m.T,
                                       ctypes.byref(m.params), self.ev._dev(rho0, "rho0"), mb, float(lam),
                                       float(clip), self.ev._stream(), ctypes.byref(sid))
        if st == -8:
            return None
        self.ev._check(st)
        self._marshal[int(sid.value)] = (problem, m)
        return int(sid.value)

    def step(self, ids):
        """One step of the listed sessions; returns their statuses."""
        n = len(ids)
        arr = (ctypes.c_int64 * n)(*ids)
        st = (ctypes.c_int32 * n)()
        self.ev._check(self.lib.pnp_session_step(self.pool, n, arr, st, self.ev._stream()))
        return [int(x) for x in st]

    def view(self, sid):
        """(rho, mu_ex, slotboom, steps): CUDA tensors viewing the session's
        resident arrays (valid until it closes)."""
        torch = _torch()
        problem, m = self._marshal[sid]
        rp, mp, sp_, steps = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        self.ev._check(self.lib.pnp_session_view(self.pool, sid, ctypes.byref(rp), ctypes.byref(mp),
                                                 ctypes.byref(sp_), ctypes.byref(steps)))
        shape = (m.S, problem.n, problem.n, problem.n)
        base = self.arena.data_ptr()
        out = []
        for ptr in (rp, mp, sp_):
            off = int(ptr.value) - base
            nb = 8 * m.S * problem.n ** 3
            out.append(self.arena[off:off + nb].view(torch.float64).view(shape))
        return out[0], out[1], out[2], int(steps.value)

    def close_session(self, sid):
        self.ev._check(self.lib.pnp_session_close(self.pool, sid))
        self._marshal.pop(sid, None)
