"""Python binding of the MI355X interpolated-Ewald library (libankh.so).

Argument marshalling only: every step of an evaluation runs in the HIP
kernels behind the C ABI declared in include/ankh.h.  The functions below
carry the C names (`ankh_plan`, `ankh_energy`, `ankh_energy_forces`,
`ankh_energy_derivs`, `ankh_energy_octupole`, `ankh_induce`, ...);
`Plan` wraps a plan handle and `AnkhEnergy` is the autograd function whose
backward returns -g F for the positions, g dE/dmu for the dipoles and, when
asked for, g dE/dq and g dE/dTheta.

Device memory and streams come from PyTorch (ROCm): every array argument is
a contiguous float64 tensor on the GPU.  There is no CPU fallback: the module
raises if the library is not built or no GPU is present.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libankh.so")

ANKH_FP64 = 0
ANKH_MIXED = 1
ANKH_MIXED_BF16X3 = 2
ANKH_FAR_AUTO = 0
ANKH_FAR_FMM = 1
ANKH_FAR_FFT = 2

STATUS = {
    0: "ok", 1: "invalid argument", 2: "non-finite input", 3: "quadrupole or octupole not traceless",
    4: "leaf overflow", 5: "accuracy unreachable in this precision", 6: "out of device memory",
    7: "HIP runtime error", 8: "induced dipoles not converged",
}

STAGES = ["sort", "gather", "p2m", "m2m", "m2l", "periodic", "l2l", "l2p", "p2p", "p2p_sum", "reduce"]


class AnkhError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, 'unknown')} (status {status})")
        self.status = status


class _Overrides(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("order", ctypes.c_int32), ("images", ctypes.c_int32),
                ("xi", ctypes.c_double), ("root_order", ctypes.c_int32), ("m2l_tol", ctypes.c_double),
                ("far_field", ctypes.c_int32), ("eq_order", ctypes.c_int32), ("leaves", ctypes.c_int32),
                ("fft_split", ctypes.c_int32), ("overlap", ctypes.c_int32), ("force_accuracy", ctypes.c_double),
                ("workspace_limit", ctypes.c_int64)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int64), ("depth", ctypes.c_int32), ("order", ctypes.c_int32),
                ("images", ctypes.c_int32), ("max_order", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("root_order", ctypes.c_int32), ("xi", ctypes.c_double), ("box_radius", ctypes.c_double), ("rel_accuracy", ctypes.c_double),
                ("plan_ms", ctypes.c_double), ("workspace_bytes", ctypes.c_int64), ("m2l_flops", ctypes.c_double),
                ("near_pairs", ctypes.c_int64), ("stage_ms", ctypes.c_double * len(STAGES)), ("timed_evals", ctypes.c_int64),
                ("m2l_rank", ctypes.c_int32 * 8), ("far_field", ctypes.c_int32), ("eq_order", ctypes.c_int32),
                ("overlap", ctypes.c_int32), ("fft_split", ctypes.c_int32), ("leaves_per_axis", ctypes.c_int32),
                ("near_precision", ctypes.c_int32), ("far_precision", ctypes.c_int32)]


_lib = None

EXPORTS = ["ankh_plan", "ankh_energy", "ankh_energy_forces", "ankh_sync", "ankh_get_stats", "ankh_set_timing",
           "ankh_last_terms", "ankh_leaf_multipoles", "ankh_destroy", "ankh_status_string", "ankh_induce",
           "ankh_energy_derivs", "ankh_energy_derivs_noalloc", "ankh_energy_octupole"]


def load_library(path: str = LIB_PATH):
    """Load libankh.so and declare the C signatures (no GPU call is made)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libankh.so is not built ({path}); run paper_2212_08284_amd/build.py")
    L = ctypes.CDLL(path)
    vp, dp, i64 = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64
    L.ankh_plan.restype = ctypes.c_int
    L.ankh_plan.argtypes = [ctypes.POINTER(vp), i64, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                            ctypes.c_int32, ctypes.POINTER(_Overrides), vp]
    L.ankh_energy.restype = ctypes.c_int
    L.ankh_energy.argtypes = [vp, dp, dp, dp, dp, dp]
    L.ankh_energy_forces.restype = ctypes.c_int
    L.ankh_energy_forces.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp]
    L.ankh_energy_derivs.restype = ctypes.c_int
    L.ankh_energy_derivs.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.ankh_energy_derivs_noalloc.restype = ctypes.c_int
    L.ankh_energy_derivs_noalloc.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.ankh_energy_octupole.restype = ctypes.c_int
    L.ankh_energy_octupole.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.ankh_induce.restype = ctypes.c_int
    L.ankh_induce.argtypes = [vp, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int32, dp, dp, dp,
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    L.ankh_sync.restype = ctypes.c_int
    L.ankh_sync.argtypes = [vp]
    L.ankh_get_stats.restype = ctypes.c_int
    L.ankh_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
    L.ankh_set_timing.restype = ctypes.c_int
    L.ankh_set_timing.argtypes = [vp, ctypes.c_int32]
    L.ankh_last_terms.restype = ctypes.c_int
    L.ankh_last_terms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.ankh_leaf_multipoles.restype = ctypes.c_int
    L.ankh_leaf_multipoles.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64]
    L.ankh_destroy.restype = None
    L.ankh_destroy.argtypes = [vp]
    L.ankh_status_string.restype = ctypes.c_char_p
    L.ankh_status_string.argtypes = [ctypes.c_int]
    _lib = L
    return L


def _check(st: int, where: str):
    if st != 0:
        raise AnkhError(st, where)


def _dev(t, n_cols, n, name, optional=False):
    if t is None:
        if optional:
            return None, None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    t = t.contiguous()
    want = (n,) if n_cols == 1 else (n, n_cols)
    if tuple(t.shape) != want:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want}")
    return t, ctypes.c_void_p(t.data_ptr())


# ---- C-named entry points ------------------------------------------------------

def ankh_plan(n_atoms: int, box_radius: float, rel_accuracy: float, max_order: int = 2,
              precision: int = ANKH_FP64, depth: int | None = None, order: int | None = None,
              images: int | None = None, xi: float | None = None, root_order: int | None = None,
              m2l_tol: float | None = None, stream=None, far_field: int = 0, eq_order: int | None = None,
              overlap: bool | None = None, fft_split: bool = False, leaves: int | None = None,
              force_accuracy: float | None = None, workspace_limit: int | None = None):
    """Create a plan; returns the opaque handle (ctypes.c_void_p).  m2l_tol: singular-value cutoff of the
    compressed M2L (None = automatic, negative = no compression).  far_field: ANKH_FAR_FMM / ANKH_FAR_FFT
    (0 = automatic); eq_order: equispaced nodes per axis of ANKH-FFT (None = the Chebyshev order); overlap:
    far-field chain beside the pair kernel (None = automatic); fft_split: ANKH-FFT cell transforms in three
    passes even when one block could hold them (testing); leaves: ANKH-FFT leaves per axis (None = 2^depth);
    force_accuracy: target relative RMS force error (None = only the energy target); workspace_limit: most
    device bytes the plan may hold (None = no limit)."""
    L = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU: the interpolated-Ewald library runs on the GPU only")
    ov = _Overrides(-1 if depth is None else int(depth), 0 if order is None else int(order),
                    0 if images is None else int(images), 0.0 if xi is None else float(xi),
                    0 if root_order is None else int(root_order), 0.0 if m2l_tol is None else float(m2l_tol),
                    int(far_field), 0 if eq_order is None else int(eq_order), 0 if leaves is None else int(leaves),
                    1 if fft_split else 0,
                    0 if overlap is None else (1 if overlap else 2),
                    0.0 if force_accuracy is None else float(force_accuracy),
                    0 if workspace_limit is None else int(workspace_limit))
    if stream is None:
        stream = torch.cuda.current_stream()
    h = ctypes.c_void_p()
    _check(L.ankh_plan(ctypes.byref(h), int(n_atoms), float(box_radius), float(rel_accuracy), int(max_order),
                       int(precision), ctypes.byref(ov), ctypes.c_void_p(stream.cuda_stream)), "ankh_plan")
    return h


def ankh_energy(plan, pos, q, mu, theta, energy):
    _check(load_library().ankh_energy(plan, pos, q, mu, theta, energy), "ankh_energy")


def ankh_energy_forces(plan, pos, q, mu, theta, energy, forces, dE_dmu):
    _check(load_library().ankh_energy_forces(plan, pos, q, mu, theta, energy, forces, dE_dmu), "ankh_energy_forces")


def ankh_energy_derivs(plan, pos, q, mu, theta, energy, forces, dE_dmu, dE_dq, dE_dtheta):
    _check(load_library().ankh_energy_derivs(plan, pos, q, mu, theta, energy, forces, dE_dmu, dE_dq, dE_dtheta),
           "ankh_energy_derivs")


def ankh_energy_derivs_noalloc(plan, pos, q, mu, theta, energy, forces, dE_dmu, dE_dq, dE_dtheta):
    _check(load_library().ankh_energy_derivs_noalloc(plan, pos, q, mu, theta, energy, forces, dE_dmu, dE_dq,
                                                      dE_dtheta), "ankh_energy_derivs_noalloc")


def ankh_energy_octupole(plan, pos, q, mu, theta, omega, energy, forces, dE_dmu):
    _check(load_library().ankh_energy_octupole(plan, pos, q, mu, theta, omega, energy, forces, dE_dmu),
           "ankh_energy_octupole")


def ankh_induce(plan, pos, q, mu, theta, alpha, tol, max_iter, mu_ind, energy, forces):
    """Returns (status, iterations, rel_residual); raises on every status but ANKH_ERR_NOT_CONVERGED (8)."""
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    st = load_library().ankh_induce(plan, pos, q, mu, theta, alpha, float(tol), int(max_iter), mu_ind, energy,
                                    forces, ctypes.byref(it), ctypes.byref(res))
    if st not in (0, 8):
        raise AnkhError(st, "ankh_induce")
    return st, it.value, res.value


def ankh_sync(plan):
    _check(load_library().ankh_sync(plan), "ankh_sync")


def ankh_get_stats(plan) -> dict:
    s = _Stats()
    _check(load_library().ankh_get_stats(plan, ctypes.byref(s)), "ankh_get_stats")
    d = {f: getattr(s, f) for f, _ in _Stats._fields_ if f not in ("stage_ms", "m2l_rank")}
    d["m2l_rank"] = [s.m2l_rank[i] for i in range(8)]
    d["stage_ms"] = {STAGES[i]: s.stage_ms[i] for i in range(len(STAGES))}
    return d


def ankh_set_timing(plan, enable):
    """enable: False / 0 off, True / 1 every stage boundary, 2 around the M2L and pair-kernel stages only."""
    _check(load_library().ankh_set_timing(plan, int(enable)), "ankh_set_timing")


def ankh_last_terms(plan) -> dict:
    buf = (ctypes.c_double * 7)()
    _check(load_library().ankh_last_terms(plan, buf), "ankh_last_terms")
    keys = ["near", "far_levels", "periodic", "self", "background", "total", "charge"]
    return {k: buf[i] for i, k in enumerate(keys)}


def ankh_leaf_multipoles(plan, count: int):
    import numpy as np
    out = np.zeros(count)
    _check(load_library().ankh_leaf_multipoles(plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), count),
           "ankh_leaf_multipoles")
    return out


def ankh_destroy(plan):
    if plan is not None and plan.value:
        load_library().ankh_destroy(plan)


def ankh_status_string(status: int) -> str:
    return load_library().ankh_status_string(int(status)).decode()


# ---- convenience wrapper ----------------------------------------------------------

class Plan:
    """A plan for n atoms in a cubic box of half-edge box_radius (see ankh.h)."""

    def __init__(self, n_atoms, box_radius, rel_accuracy=1e-6, max_order=2, precision="fp64", depth=None,
                 order=None, images=None, xi=None, root_order=None, m2l_tol=None, stream=None, far="auto",
                 eq_order=None, overlap=None, fft_split=False, leaves=None, force_accuracy=None,
                 workspace_limit=None):
        prec = ({"fp64": ANKH_FP64, "mixed": ANKH_MIXED, "mixed_bf16x3": ANKH_MIXED_BF16X3}[precision]
                if isinstance(precision, str) else int(precision))
        far_field = ({"auto": ANKH_FAR_AUTO, "fmm": ANKH_FAR_FMM, "fft": ANKH_FAR_FFT}[far]
                     if isinstance(far, str) else int(far))
        self.n = int(n_atoms)
        self.max_order = int(max_order)
        self.handle = ankh_plan(n_atoms, box_radius, rel_accuracy, max_order, prec, depth, order, images, xi,
                                root_order, m2l_tol, stream, far_field, eq_order, overlap, fft_split, leaves,
                                force_accuracy, workspace_limit)
        self.stats = ankh_get_stats(self.handle)

    def _args(self, pos, q, mu, theta):
        n = self.n
        pos, pp = _dev(pos, 3, n, "pos")
        q, qp = _dev(q, 1, n, "q")
        mu, mp = _dev(mu, 3, n, "mu", optional=True)
        theta, tp = _dev(theta, 6, n, "theta", optional=True)
        return (pos, q, mu, theta), (pp, qp, mp, tp)

    def energy(self, pos, q, mu=None, theta=None):
        keep, (pp, qp, mp, tp) = self._args(pos, q, mu, theta)
        e = torch.empty(1, dtype=torch.float64, device=pos.device)
        ankh_energy(self.handle, pp, qp, mp, tp, ctypes.c_void_p(e.data_ptr()))
        return e

    def energy_forces(self, pos, q, mu=None, theta=None, fields=True):
        keep, (pp, qp, mp, tp) = self._args(pos, q, mu, theta)
        e = torch.empty(1, dtype=torch.float64, device=pos.device)
        F = torch.empty((self.n, 3), dtype=torch.float64, device=pos.device)
        G = torch.empty((self.n, 3), dtype=torch.float64, device=pos.device) if fields else None
        ankh_energy_forces(self.handle, pp, qp, mp, tp, ctypes.c_void_p(e.data_ptr()),
                           ctypes.c_void_p(F.data_ptr()), None if G is None else ctypes.c_void_p(G.data_ptr()))
        return e, F, G

    def energy_octupole(self, pos, q, mu, theta, omega, forces=True, fields=True):
        """Energy (and forces / fields) with octupoles omega [n][10] (xxx, xxy, xxz, xyy, xyz, xzz, yyy, yyz,
        yzz, zzz); the plan needs max_order 3.  Returns (energy [1], forces or None, dE/dmu or None)."""
        keep, (pp, qp, mp, tp) = self._args(pos, q, mu, theta)
        omega, op = _dev(omega, 10, self.n, "omega")
        dev = pos.device
        e = torch.empty(1, dtype=torch.float64, device=dev)
        F = torch.empty((self.n, 3), dtype=torch.float64, device=dev) if forces else None
        G = torch.empty((self.n, 3), dtype=torch.float64, device=dev) if fields else None
        ankh_energy_octupole(self.handle, pp, qp, mp, tp, op, ctypes.c_void_p(e.data_ptr()),
                             None if F is None else ctypes.c_void_p(F.data_ptr()),
                             None if G is None else ctypes.c_void_p(G.data_ptr()))
        return e, F, G

    def energy_derivs(self, pos, q, mu=None, theta=None, forces=True, fields=True, potentials=True,
                      theta_grad=True, noalloc=False):
        """Energy and the requested derivatives (see ankh_energy_derivs in ankh.h): a dict with "energy"
        and, as asked, "forces" -dE/dx, "dEdmu", "dEdq" [n] and "dEdtheta" [n][6].  noalloc: through
        ankh_energy_derivs_noalloc (the library allocates nothing in the call; the output tensors are still
        allocated here, by torch)."""
        keep, (pp, qp, mp, tp) = self._args(pos, q, mu, theta)
        dev = pos.device
        out = {"energy": torch.empty(1, dtype=torch.float64, device=dev)}
        if forces:
            out["forces"] = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        if fields:
            out["dEdmu"] = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        if potentials:
            out["dEdq"] = torch.empty(self.n, dtype=torch.float64, device=dev)
        if theta_grad:
            out["dEdtheta"] = torch.empty((self.n, 6), dtype=torch.float64, device=dev)
        ptr = lambda k: ctypes.c_void_p(out[k].data_ptr()) if k in out else None
        fn = ankh_energy_derivs_noalloc if noalloc else ankh_energy_derivs
        fn(self.handle, pp, qp, mp, tp, ptr("energy"), ptr("forces"), ptr("dEdmu"), ptr("dEdq"), ptr("dEdtheta"))
        return out

    def induce(self, pos, q, mu, theta, alpha, tol=1e-8, max_iter=100, energy=True, forces=False,
               check=True):
        """Induced dipoles of the polarisabilities alpha [n] (see ankh_induce in ankh.h).  Returns
        (mu_ind, U or None, forces or None, iterations, rel_residual).  With check, raises AnkhError
        if the tolerance was not reached and reports latched input errors (one ankh_sync)."""
        keep, (pp, qp, mp, tp) = self._args(pos, q, mu, theta)
        alpha, ap = _dev(alpha, 1, self.n, "alpha")
        mi = torch.empty((self.n, 3), dtype=torch.float64, device=pos.device)
        e = torch.empty(1, dtype=torch.float64, device=pos.device) if energy else None
        F = torch.empty((self.n, 3), dtype=torch.float64, device=pos.device) if forces else None
        st, it, res = ankh_induce(self.handle, pp, qp, mp, tp, ap, tol, max_iter, ctypes.c_void_p(mi.data_ptr()),
                                  None if e is None else ctypes.c_void_p(e.data_ptr()),
                                  None if F is None else ctypes.c_void_p(F.data_ptr()))
        if check:
            ankh_sync(self.handle)
            if st != 0:
                raise AnkhError(st, f"ankh_induce ({it} iterations, residual {res:.3g})")
        return mi, e, F, it, res

    def sync(self):
        ankh_sync(self.handle)

    def get_stats(self):
        return ankh_get_stats(self.handle)

    def set_timing(self, on=True):
        ankh_set_timing(self.handle, on)

    def last_terms(self):
        return ankh_last_terms(self.handle)

    def leaf_multipoles(self):
        s = self.stats
        nleaf = 8 ** s["depth"]
        nu = s["order"] ** 3
        return ankh_leaf_multipoles(self.handle, nleaf * nu).reshape(nleaf, nu)

    def close(self):
        if getattr(self, "handle", None) is not None:
            ankh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AnkhEnergy(torch.autograd.Function):
    """E(pos, q, mu, theta) with the hand-written adjoint: dE/dpos = -F, dE/dmu = the fields, and, when q or
    theta require a gradient, dE/dq (site potentials) and the traceless dE/dTheta from ankh_energy_derivs."""

    @staticmethod
    def forward(ctx, pos, q, mu, theta, plan: Plan):
        want_q = ctx.needs_input_grad[1]
        want_th = theta is not None and ctx.needs_input_grad[3]
        ctx.has_mu = mu is not None
        ctx.want_q, ctx.want_th = want_q, want_th
        args = (pos.detach(), q.detach(), None if mu is None else mu.detach(),
                None if theta is None else theta.detach())
        if want_q or want_th:
            out = plan.energy_derivs(*args, fields=ctx.has_mu, potentials=want_q, theta_grad=want_th)
            F = out["forces"]
            G = out.get("dEdmu")
            ctx.save_for_backward(F, G if G is not None else F.new_zeros(0),
                                  out["dEdq"] if want_q else F.new_zeros(0),
                                  out["dEdtheta"] if want_th else F.new_zeros(0))
            return out["energy"][0]
        e, F, G = plan.energy_forces(*args, fields=ctx.has_mu)
        ctx.save_for_backward(F, G if G is not None else F.new_zeros(0), F.new_zeros(0), F.new_zeros(0))
        return e[0]

    @staticmethod
    def backward(ctx, g):
        F, G, dq, dth = ctx.saved_tensors
        dpos = -g * F
        dmu = g * G if ctx.has_mu else None
        return dpos, (g * dq if ctx.want_q else None), dmu, (g * dth if ctx.want_th else None), None


def energy(pos, q, mu=None, theta=None, plan: Plan | None = None):
    """Differentiable energy in the positions, charges, dipoles and quadrupoles."""
    if plan is None:
        raise ValueError("energy() needs a Plan")
    return AnkhEnergy.apply(pos, q, mu, theta, plan)
