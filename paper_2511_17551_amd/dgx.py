"""ctypes binding of libdgx (include/dgx.h): argument marshalling only.

Every function here has the name of the C entry point it calls and performs
no arithmetic of the method: the right-hand side, time stepping,
thermochemistry and surrogate all run in the HIP kernels of libdgx.so.  The
library must be built (``python -m paper_2511_17551_amd.build``); importing
this module on a machine without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgx.so")

DGX_OK = 0
ERRORS = {-1: "DGX_E_INVAL", -2: "DGX_E_NOMEM", -3: "DGX_E_DEVICE", -4: "DGX_E_NONPHYSICAL",
          -5: "DGX_E_NOCONV", -6: "DGX_E_STATE"}
GUESS_FREESTREAM = 0
GUESS_SURROGATE = 1
SUR_PARAMS = 64 * 6 + 64 + 2 * (64 * 64 + 64) + 64 + 1
SUR_NORM = 14


class DgxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (ERRORS.get(code, code), msg))
        self.code = code


class dgx_species(C.Structure):
    _fields_ = [("nspecies", C.c_int), ("molecule", C.c_int * 5), ("W", C.c_double * 5),
                ("theta_v", C.c_double * 5), ("theta_r", C.c_double * 5), ("sigma", C.c_double * 5),
                ("Qe", C.c_double * 5), ("e0", C.c_double * 5), ("Ru", C.c_double), ("NA", C.c_double),
                ("hP", C.c_double), ("p_ref", C.c_double)]


class dgx_reactions(C.Structure):
    _fields_ = [("nreactions", C.c_int), ("A", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)),
                ("theta_a", C.POINTER(C.c_double)), ("nu", C.POINTER(C.c_int32)),
                ("nup", C.POINTER(C.c_int32))]


class dgx_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("N", C.c_int), ("equation", C.c_int), ("volume_flux", C.c_int),
                ("surface_flux", C.c_int), ("gamma", C.c_double), ("R", C.c_double), ("mu", C.c_double),
                ("Pr", C.c_double), ("shock", C.c_int), ("alpha_max", C.c_double), ("alpha_min", C.c_double),
                ("ind_var", C.c_int), ("alpha_smooth", C.c_int), ("force_alpha", C.c_double),
                ("newton_tol", C.c_double), ("newton_maxit", C.c_int), ("T_guess", C.c_double),
                ("positivity", C.c_int),
                ("species", C.POINTER(dgx_species)), ("reactions", C.POINTER(dgx_reactions)),
                ("sutherland_S", C.c_double), ("sutherland_T0", C.c_double)]


class dgx_mesh(C.Structure):
    _fields_ = [("nelem", C.c_int), ("x", C.POINTER(C.c_double)), ("nface", C.c_int),
                ("faces", C.POINTER(C.c_int32)), ("nbface", C.c_int), ("bfaces", C.POINTER(C.c_int32)),
                ("nmortar", C.c_int), ("mortars", C.POINTER(C.c_int32)), ("nbc", C.c_int),
                ("bc_kind", C.POINTER(C.c_int32)), ("bc_state", C.POINTER(C.c_double))]


class dgx_amr_controller(C.Structure):
    _fields_ = [("base_level", C.c_int), ("med_level", C.c_int), ("max_level", C.c_int),
                ("med_threshold", C.c_double), ("max_threshold", C.c_double)]


class dgx_newton_stats(C.Structure):
    _fields_ = [("nodes", C.c_int64), ("iters_total", C.c_int64), ("iters_max", C.c_int32),
                ("iters_wave_max_mean", C.c_double), ("nonconverged", C.c_int64), ("first_bad", C.c_int64),
                ("substeps_total", C.c_int64), ("substeps_max", C.c_int32), ("fallbacks", C.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdgx.so is not built (run python -m paper_2511_17551_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    sig = {
        "dgx_create": ([C.POINTER(dgx_config), C.POINTER(vp)], C.c_int),
        "dgx_set_mesh": ([vp, C.POINTER(dgx_mesh)], C.c_int),
        "dgx_rhs": ([vp, vp, C.c_double, vp, vp], C.c_int),
        "dgx_ssprk3_step": ([vp, vp, C.c_double, C.c_double, C.c_int, vp], C.c_int),
        "dgx_limit_positivity": ([vp, vp, vp], C.c_int),
        "dgx_max_dt": ([vp, vp, C.c_double, C.POINTER(C.c_double), vp], C.c_int),
        "dgx_thermo": ([vp, vp, C.c_int64, vp, vp, C.c_int, C.POINTER(dgx_newton_stats), vp], C.c_int),
        "dgx_thermo_noalloc": ([vp, vp, C.c_int64, vp, vp, C.c_int, C.POINTER(dgx_newton_stats), vp], C.c_int),
        "dgx_chem_step": ([vp, vp, C.c_double, C.c_double, C.c_int, C.POINTER(dgx_newton_stats), vp], C.c_int),
        "dgx_last_alpha": ([vp], vp),
        "dgx_surrogate_set": ([vp, C.POINTER(C.c_float), C.c_size_t], C.c_int),
        "dgx_surrogate_get": ([vp, C.POINTER(C.c_float), C.c_size_t], C.c_int),
        "dgx_surrogate_train": ([vp, vp, vp, C.c_int64, C.c_int, C.c_int, C.c_float, C.c_uint64,
                                 C.POINTER(C.c_float), vp], C.c_int),
        "dgx_surrogate_predict": ([vp, vp, C.c_int64, vp, vp], C.c_int),
        "dgx_surrogate_init": ([vp, vp, vp, C.c_int64, C.c_uint64, vp], C.c_int),
        "dgx_surrogate_grad": ([vp, vp, vp, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float), vp], C.c_int),
        "dgx_check": ([vp, vp], C.c_int),
        "dgx_species_energy": ([vp, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
        "dgx_mixture_energy": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int64,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)], C.c_int),
        "dgx_kernel_times": ([vp, vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_char_p,
                              C.c_size_t, vp], C.c_int),
        "dgx_autotune": ([vp, vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), vp], C.c_int),
        "dgx_set_launch": ([vp, C.c_int, C.c_int], C.c_int),
        "dgx_get_launch": ([vp, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "dgx_set_octree": ([vp, C.c_int, C.c_int, C.POINTER(C.c_int32)], C.c_int),
        "dgx_get_octree": ([vp, C.POINTER(C.c_int32), C.c_int], C.c_int),
        "dgx_amr_indicator": ([vp, vp, C.c_int, C.c_int, vp, vp], C.c_int),
        "dgx_amr_plan": ([vp, C.POINTER(C.c_double), C.POINTER(dgx_amr_controller), C.POINTER(C.c_int)], C.c_int),
        "dgx_amr_apply": ([vp, vp, vp, vp], C.c_int),
        "dgx_last_error": ([vp], C.c_char_p),
        "dgx_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()
EXPORTED = ("dgx_create", "dgx_set_mesh", "dgx_rhs", "dgx_ssprk3_step", "dgx_limit_positivity", "dgx_max_dt", "dgx_thermo",
            "dgx_thermo_noalloc",
            "dgx_chem_step",
            "dgx_last_alpha", "dgx_surrogate_set", "dgx_surrogate_get", "dgx_surrogate_train",
            "dgx_surrogate_predict", "dgx_surrogate_init", "dgx_surrogate_grad", "dgx_check", "dgx_species_energy", "dgx_mixture_energy", "dgx_kernel_times", "dgx_autotune",
            "dgx_set_launch", "dgx_get_launch", "dgx_set_octree", "dgx_get_octree", "dgx_amr_indicator",
            "dgx_amr_plan", "dgx_amr_apply", "dgx_last_error", "dgx_destroy")


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


def _dev(t):
    """Device pointer of a torch tensor (must be contiguous)."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(int(stream))


def _raise(ctx, rc):
    if rc != DGX_OK:
        msg = lib.dgx_last_error(ctx).decode() if ctx else ""
        raise DgxError(rc, msg)


def make_species(sp):
    s = dgx_species()
    s.nspecies = 5
    for i in range(5):
        s.molecule[i] = int(sp.molecule[i])
        s.W[i] = sp.W[i]
        s.theta_v[i] = sp.theta_v[i]
        s.theta_r[i] = sp.theta_r[i]
        s.sigma[i] = sp.sigma[i]
        s.Qe[i] = sp.Qe[i]
        s.e0[i] = sp.e0[i]
    s.Ru, s.NA, s.hP, s.p_ref = sp.Ru, sp.NA, sp.hP, sp.p_ref
    return s


class _Keep:
    """Holds ctypes objects alive while the C side copies them."""


_LIVE = set()   # contexts created and not yet destroyed (host-side guard)


def dgx_create(cfg: dict, species=None, reactions=None):
    keep = _Keep()
    c = dgx_config()
    c.dim, c.N, c.equation = cfg["dim"], cfg["N"], cfg["eq"]
    c.volume_flux, c.surface_flux = cfg["volume_flux"], cfg["surface_flux"]
    c.gamma, c.R, c.mu, c.Pr = cfg["gamma"], cfg["R"], cfg["mu"], cfg["Pr"]
    c.shock = int(bool(cfg["shock"]))
    c.alpha_max, c.alpha_min = cfg["alpha_max"], cfg["alpha_min"]
    c.ind_var, c.alpha_smooth, c.force_alpha = cfg["ind_var"], int(bool(cfg["alpha_smooth"])), cfg["force_alpha"]
    c.newton_tol, c.newton_maxit, c.T_guess = cfg["newton_tol"], cfg["newton_maxit"], cfg["T_guess"]
    c.positivity = int(bool(cfg.get("positivity", False)))
    c.sutherland_S, c.sutherland_T0 = cfg.get("sutherland_S", 0.0), cfg.get("sutherland_T0", 1.0)
    if species is not None:
        keep.sp = make_species(species)
        c.species = C.pointer(keep.sp)
    if reactions is not None:
        r = dgx_reactions()
        keep.A = np.ascontiguousarray(reactions.A, np.float64)
        keep.b = np.ascontiguousarray(reactions.b, np.float64)
        keep.th = np.ascontiguousarray(reactions.theta_a, np.float64)
        keep.nu = np.ascontiguousarray(reactions.nu, np.int32)
        keep.nup = np.ascontiguousarray(reactions.nup, np.int32)
        r.nreactions = keep.A.shape[0]
        r.A, r.b, r.theta_a = _ptr(keep.A), _ptr(keep.b), _ptr(keep.th)
        r.nu, r.nup = _ptr(keep.nu, C.c_int32), _ptr(keep.nup, C.c_int32)
        keep.r = r
        c.reactions = C.pointer(keep.r)
    h = C.c_void_p()
    rc = lib.dgx_create(C.byref(c), C.byref(h))
    if rc != DGX_OK:
        raise DgxError(rc, "dgx_create rejected the configuration")
    _LIVE.add(h.value)
    return h


def dgx_set_mesh(ctx, mesh):
    x = np.ascontiguousarray(mesh.x, np.float64)
    faces = np.ascontiguousarray(mesh.faces, np.int32)
    bfaces = np.ascontiguousarray(mesh.bfaces, np.int32)
    mort = np.ascontiguousarray(mesh.mortars, np.int32)
    kind = np.ascontiguousarray(mesh.bc_kind, np.int32)
    state = np.ascontiguousarray(mesh.bc_state, np.float64)
    m = dgx_mesh()
    m.nelem = x.shape[1]
    m.x = _ptr(x)
    m.nface, m.faces = faces.shape[0], _ptr(faces, C.c_int32)
    m.nbface, m.bfaces = bfaces.shape[0], _ptr(bfaces, C.c_int32)
    m.nmortar, m.mortars = mort.shape[0], _ptr(mort, C.c_int32)
    m.nbc, m.bc_kind, m.bc_state = kind.shape[0], _ptr(kind, C.c_int32), _ptr(state)
    _raise(ctx, lib.dgx_set_mesh(ctx, C.byref(m)))


def dgx_set_octree(ctx, base, leaves):
    lv = np.ascontiguousarray(leaves, np.int32).reshape(-1, 4)
    _raise(ctx, lib.dgx_set_octree(ctx, int(base), lv.shape[0], _ptr(lv, C.c_int32)))


def dgx_get_octree(ctx):
    n = lib.dgx_get_octree(ctx, None, 0)
    if n < 0:
        _raise(ctx, n)
    out = np.empty((n, 4), np.int32)
    rc = lib.dgx_get_octree(ctx, _ptr(out, C.c_int32), n)
    if rc < 0:
        _raise(ctx, rc)
    return out


def dgx_amr_indicator(ctx, u, kind, variable, ind, stream=None):
    _raise(ctx, lib.dgx_amr_indicator(ctx, _dev(u), int(kind), int(variable), _dev(ind), _stream(stream)))


def dgx_amr_plan(ctx, ind, controller):
    ind = np.ascontiguousarray(ind, np.float64)
    c = dgx_amr_controller(*[int(controller[k]) for k in ("base_level", "med_level", "max_level")],
                           float(controller["med_threshold"]), float(controller["max_threshold"]))
    n = C.c_int()
    _raise(ctx, lib.dgx_amr_plan(ctx, _ptr(ind), C.byref(c), C.byref(n)))
    return n.value


def dgx_amr_apply(ctx, u_old, u_new, stream=None):
    _raise(ctx, lib.dgx_amr_apply(ctx, _dev(u_old), _dev(u_new), _stream(stream)))


def dgx_rhs(ctx, u, t, du, stream=None):
    _raise(ctx, lib.dgx_rhs(ctx, _dev(u), float(t), _dev(du), _stream(stream)))


def dgx_ssprk3_step(ctx, u, t, dt, nsteps, stream=None):
    _raise(ctx, lib.dgx_ssprk3_step(ctx, _dev(u), float(t), float(dt), int(nsteps), _stream(stream)))


def dgx_limit_positivity(ctx, u, stream=None):
    _raise(ctx, lib.dgx_limit_positivity(ctx, _dev(u), _stream(stream)))


def dgx_max_dt(ctx, u, cfl, stream=None):
    out = C.c_double()
    _raise(ctx, lib.dgx_max_dt(ctx, _dev(u), float(cfl), C.byref(out), _stream(stream)))
    return out.value


def dgx_thermo(ctx, u, T, p=None, guess=GUESS_FREESTREAM, nstates=0, stream=None, check=True, stats=True):
    if not stats:
        _raise(ctx, lib.dgx_thermo(ctx, _dev(u), int(nstates), _dev(T), _dev(p), int(guess), None,
                                   _stream(stream)))
        return None
    st = dgx_newton_stats()
    rc = lib.dgx_thermo(ctx, _dev(u), int(nstates), _dev(T), _dev(p), int(guess), C.byref(st), _stream(stream))
    if check:
        _raise(ctx, rc)
    return dict(nodes=st.nodes, iters_total=st.iters_total, iters_max=st.iters_max,
                iters_wave_max_mean=st.iters_wave_max_mean, nonconverged=st.nonconverged,
                first_bad=st.first_bad, fallbacks=st.fallbacks, rc=rc)


NOALLOC_MAX_STATES = 1048576


def dgx_thermo_noalloc(ctx, u, T, p=None, guess=GUESS_FREESTREAM, nstates=0, stream=None, check=True, stats=True):
    """dgx_thermo with its scratch in the library's static device buffer (no
    allocation; at most NOALLOC_MAX_STATES states)."""
    if not stats:
        _raise(ctx, lib.dgx_thermo_noalloc(ctx, _dev(u), int(nstates), _dev(T), _dev(p), int(guess), None,
                                           _stream(stream)))
        return None
    st = dgx_newton_stats()
    rc = lib.dgx_thermo_noalloc(ctx, _dev(u), int(nstates), _dev(T), _dev(p), int(guess), C.byref(st),
                                _stream(stream))
    if check:
        _raise(ctx, rc)
    return dict(nodes=st.nodes, iters_total=st.iters_total, iters_max=st.iters_max,
                iters_wave_max_mean=st.iters_wave_max_mean, nonconverged=st.nonconverged,
                first_bad=st.first_bad, fallbacks=st.fallbacks, rc=rc)


def dgx_chem_step(ctx, u, dt, tol=1e-13, maxit=50, stream=None, check=True, stats=True):
    """Backward-Euler chemistry over dt (substeps where the single step
    fails) in place on u's species rows."""
    if not stats:
        _raise(ctx, lib.dgx_chem_step(ctx, _dev(u), float(dt), float(tol), int(maxit), None, _stream(stream)))
        return None
    st = dgx_newton_stats()
    rc = lib.dgx_chem_step(ctx, _dev(u), float(dt), float(tol), int(maxit), C.byref(st), _stream(stream))
    if check:
        _raise(ctx, rc)
    return dict(nodes=st.nodes, iters_total=st.iters_total, iters_max=st.iters_max,
                iters_wave_max_mean=st.iters_wave_max_mean, nonconverged=st.nonconverged,
                first_bad=st.first_bad, substeps_total=st.substeps_total, substeps_max=st.substeps_max, rc=rc)


def dgx_last_alpha(ctx, nelem):
    """Copy of the last blending factors (torch tensor), or None."""
    import torch
    p = lib.dgx_last_alpha(ctx)
    if not p:
        return None
    out = torch.empty(nelem, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    _copy_device(out, p, nelem * 8)
    return out


def _copy_device(dst, src_ptr, nbytes):
    """Copy nbytes from a library-owned device pointer into a torch tensor."""
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipMemcpy.restype = C.c_int
    rc = hip.hipMemcpy(C.c_void_p(dst.data_ptr()), C.c_void_p(src_ptr), nbytes, 3)
    if rc != 0:
        raise DgxError(-3, "hipMemcpy failed")


def dgx_surrogate_set(ctx, params):
    a = np.ascontiguousarray(params, np.float32)
    _raise(ctx, lib.dgx_surrogate_set(ctx, _ptr(a, C.c_float), a.size))


def dgx_surrogate_get(ctx):
    a = np.zeros(SUR_PARAMS + SUR_NORM, np.float32)
    _raise(ctx, lib.dgx_surrogate_get(ctx, _ptr(a, C.c_float), a.size))
    return a


def dgx_surrogate_train(ctx, states, T, epochs, batch, lr, seed=42, stream=None):
    count = T.shape[0]
    loss = np.zeros(epochs, np.float32)
    _raise(ctx, lib.dgx_surrogate_train(ctx, _dev(states), _dev(T), count, epochs, batch, lr, seed,
                                        _ptr(loss, C.c_float), _stream(stream)))
    return loss


def dgx_surrogate_init(ctx, states, T, seed=41, stream=None):
    _raise(ctx, lib.dgx_surrogate_init(ctx, _dev(states), _dev(T), T.shape[0], int(seed), _stream(stream)))


def dgx_surrogate_grad(ctx, states, T, stream=None):
    g = np.zeros(SUR_PARAMS, np.float32)
    loss = C.c_float()
    _raise(ctx, lib.dgx_surrogate_grad(ctx, _dev(states), _dev(T), T.shape[0], _ptr(g, C.c_float), C.byref(loss),
                                       _stream(stream)))
    return g, loss.value


def dgx_surrogate_predict(ctx, states, Tg, stream=None):
    _raise(ctx, lib.dgx_surrogate_predict(ctx, _dev(states), Tg.shape[0], _dev(Tg), _stream(stream)))


def dgx_check(ctx, stream=None):
    _raise(ctx, lib.dgx_check(ctx, _stream(stream)))


def dgx_check_code(ctx, stream=None):
    return lib.dgx_check(ctx, _stream(stream))


def dgx_species_energy(ctx, T):
    e = (C.c_double * 5)()
    cv = (C.c_double * 5)()
    _raise(ctx, lib.dgx_species_energy(ctx, float(T), e, cv))
    return np.array(e[:]), np.array(cv[:])


def dgx_mixture_energy(ctx, rs, T):
    """(rho e, rho cv) of host states: rs (5, n), T (n,) -> two (n,) arrays."""
    rs = np.ascontiguousarray(rs, np.float64)
    T = np.ascontiguousarray(T, np.float64)
    n = T.shape[0]
    if rs.shape != (5, n):
        raise ValueError("rs must have shape (5, n)")
    rhoe = np.empty(n)
    rhocv = np.empty(n)
    _raise(ctx, lib.dgx_mixture_energy(ctx, _ptr(rs), _ptr(T), n, _ptr(rhoe), _ptr(rhocv)))
    return rhoe, rhocv


def dgx_kernel_times(ctx, u, reps=20, stream=None):
    """{kernel name: average ms} of one fused-stage right-hand side."""
    ms = (C.c_double * 8)()
    nk = C.c_int()
    names = C.create_string_buffer(256)
    _raise(ctx, lib.dgx_kernel_times(ctx, _dev(u), int(reps), ms, C.byref(nk), names, 256, _stream(stream)))
    return dict(zip(names.value.decode().split(","), ms[:nk.value]))


def dgx_autotune(ctx, u, reps=10, stream=None):
    """Returns (chosen elements per workgroup, {candidate: ms})."""
    epb = C.c_int()
    ms = (C.c_double * 4)()
    _raise(ctx, lib.dgx_autotune(ctx, _dev(u), int(reps), C.byref(epb), ms, _stream(stream)))
    return epb.value, {c: ms[i] for i, c in enumerate((1, 2, 4, 8)) if ms[i] >= 0}


def dgx_set_launch(ctx, epb, order=-1):
    """Elements per workgroup and launch form (0 round-robin over the XCDs,
    1 XCD-contiguous, 2 work-list queue, -1 keep)."""
    _raise(ctx, lib.dgx_set_launch(ctx, int(epb), int(order)))


def dgx_get_launch(ctx):
    """(elements per workgroup, launch form 0/1/2) in use."""
    epb, order = C.c_int(), C.c_int()
    _raise(ctx, lib.dgx_get_launch(ctx, C.byref(epb), C.byref(order)))
    return epb.value, order.value


def dgx_last_error(ctx):
    return lib.dgx_last_error(ctx).decode()


def dgx_destroy(ctx):
    _LIVE.discard(ctx.value if isinstance(ctx, C.c_void_p) else ctx)
    lib.dgx_destroy(ctx)


class Solver:
    """A context bound to one workload (a ``workloads.Case``)."""

    def __init__(self, case):
        self.case = case
        self.ctx = dgx_create(case.cfg, case.species, case.reactions)
        try:
            dgx_set_mesh(self.ctx, case.mesh)
        except Exception:
            dgx_destroy(self.ctx)
            raise
        self.shape = (case.cfg["nvar"], case.mesh.nelem, case.mesh.nnodes)

    def rhs(self, u, du=None, t=0.0):
        import torch
        if du is None:
            du = torch.empty_like(u)
        dgx_rhs(self.ctx, u, t, du)
        return du

    def ssprk3(self, u, dt, nsteps, t=0.0):
        dgx_ssprk3_step(self.ctx, u, t, dt, nsteps)
        return u

    def check(self):
        dgx_check(self.ctx)

    # dynamic AMR (octree meshes)
    def set_octree(self, base, leaves):
        """Replace the mesh by the octree's; returns the leaves in element order."""
        dgx_set_octree(self.ctx, base, leaves)
        return self.octree()

    def octree(self):
        return dgx_get_octree(self.ctx)

    def amr_indicator(self, u, kind, variable):
        import torch
        ind = torch.empty(u.shape[1], dtype=torch.float64, device=u.device)
        dgx_amr_indicator(self.ctx, u, kind, variable, ind)
        return ind

    def amr_adapt(self, u, ind, controller):
        """One adaptation pass from host indicator values; returns the state
        on the new mesh (a new tensor)."""
        import torch
        n = dgx_amr_plan(self.ctx, ind, controller)
        out = torch.empty((u.shape[0], n, u.shape[2]), dtype=u.dtype, device=u.device)
        dgx_amr_apply(self.ctx, u, out)
        return out

    def close(self):
        if self.ctx:
            dgx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mixture_energy_fns(ctx):
    """energy(rho_s, T), cv(rho_s, T) from dgx_mixture_energy (used to build
    mixture states when the oracle is not involved): the arrays are broadcast
    to one shape, flattened to (5, n) and (n,), and the library's results
    reshaped back."""
    def make(which):
        def fn(rs, T):
            if (ctx.value if isinstance(ctx, C.c_void_p) else ctx) not in _LIVE:
                raise RuntimeError("mixture energy functions used after their context was destroyed")
            rs = np.asarray(rs, float)
            T = np.asarray(T, float)
            shape = np.broadcast_shapes(rs.shape[1:], T.shape)
            rsb = np.broadcast_to(rs, (rs.shape[0],) + shape).reshape(rs.shape[0], -1)
            Tb = np.broadcast_to(T, shape).reshape(-1)
            return dgx_mixture_energy(ctx, rsb, Tb)[which].reshape(shape)
        return fn
    return make(0), make(1)
