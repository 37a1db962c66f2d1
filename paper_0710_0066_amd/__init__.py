"""Python binding of libsapmi (include/sapmi.h): argument marshalling only.

Every operator, solve, force and trajectory runs in the library's HIP kernels on the
current HIP device; PyTorch only allocates device memory and supplies the stream. There
is no CPU fallback: if the shared library has not been built this module raises on
import.

The module-level functions carry the C names (apply_M, apply_W1_block, solve_full,
solve_blocks, block_pf_force, schwarz_boundary_force, gauge_force, hmc_trajectory,
sap_*); ``Context`` wraps a ``sap_ctx*`` and allocates fields with torch.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libsapmi.so")

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python paper_0710_0066_amd/build.py`")

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7) as the system
# one this library links against, and the first copy loaded serves the whole process.
# torch only works with its own copy (loading this library first leaves torch with "No HIP
# GPUs are available"), so torch is imported before the library is loaded.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(_LIB_PATH)

SAP_OK, SAP_E_ARG, SAP_E_NOMEM, SAP_E_HIP, SAP_E_NOCONV, SAP_E_NONFINITE, SAP_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
SAP_F64, SAP_F32, SAP_F16 = 0, 1, 2   # FP16: half2 components with an FP32 norm per site
SAP_ALL, SAP_BLACK, SAP_WHITE = 0, 1, 2
_STATUS = {0: "SAP_OK", -1: "SAP_E_ARG", -2: "SAP_E_NOMEM", -3: "SAP_E_HIP", -4: "SAP_E_NOCONV",
           -5: "SAP_E_NONFINITE", -6: "SAP_E_STATE"}


class SapError(RuntimeError):
    def __init__(self, code, msg, info=None):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code
        self.info = info


class sap_geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("l0", ctypes.c_int), ("l0_sub", ctypes.c_int),
                ("kappa", ctypes.c_double), ("max_rhs", ctypes.c_int)]


class sap_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("inner_prec", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("method", ctypes.c_int),
                ("sap_ncy", ctypes.c_int), ("sap_block_terms", ctypes.c_int)]


class sap_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("true_rel_res", ctypes.c_double)]


class sap_hmc_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("tau", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("n_outer", ctypes.c_int), ("n_inner", ctypes.c_int),
                ("scheme_outer", ctypes.c_int), ("scheme_inner", ctypes.c_int),
                ("force_solve", sap_solve_opts), ("action_solve", sap_solve_opts),
                ("p0", ctypes.c_void_p), ("xi1", ctypes.c_void_p), ("xi2", ctypes.c_void_p),
                ("u_metropolis", ctypes.c_double), ("step_scale", ctypes.c_void_p),
                ("time_shift", ctypes.c_int)]


class sap_hmc4_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("tau", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("rho", ctypes.c_double), ("n", ctypes.c_int * 5), ("scheme", ctypes.c_int * 5),
                ("force_solve", sap_solve_opts), ("action_solve", sap_solve_opts),
                ("p0", ctypes.c_void_p), ("xi1", ctypes.c_void_p), ("xi2", ctypes.c_void_p),
                ("g3", ctypes.c_void_p), ("g4", ctypes.c_void_p), ("u_metropolis", ctypes.c_double),
                ("step_scale", ctypes.c_void_p), ("time_shift", ctypes.c_int),
                ("part_solve", ctypes.POINTER(sap_solve_opts))]


class sap_hmc4_info(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("H0", ctypes.c_double), ("H1", ctypes.c_double),
                ("S0", ctypes.c_double * 5), ("S1", ctypes.c_double * 5), ("plaq", ctypes.c_double),
                ("accepted", ctypes.c_int), ("solver_iters", ctypes.c_longlong)]


class sap_hmc_info(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("H0", ctypes.c_double), ("H1", ctypes.c_double),
                ("S_G0", ctypes.c_double), ("S_G1", ctypes.c_double),
                ("S_W0", ctypes.c_double), ("S_W1", ctypes.c_double),
                ("S_R0", ctypes.c_double), ("S_R1", ctypes.c_double),
                ("plaq", ctypes.c_double), ("accepted", ctypes.c_int),
                ("solver_iters", ctypes.c_longlong)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SIGS = {
    "sap_version": ([], _I),
    "sap_check_geom": ([ctypes.POINTER(sap_geom)], _I),
    "sap_create": ([ctypes.POINTER(sap_geom), ctypes.POINTER(_P)], _I),
    "sap_destroy": ([_P], None),
    "sap_last_error": ([_P], ctypes.c_char_p),
    "sap_field_bytes": ([_P, _I, _I], ctypes.c_size_t),
    "sap_momenta_bytes": ([_P], ctypes.c_size_t),
    "sap_set_gauge": ([_P, _P, _P], _I),
    "sap_get_gauge": ([_P, _P, _P], _I),
    "sap_pack_spinor": ([_P, _P, _P, _I, _I, _P], _I),
    "sap_unpack_spinor": ([_P, _P, _P, _I, _I, _P], _I),
    "sap_pack_momenta": ([_P, _P, _P, _P], _I),
    "sap_unpack_momenta": ([_P, _P, _P, _P], _I),
    "apply_M": ([_P, _P, _P, _I, _I, _P], _I),
    "apply_W1_block": ([_P, _P, _P, _I, _I, _I, _I, _I, _P], _I),
    "apply_Dslash_eo": ([_P, _P, _P, _I, _I, _I, _P], _I),
    "solve_full": ([_P, _P, _P, _I, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
    "solve_blocks": ([_P, _P, _P, _I, _I, _I, _I, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
    "block_pf_force": ([_P, _P, _D, _P, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
    "schwarz_boundary_force": ([_P, _P, _D, _P, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
    "gauge_force": ([_P, _P, _D, _D, _P, _P], _I),
    "schwarz_heat_bath": ([_P, _P, _P, ctypes.POINTER(sap_solve_opts), _P], _I),
    "schwarz_action": ([_P, _P, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
    "sap_update_links": ([_P, _P, _D, _P], _I),
    "sap_plaquette": ([_P, _P, _P], _I),
    "sap_shift_gauge": ([_P, _I, _P], _I),
    "sap_force_profile": ([_P, _P, _P, _P], _I),
    "sap_force_profile_noalloc": ([_P, _P, _P, _P], _I),
    "sap_force_profile_noalloc_max": ([], ctypes.c_size_t),
    "sap_stream_probe": ([_P, _P, ctypes.c_size_t, _I, _P], _I),
    "sap_stream_probe_blocks": ([], _I),
    "sap_tune": ([_P, _I, _P, _P], _I),
    "sap_set_hop_map": ([_P, _I, _I, _I, _I], _I),
    "hmc_trajectory": ([_P, _P, ctypes.POINTER(sap_hmc_params), ctypes.POINTER(sap_hmc_info), _P], _I),
    "hmc_trajectory_4pf": ([_P, _P, ctypes.POINTER(sap_hmc4_params), ctypes.POINTER(sap_hmc4_info), _P], _I),
    "eo_pf_heat_bath": ([_P, _P, _P, _I, _D, ctypes.POINTER(sap_solve_opts), _P], _I),
    "eo_pf_force": ([_P, _P, _D, _P, _I, _D, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
    "schwarz2_heat_bath": ([_P, _P, _P, ctypes.POINTER(sap_solve_opts), _P], _I),
    "schwarz2_force": ([_P, _P, _D, _P, ctypes.POINTER(sap_solve_opts), _P, _P], _I),
}
for _name, (_args, _ret) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _ret


def lib_path() -> str:
    return _LIB_PATH


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)



def _buf(ctx, t, nbytes, what, optional=False):
    """Device pointer of t after checking it: the library reads and writes through raw
    pointers, so the tensor must be a contiguous floating-point or complex tensor on the
    context's device holding at least nbytes (an undersized buffer would become an
    out-of-bounds device access). None gives NULL when optional, else SapError."""
    if t is None:
        if optional:
            return None
        raise SapError(SAP_E_ARG, f"{what} is None")
    import torch
    if not isinstance(t, torch.Tensor):
        raise SapError(SAP_E_ARG, f"{what}: expected a torch.Tensor, got {type(t).__name__}")
    if t.device.type != "cuda" or (ctx is not None and t.device.index != ctx.device):
        raise SapError(SAP_E_ARG, f"{what}: must live on the context's device cuda:{ctx.device if ctx else '?'}, "
                                  f"not {t.device}")
    if not (t.is_floating_point() or t.is_complex()):
        raise SapError(SAP_E_ARG, f"{what}: dtype {t.dtype} is not a floating-point or complex type")
    if not t.is_contiguous():
        raise SapError(SAP_E_ARG, f"{what}: must be contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise SapError(SAP_E_ARG, f"{what}: {have} bytes, the call needs {nbytes}")
    return ctypes.c_void_p(t.data_ptr())


def _field(ctx, t, nrhs, prec, what, optional=False):
    """A library-layout spinor field of nrhs right-hand sides at precision prec."""
    if not (isinstance(nrhs, int) and nrhs >= 1):
        raise SapError(SAP_E_ARG, f"nrhs must be a positive int, got {nrhs!r}")
    if prec not in (SAP_F64, SAP_F32, SAP_F16):
        raise SapError(SAP_E_ARG, f"unknown precision {prec!r}")
    return _buf(ctx, t, _lib.sap_field_bytes(ctx.ptr, prec, nrhs), what, optional)


def _mom(ctx, t, what, optional=False):
    """A library-layout momentum / force field."""
    return _buf(ctx, t, _lib.sap_momenta_bytes(ctx.ptr), what, optional)


def _check(ctx_ptr, rc, info=None):
    if rc != SAP_OK:
        msg = _lib.sap_last_error(ctx_ptr)
        raise SapError(rc, msg.decode() if msg else "", info)


def sap_version() -> int:
    return _lib.sap_version()


def sap_check_geom(L, l0, l0_sub=0, kappa=0.1, max_rhs=1) -> int:
    g = sap_geom((ctypes.c_int * 4)(*L), l0, l0_sub, kappa, max_rhs)
    return _lib.sap_check_geom(ctypes.byref(g))


SAP_CG, SAP_BICGSTAB, SAP_GEOM, SAP_SAP_BICGSTAB = 0, 1, 2, 3


def solve_opts(tol=1e-10, max_iter=100000, inner_prec=SAP_F32, inner_tol=1e-5, max_outer=50, method=SAP_CG,
               sap_ncy=1, sap_block_terms=0):
    return sap_solve_opts(tol, max_iter, inner_prec, inner_tol, max_outer, method, sap_ncy, sap_block_terms)


# ---- C entry points with their own names -------------------------------------------

def apply_M(ctx, out, inp, nrhs, prec):
    po, pi = _field(ctx, out, nrhs, prec, "out"), _field(ctx, inp, nrhs, prec, "in")
    _check(ctx.ptr, _lib.apply_M(ctx.ptr, po, pi, nrhs, prec, _stream()))


def apply_W1_block(ctx, out, inp, nrhs, level=1, block=-1, color=SAP_ALL, prec=SAP_F64):
    po, pi = _field(ctx, out, nrhs, prec, "out"), _field(ctx, inp, nrhs, prec, "in")
    _check(ctx.ptr, _lib.apply_W1_block(ctx.ptr, po, pi, nrhs, level, block, color, prec, _stream()))


def apply_Dslash_eo(ctx, out, inp, nrhs, parity, prec):
    po, pi = _field(ctx, out, nrhs, prec, "out"), _field(ctx, inp, nrhs, prec, "in")
    _check(ctx.ptr, _lib.apply_Dslash_eo(ctx.ptr, po, pi, nrhs, parity, prec, _stream()))


def solve_full(ctx, x, b, nrhs, opts):
    px, pb = _field(ctx, x, nrhs, SAP_F64, "x"), _field(ctx, b, nrhs, SAP_F64, "b")
    info = (sap_solve_info * nrhs)()
    rc = _lib.solve_full(ctx.ptr, px, pb, nrhs, ctypes.byref(opts), info, _stream())
    _check(ctx.ptr, rc, info)
    return list(info)


def solve_blocks(ctx, x, b, nrhs, level, color, opts, block=-1):
    if level not in (1, 2) or (level == 2 and not ctx.l0_sub):
        raise SapError(SAP_E_ARG, "level must be 1, or 2 with l0_sub set")
    px, pb = _field(ctx, x, nrhs, SAP_F64, "x"), _field(ctx, b, nrhs, SAP_F64, "b")
    nb = ctx.nblocks(level)
    info = (sap_solve_info * (nb * nrhs))()
    rc = _lib.solve_blocks(ctx.ptr, px, pb, nrhs, level, color, block, ctypes.byref(opts), info, _stream())
    _check(ctx.ptr, rc, info)
    return list(info)


def block_pf_force(ctx, F, coef, phi, opts):
    S = ctypes.c_double(0.0)
    pF, pp = _mom(ctx, F, "F"), _field(ctx, phi, 1, SAP_F64, "phi")
    _check(ctx.ptr, _lib.block_pf_force(ctx.ptr, pF, coef, pp, ctypes.byref(opts), ctypes.byref(S), _stream()))
    return S.value


def schwarz_boundary_force(ctx, F, coef, chi, opts):
    S = ctypes.c_double(0.0)
    pF, pc = _mom(ctx, F, "F"), _field(ctx, chi, 1, SAP_F64, "chi")
    _check(ctx.ptr, _lib.schwarz_boundary_force(ctx.ptr, pF, coef, pc, ctypes.byref(opts), ctypes.byref(S),
                                                _stream()))
    return S.value


def gauge_force(ctx, F, coef, beta):
    S = ctypes.c_double(0.0)
    _check(ctx.ptr, _lib.gauge_force(ctx.ptr, _mom(ctx, F, "F"), coef, beta, ctypes.byref(S), _stream()))
    return S.value


def schwarz_heat_bath(ctx, chi, g, opts):
    pc, pg = _field(ctx, chi, 1, SAP_F64, "chi"), _field(ctx, g, 1, SAP_F64, "g")
    _check(ctx.ptr, _lib.schwarz_heat_bath(ctx.ptr, pc, pg, ctypes.byref(opts), _stream()))


def schwarz_action(ctx, chi, opts):
    S = ctypes.c_double(0.0)
    _check(ctx.ptr, _lib.schwarz_action(ctx.ptr, _field(ctx, chi, 1, SAP_F64, "chi"), ctypes.byref(opts),
                                        ctypes.byref(S), _stream()))
    return S.value


def sap_update_links(ctx, p, dt):
    _check(ctx.ptr, _lib.sap_update_links(ctx.ptr, _mom(ctx, p, "p"), dt, _stream()))


def sap_plaquette(ctx):
    v = ctypes.c_double(0.0)
    _check(ctx.ptr, _lib.sap_plaquette(ctx.ptr, ctypes.byref(v), _stream()))
    return v.value


def sap_tune(ctx, nrhs):
    """Tune the hop mapping for nrhs; returns microseconds per launch per variant."""
    us = (ctypes.c_float * (6 * HOP_NMAP))()
    _check(ctx.ptr, _lib.sap_tune(ctx.ptr, nrhs, us, _stream()))
    names = ["full_f64", "full_f32", "eo_f64", "eo_f32", "full_f16", "eo_f16"]
    return {n: {m: us[HOP_NMAP * i + k] for k, m in enumerate(HOP_MAP_NAMES) if us[HOP_NMAP * i + k] >= 0}
            for i, n in enumerate(names)}


HOP_MAP_SITE, HOP_MAP_LANE4, HOP_MAP_WAVE4, HOP_MAP_STREAM, HOP_SWEEP = 0, 1, 2, 3, 4
HOP_MAP_REG2, HOP_MAP_REG4, HOP_MAP_REG2_SWEEP, HOP_MAP_REG4_SWEEP = 7, 8, 9, 10
HOP_MAP_MARCH1, HOP_MAP_MARCH2, HOP_MAP_MARCH4 = 11, 12, 13
HOP_MAP_WALK1, HOP_MAP_WALK2 = 14, 15
HOP_MAP_BAND1 = 16
HOP_MAP_SLAB1, HOP_MAP_SLAB1W, HOP_MAP_SLAB2, HOP_MAP_SLABD = 17, 18, 19, 20
HOP_NMAP = 21
HOP_MAP_NAMES = ["site", "lane4", "wave4", "stream", "site_sweep", "lane4_sweep", "wave4_sweep", "reg2", "reg4",
                 "reg2_sweep", "reg4_sweep", "march1", "march2", "march4", "walk1", "walk2", "band1",
                 "slab1", "slab1w", "slab2", "slabd"]


def sap_set_hop_map(ctx, full, prec, nrhs, hop_map):
    _check(ctx.ptr, _lib.sap_set_hop_map(ctx.ptr, int(full), prec, nrhs, hop_map))


def sap_force_profile(ctx, F):
    """x0 profile of the force F (sap momenta layout): a list of two lists of L0 floats,
    [mean |F| over the spatial links of each slice, mean |F| over its time links]."""
    L0 = ctx.L[0]
    out = (ctypes.c_double * (2 * L0))()
    _check(ctx.ptr, _lib.sap_force_profile(ctx.ptr, _mom(ctx, F, "F"), out, _stream()))
    return [list(out[:L0]), list(out[L0:])]


def sap_force_profile_noalloc(ctx, F, prof):
    """The x0 profile of F written to the device tensor prof (2*L0 float64) on the current
    stream, without allocating and without synchronising (see sap_force_profile)."""
    pF, pq = _mom(ctx, F, "F"), _buf(ctx, prof, 2 * ctx.L[0] * 8, "prof")
    _check(ctx.ptr, _lib.sap_force_profile_noalloc(ctx.ptr, pF, pq, _stream()))


def sap_force_profile_noalloc_max() -> int:
    return _lib.sap_force_profile_noalloc_max()


def eo_pf_heat_bath(ctx, phi, xi, kind, rho, opts):
    pp, px = _field(ctx, phi, 1, SAP_F64, "phi"), _field(ctx, xi, 1, SAP_F64, "xi")
    _check(ctx.ptr, _lib.eo_pf_heat_bath(ctx.ptr, pp, px, kind, rho, ctypes.byref(opts), _stream()))


def eo_pf_force(ctx, F, coef, phi, kind, rho, opts):
    """F += coef * dS/dw of S1 (kind 1) or S2 (kind 2); F None: action only. Returns S."""
    S = ctypes.c_double(0.0)
    pF, pp = _mom(ctx, F, "F", optional=True), _field(ctx, phi, 1, SAP_F64, "phi")
    _check(ctx.ptr, _lib.eo_pf_force(ctx.ptr, pF, coef, pp, kind, rho, ctypes.byref(opts), ctypes.byref(S),
                                     _stream()))
    return S.value


def schwarz2_heat_bath(ctx, chi, g, opts):
    pc, pg = _field(ctx, chi, 1, SAP_F64, "chi"), _field(ctx, g, 1, SAP_F64, "g")
    _check(ctx.ptr, _lib.schwarz2_heat_bath(ctx.ptr, pc, pg, ctypes.byref(opts), _stream()))


def schwarz2_force(ctx, F, coef, chi, opts):
    """F += coef * dS/dw of the level-2 Schwarz term (S3); F None: action only. Returns S."""
    S = ctypes.c_double(0.0)
    pF, pc = _mom(ctx, F, "F", optional=True), _field(ctx, chi, 1, SAP_F64, "chi")
    _check(ctx.ptr, _lib.schwarz2_force(ctx.ptr, pF, coef, pc, ctypes.byref(opts), ctypes.byref(S), _stream()))
    return S.value


def hmc4_params(beta, tau, rho, n, p0, xi1, xi2, g3, g4, u_metropolis, force_solve, action_solve,
                scheme=(1, 1, 0, 0, 0), lam=1.0 / 6.0, step_scale=None, time_shift=0, part_solve=None):
    """sap_hmc4_params from torch tensors. part_solve: None, or 8 sap_solve_opts (the force
    solves of S1..S4, then their heat-bath and action solves), kept alive on the result."""
    P = sap_hmc4_params()
    if part_solve is not None:
        if len(part_solve) != 8:
            raise SapError(SAP_E_ARG, "part_solve needs 8 entries (force S1..S4, action S1..S4)")
        P._parts = (sap_solve_opts * 8)(*part_solve)
        P.part_solve = ctypes.cast(P._parts, ctypes.POINTER(sap_solve_opts))
    P.beta, P.tau, P.lambda_, P.rho = beta, tau, lam, rho
    P.n = (ctypes.c_int * 5)(*n)
    P.scheme = (ctypes.c_int * 5)(*scheme)
    P.force_solve, P.action_solve = force_solve, action_solve
    P.p0, P.xi1, P.xi2 = p0.data_ptr(), xi1.data_ptr(), xi2.data_ptr()
    P.g3, P.g4 = g3.data_ptr(), g4.data_ptr()
    P._tensors = {"p0": p0, "xi1": xi1, "xi2": xi2, "g3": g3, "g4": g4}
    P.u_metropolis = u_metropolis
    if step_scale is not None:
        import numpy as np
        P._scale = np.ascontiguousarray(step_scale, dtype=np.float64)
        P.step_scale = P._scale.ctypes.data
    P.time_shift = time_shift
    return P


def _check_hmc_buffers(ctx, U, params):
    """The trajectory reads and writes the canonical gauge field U, reads the momenta (sap
    layout) and the canonical noise spinors whose pointers the params hold."""
    pU = _buf(ctx, U, ctx.V * 36 * 16, "U")
    ten = getattr(params, "_tensors", None)
    if ten is None:
        raise SapError(SAP_E_ARG, "params must come from hmc_params / hmc4_params (they keep the tensors)")
    _mom(ctx, ten["p0"], "p0")
    for k, v in ten.items():
        if k != "p0":
            _buf(ctx, v, ctx.V * 12 * 16, k)
    if getattr(params, "_scale", None) is not None and params._scale.size < 4 * ctx.L[0]:
        raise SapError(SAP_E_ARG, f"step_scale must hold {4 * ctx.L[0]} values ([L0][4])")
    return pU


def hmc_trajectory_4pf(ctx, U, params):
    pU = _check_hmc_buffers(ctx, U, params)
    info = sap_hmc4_info()
    _check(ctx.ptr, _lib.hmc_trajectory_4pf(ctx.ptr, pU, ctypes.byref(params), ctypes.byref(info), _stream()))
    return info


def sap_shift_gauge(ctx, n):
    _check(ctx.ptr, _lib.sap_shift_gauge(ctx.ptr, n, _stream()))


def hmc_params(beta, tau, n_outer, n_inner, p0, xi1, xi2, u_metropolis, force_solve, action_solve,
               lam=1.0 / 6.0, scheme_outer=1, scheme_inner=1, step_scale=None, time_shift=0):
    """sap_hmc_params from torch tensors (p0 in the sap momentum layout, xi canonical);
    step_scale: host float64 array [L0, 4] (kept alive on the returned object)."""
    prm = sap_hmc_params(beta, tau, lam, n_outer, n_inner, scheme_outer, scheme_inner, force_solve,
                         action_solve, p0.data_ptr(), xi1.data_ptr(), xi2.data_ptr(), u_metropolis,
                         None, time_shift)
    prm._tensors = {"p0": p0, "xi1": xi1, "xi2": xi2}
    if step_scale is not None:
        import numpy as np
        prm._scale = np.ascontiguousarray(step_scale, dtype=np.float64)
        prm.step_scale = prm._scale.ctypes.data
    return prm


def hmc_trajectory(ctx, U, params):
    pU = _check_hmc_buffers(ctx, U, params)
    info = sap_hmc_info()
    _check(ctx.ptr, _lib.hmc_trajectory(ctx.ptr, pU, ctypes.byref(params), ctypes.byref(info), _stream()))
    return info


def sap_stream_probe(dst, src, nbytes, mode):
    """Plain streaming kernel over device tensors (mode 0 copy, 1 copy with non-temporal
    stores, 2 read with one float partial per workgroup written to dst)."""
    need = nbytes if mode < 2 else 4 * _lib.sap_stream_probe_blocks()
    pd, ps = _buf(None, dst, need, "dst"), _buf(None, src, nbytes, "src")
    rc = _lib.sap_stream_probe(pd, ps, nbytes, mode, _stream())
    if rc != SAP_OK:
        raise SapError(rc, "sap_stream_probe failed")


# ---- context ------------------------------------------------------------------------

class Context:
    """Owns one ``sap_ctx``: geometry, gauge copies and solver workspace on the current
    HIP device. Fields are torch tensors in the library layout (see ``include/sapmi.h``)."""

    def __init__(self, L, l0, kappa, l0_sub=0, max_rhs=1):
        self.L = tuple(int(v) for v in L)
        self.l0, self.l0_sub, self.kappa, self.max_rhs = int(l0), int(l0_sub), float(kappa), int(max_rhs)
        self.V = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self.Vh = self.V // 2
        g = sap_geom((ctypes.c_int * 4)(*self.L), self.l0, self.l0_sub, self.kappa, self.max_rhs)
        p = ctypes.c_void_p()
        rc = _lib.sap_create(ctypes.byref(g), ctypes.byref(p))
        _check(None, rc)
        self.ptr = p
        import torch
        self.device = torch.cuda.current_device()     # sap_create bound the context to it

    def close(self):
        if getattr(self, "ptr", None):
            _lib.sap_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def nblocks(self, level):
        return self.L[0] // (self.l0 if level == 1 else self.l0_sub)

    # allocation helpers (torch is only the allocator here)
    def field_bytes(self, nrhs=1, prec=SAP_F64):
        return _lib.sap_field_bytes(self.ptr, prec, nrhs)

    def new_field(self, nrhs=1, prec=SAP_F64):
        import torch
        dt = torch.float64 if prec == SAP_F64 else torch.float32
        n = self.field_bytes(nrhs, prec) // (8 if prec == SAP_F64 else 4)
        return torch.zeros(n, dtype=dt, device="cuda")

    def new_momenta(self):
        import torch
        return torch.zeros(_lib.sap_momenta_bytes(self.ptr) // 8, dtype=torch.float64, device="cuda")

    def set_gauge(self, U):
        """U: canonical complex128 gauge field on the device (any shape with V*4*9 entries);
        the links must be SU(3) (checked by the library)."""
        _check(self.ptr, _lib.sap_set_gauge(self.ptr, _buf(self, U, self.V * 36 * 16, "U"), _stream()))

    def get_gauge(self, U):
        _check(self.ptr, _lib.sap_get_gauge(self.ptr, _buf(self, U, self.V * 36 * 16, "U"), _stream()))

    def pack_spinor(self, out, psi, nrhs, prec=SAP_F64):
        po = _field(self, out, nrhs, prec, "out")
        _check(self.ptr, _lib.sap_pack_spinor(self.ptr, po, _buf(self, psi, nrhs * self.V * 12 * 16, "psi"),
                                              nrhs, prec, _stream()))

    def unpack_spinor(self, out, f, nrhs, prec=SAP_F64):
        pf = _field(self, f, nrhs, prec, "f")
        _check(self.ptr, _lib.sap_unpack_spinor(self.ptr, _buf(self, out, nrhs * self.V * 12 * 16, "out"), pf,
                                                nrhs, prec, _stream()))

    def pack_momenta(self, out, p):
        _check(self.ptr, _lib.sap_pack_momenta(self.ptr, _mom(self, out, "out"),
                                               _buf(self, p, self.V * 32 * 8, "p"), _stream()))

    def unpack_momenta(self, out, f):
        _check(self.ptr, _lib.sap_unpack_momenta(self.ptr, _buf(self, out, self.V * 32 * 8, "out"),
                                                 _mom(self, f, "f"), _stream()))
