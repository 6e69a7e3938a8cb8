"""Thin ctypes binding of libqdmf.so.

The functions below carry the C ABI's names and only marshal arguments; every numerical
step runs in the library's HIP kernels.  Device buffers come from PyTorch (ROCm) tensors;
the library never falls back to a CPU path: if libqdmf.so is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqdmf.so")

QDMF_NE, QDMF_AS = 0, 1
QDMF_FP64, QDMF_MIXED = 0, 1
QDMF_ORDER_AMD, QDMF_ORDER_USER, QDMF_ORDER_GRID_ND, QDMF_ORDER_ND, QDMF_ORDER_AUTO = 0, 1, 2, 3, 4
QDMF_ERR_INVALID_ARG = -1
QDMF_ERR_HIP = -2
QDMF_ERR_OOM = -3
QDMF_ERR_INDEX_OVERFLOW = -4
QDMF_ERR_NOT_ANALYSED = -5
QDMF_ERR_NOT_FACTORISED = -6
QDMF_ERR_NO_MATRIX = -7
QDMF_ERR_UNSUPPORTED = -8
QDMF_WARN_DYN_REG = 1
QDMF_WARN_INERTIA = 2
QDMF_WARN_NOT_CONVERGED = 3
QDMF_WARN_LARGE_REG = 4

EXPORTED = ["qdmf_default_options", "qdmf_create", "qdmf_set_stream", "qdmf_analyse",
            "qdmf_symbolic", "qdmf_set_matrix", "qdmf_factorise", "qdmf_solve", "qdmf_solve_noalloc",
            "qdmf_factor_stats", "qdmf_solve_stats", "qdmf_export_d", "qdmf_export_front",
            "qdmf_graph_capture", "qdmf_graph_launch", "qdmf_destroy", "qdmf_status_string",
            "qdmf_last_message", "qdmf_profile_kind", "qdmf_profile_read", "qdmf_batch_analyse",
            "qdmf_batch_offsets", "qdmf_batch_factorise", "qdmf_batch_stats", "qdmf_choose_mode",
            "qdmf_ipm_default_options", "qdmf_ipm_solve", "qdmf_analyse_qp", "qdmf_set_hessian",
            "qdmf_export_flags", "qdmf_batch_factorise_dev", "qdmf_batch_graph_capture", "qdmf_peak_probe"]
QDMF_K_SMALL, QDMF_K_ASSEMBLE, QDMF_K_WINDOW, QDMF_K_SYRK, QDMF_K_FINALIZE, QDMF_K_FWD, QDMF_K_BWD, \
    QDMF_K_SYRK128 = range(8)
KERNEL_KIND_NAMES = {0: "k_small", 1: "k_assemble", 2: "k_window", 3: "k_syrk", 4: "k_finalize", 5: "k_fwd",
                     6: "k_bwd", 7: "k_syrk128"}


class qdmf_options(C.Structure):
    _fields_ = [("nb", C.c_int32), ("alpha", C.c_double), ("eps_lift", C.c_double),
                ("presort", C.c_int32), ("max_refine", C.c_int32), ("max_refine_mixed", C.c_int32),
                ("target_berr", C.c_double), ("target_berr_mixed", C.c_double),
                ("tau_big", C.c_double), ("ordering", C.c_int32), ("grid", C.c_int32 * 3),
                ("amalgamate", C.c_int32), ("f_mix", C.c_int32), ("small_front", C.c_int32),
                ("mem_cap_bytes", C.c_int64), ("split_solve_front", C.c_int32),
                ("syrk_group_front", C.c_int32), ("syrk_group", C.c_int32),
                ("syrk_tile_front", C.c_int32), ("mixed_check", C.c_int32),
                ("lookahead_front", C.c_int32), ("graph_poll", C.c_int32)]


class qdmf_mode_choice(C.Structure):
    _fields_ = [("mode", C.c_int32), ("ndense", C.c_int32), ("ne_abandoned", C.c_int32),
                ("nnz_l_as", C.c_int64), ("nnz_ne_pattern", C.c_int64), ("nnz_l_ne", C.c_int64),
                ("flops_as", C.c_double), ("flops_ne", C.c_double)]


class qdmf_ipm_options(C.Structure):
    _fields_ = [("tau", C.c_double), ("rho", C.c_double), ("delta", C.c_double), ("max_iter", C.c_int32),
                ("correctors", C.c_int32), ("kmax", C.c_int32), ("alpha_f", C.c_double), ("prec", C.c_int32)]


class qdmf_ipm_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("correctors", C.c_int32),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("pinf", C.c_double),
                ("dinf", C.c_double), ("mu", C.c_double), ("ms", C.c_double)]


class qdmf_symbolic_info(C.Structure):
    _fields_ = [("N", C.c_int32), ("nsuper", C.c_int32), ("nlevels", C.c_int32),
                ("max_front", C.c_int32), ("nnz_l", C.c_int64), ("nnz_k", C.c_int64),
                ("flops_fact", C.c_double), ("flops_solve", C.c_double),
                ("device_bytes", C.c_int64), ("front_bytes", C.c_int64),
                ("perm", C.POINTER(C.c_int32)), ("sn_ptr", C.POINTER(C.c_int32)),
                ("sn_parent", C.POINTER(C.c_int32)), ("sn_front", C.POINTER(C.c_int32)),
                ("sn_level", C.POINTER(C.c_int32))]


class qdmf_factor_info(C.Structure):
    _fields_ = [("nneg", C.c_int64), ("npos", C.c_int64), ("nzero", C.c_int64),
                ("n2x2", C.c_int64), ("nlift", C.c_int64), ("nprop3", C.c_int64),
                ("nsign", C.c_int64), ("nzskip", C.c_int64), ("max_edyn", C.c_double),
                ("knorm", C.c_double), ("status", C.c_int32), ("nredo_fp64", C.c_int32)]


class qdmf_solve_info(C.Structure):
    _fields_ = [("nrhs", C.c_int32), ("max_steps", C.c_int32), ("berr_nw", C.c_double),
                ("berr_cw", C.c_double), ("berr_nw_initial", C.c_double), ("status", C.c_int32)]


_lib = None


def lib():
    """Load libqdmf.so; raise if it has not been built (there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2508_04370_amd.build.build()")
        try:  # one HIP runtime per process: let PyTorch's copy load first if present
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.qdmf_default_options.argtypes = [C.POINTER(qdmf_options)]
        L.qdmf_default_options.restype = None
        L.qdmf_create.argtypes = [C.POINTER(P), C.c_int, P, C.POINTER(qdmf_options)]
        L.qdmf_set_stream.argtypes = [P, P]
        L.qdmf_analyse.argtypes = [P, I32, I32, P, P, I32, P]
        L.qdmf_analyse_qp.argtypes = [P, I32, I32, P, P, P, P, P]
        L.qdmf_set_hessian.argtypes = [P, P, I32]
        L.qdmf_choose_mode.argtypes = [P, I32, I32, P, P, C.POINTER(qdmf_mode_choice)]
        L.qdmf_ipm_default_options.argtypes = [C.POINTER(qdmf_ipm_options)]
        L.qdmf_ipm_default_options.restype = None
        L.qdmf_ipm_solve.argtypes = [P, P, P, P, P, P, P, P, P, C.POINTER(qdmf_ipm_options), C.POINTER(qdmf_ipm_info), P]
        L.qdmf_symbolic.argtypes = [P, C.POINTER(qdmf_symbolic_info)]
        L.qdmf_set_matrix.argtypes = [P, P, I32]
        L.qdmf_factorise.argtypes = [P, P, D, D, I32]
        L.qdmf_solve.argtypes = [P, I32, P, P, P, P]
        L.qdmf_solve_noalloc.argtypes = [P, I32, P, P, P, P]
        L.qdmf_factor_stats.argtypes = [P, C.POINTER(qdmf_factor_info)]
        L.qdmf_solve_stats.argtypes = [P, C.POINTER(qdmf_solve_info), P, P]
        L.qdmf_export_d.argtypes = [P, P, P, P, P, P]
        L.qdmf_export_flags.argtypes = [P, P]
        L.qdmf_export_front.argtypes = [P, I32, P, P]
        L.qdmf_graph_capture.argtypes = [P, P, D, D, I32, I32, I32, P, P, P, P]
        L.qdmf_graph_launch.argtypes = [P]
        L.qdmf_destroy.argtypes = [P]
        L.qdmf_destroy.restype = None
        L.qdmf_status_string.argtypes = [C.c_int]
        L.qdmf_status_string.restype = C.c_char_p
        L.qdmf_last_message.argtypes = [P]
        L.qdmf_last_message.restype = C.c_char_p
        L.qdmf_profile_kind.argtypes = [P, I32]
        L.qdmf_profile_read.argtypes = [P, P, P, P, P]
        L.qdmf_batch_analyse.argtypes = [P, I32, P, P, P, P, I32]
        L.qdmf_batch_offsets.argtypes = [P, P, P]
        L.qdmf_batch_factorise.argtypes = [P, P, P, P, I32]
        L.qdmf_batch_factorise_dev.argtypes = [P, P, P, P, I32]
        L.qdmf_peak_probe.argtypes = [C.c_int, P, P, P, P, P]
        L.qdmf_batch_graph_capture.argtypes = [P, P, P, P, I32, I32, I32, P, P, P, P]
        L.qdmf_batch_stats.argtypes = [P, P, P, P]
        for name in EXPORTED:
            getattr(L, name)
        _lib = L
    return _lib


def _np(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dev(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class QdmfError(RuntimeError):
    def __init__(self, code, where, detail=""):
        self.code = code
        msg = lib().qdmf_status_string(code).decode()
        super().__init__(f"{where}: {msg} ({code}){': ' + detail if detail else ''}")


def _check(rc, where, h=None):
    if rc < 0:
        detail = lib().qdmf_last_message(h).decode() if h else ""
        raise QdmfError(rc, where, detail)
    return rc


# ---- C ABI, one Python function per entry point ------------------------------------------

def qdmf_default_options(**overrides):
    o = qdmf_options()
    lib().qdmf_default_options(C.byref(o))
    for k, v in overrides.items():
        if k == "grid":
            o.grid = (C.c_int32 * 3)(*v)
        else:
            setattr(o, k, v)
    return o


def qdmf_create(device=0, stream=None, opt=None):
    h = C.c_void_p()
    _check(lib().qdmf_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None,
                             C.byref(opt) if opt is not None else None), "qdmf_create")
    return h


def qdmf_set_stream(h, stream):
    return _check(lib().qdmf_set_stream(h, C.c_void_p(stream) if stream else None), "qdmf_set_stream", h)


def qdmf_analyse(h, m, n, colptr, rowidx, mode, user_perm=None):
    cp = np.ascontiguousarray(colptr, np.int64)
    ri = np.ascontiguousarray(rowidx, np.int32)
    up = None if user_perm is None else np.ascontiguousarray(user_perm, np.int32)
    return _check(lib().qdmf_analyse(h, int(m), int(n), _np(cp), _np(ri), int(mode), _np(up)),
                  "qdmf_analyse", h)


def qdmf_analyse_qp(h, m, n, colptr, rowidx, q_colptr, q_rowidx, user_perm=None):
    """Quadratic program: A's pattern with Q's lower triangle (CSC, n columns)."""
    cp = np.ascontiguousarray(colptr, np.int64)
    ri = np.ascontiguousarray(rowidx, np.int32)
    qcp = np.ascontiguousarray(q_colptr, np.int64)
    qri = np.ascontiguousarray(q_rowidx, np.int32)
    up = None if user_perm is None else np.ascontiguousarray(user_perm, np.int32)
    return _check(lib().qdmf_analyse_qp(h, int(m), int(n), _np(cp), _np(ri), _np(qcp), _np(qri), _np(up)),
                  "qdmf_analyse_qp", h)


def qdmf_set_hessian(h, q_val, on_device=False):
    if on_device:
        return _check(lib().qdmf_set_hessian(h, _dev(q_val), 1), "qdmf_set_hessian", h)
    q = np.ascontiguousarray(q_val, np.float64)
    return _check(lib().qdmf_set_hessian(h, _np(q), 0), "qdmf_set_hessian", h)


def qdmf_ipm_default_options(**overrides):
    o = qdmf_ipm_options()
    lib().qdmf_ipm_default_options(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def qdmf_ipm_solve(h, b, c, x, y, zl, opt=None, l=None, u=None, zu=None):
    """Interior point driver on device tensors (contiguous float64): b (m), c (n), optional
    bounds l, u (n; None: l = 0, u = +inf), and outputs x, zl (n), y (m) and optional zu (n).
    Returns (info dict, history array of shape (iters, 4): mu, alpha_p, alpha_d, correctors
    used).  A positive status (iteration limit) is returned in the dict."""
    opt = opt if opt is not None else qdmf_ipm_default_options()
    info = qdmf_ipm_info()
    hist = np.zeros(4 * max(1, opt.max_iter))
    rc = lib().qdmf_ipm_solve(h, _dev(b), _dev(c), _dev(l), _dev(u), _dev(x), _dev(y), _dev(zl), _dev(zu),
                              C.byref(opt), C.byref(info), _np(hist))
    if rc < 0:
        _check(rc, "qdmf_ipm_solve", h)
    out = {k: getattr(info, k) for k, _ in qdmf_ipm_info._fields_}
    return out, hist[:4 * info.iters].reshape(-1, 4)


def qdmf_choose_mode(h, m, n, colptr, rowidx):
    """NE or AS for the pattern of A, with the counts the choice rests on (a dict)."""
    cp = np.ascontiguousarray(colptr, np.int64)
    ri = np.ascontiguousarray(rowidx, np.int32)
    c = qdmf_mode_choice()
    _check(lib().qdmf_choose_mode(h, int(m), int(n), _np(cp), _np(ri), C.byref(c)), "qdmf_choose_mode", h)
    return {k: getattr(c, k) for k, _ in qdmf_mode_choice._fields_}


def qdmf_symbolic(h):
    info = qdmf_symbolic_info()
    _check(lib().qdmf_symbolic(h, C.byref(info)), "qdmf_symbolic", h)
    N, ns = info.N, info.nsuper
    out = {k: getattr(info, k) for k in ("N", "nsuper", "nlevels", "max_front", "nnz_l", "nnz_k",
                                         "flops_fact", "flops_solve", "device_bytes", "front_bytes")}
    out["perm"] = np.ctypeslib.as_array(info.perm, (N,)).copy() if N else np.zeros(0, np.int32)
    out["sn_ptr"] = np.ctypeslib.as_array(info.sn_ptr, (ns + 1,)).copy()
    for k in ("sn_parent", "sn_front", "sn_level"):
        out[k] = np.ctypeslib.as_array(getattr(info, k), (ns,)).copy() if ns else np.zeros(0, np.int32)
    return out


def qdmf_set_matrix(h, a_val, on_device=False):
    if on_device:
        return _check(lib().qdmf_set_matrix(h, _dev(a_val), 1), "qdmf_set_matrix", h)
    a = np.ascontiguousarray(a_val, np.float64)
    return _check(lib().qdmf_set_matrix(h, _np(a), 0), "qdmf_set_matrix", h)


def qdmf_factorise(h, theta_dev, rho, delta, prec=QDMF_FP64):
    return _check(lib().qdmf_factorise(h, _dev(theta_dev), float(rho), float(delta), int(prec)),
                  "qdmf_factorise", h)


def qdmf_solve(h, nrhs, r7_dev, r1_dev, dx_dev, dy_dev):
    return _check(lib().qdmf_solve(h, int(nrhs), _dev(r7_dev), _dev(r1_dev), _dev(dx_dev),
                                   _dev(dy_dev)), "qdmf_solve", h)


def qdmf_solve_noalloc(h, nrhs, r7_dev, r1_dev, dx_dev, dy_dev):
    return _check(lib().qdmf_solve_noalloc(h, int(nrhs), _dev(r7_dev), _dev(r1_dev), _dev(dx_dev),
                                           _dev(dy_dev)), "qdmf_solve_noalloc", h)


NOALLOC_SCRATCH_BYTES = 64 << 20


def qdmf_factor_stats(h):
    info = qdmf_factor_info()
    rc = _check(lib().qdmf_factor_stats(h, C.byref(info)), "qdmf_factor_stats", h)
    d = {k: getattr(info, k) for k, _ in qdmf_factor_info._fields_}
    d["rc"] = rc
    return d


def qdmf_solve_stats(h, nrhs):
    info = qdmf_solve_info()
    be = np.zeros(nrhs)
    st = np.zeros(nrhs, np.int32)
    rc = _check(lib().qdmf_solve_stats(h, C.byref(info), _np(be), _np(st)), "qdmf_solve_stats", h)
    d = {k: getattr(info, k) for k, _ in qdmf_solve_info._fields_}
    d.update(rc=rc, berr_nw_per_rhs=be, steps_per_rhs=st)
    return d


def qdmf_export_d(h, N):
    po = np.zeros(N, np.int32)
    d = np.zeros(N)
    doff = np.zeros(N)
    pt = np.zeros(N, np.int8)
    ed = np.zeros(N)
    _check(lib().qdmf_export_d(h, _np(po), _np(d), _np(doff), _np(pt), _np(ed)), "qdmf_export_d", h)
    return dict(pivot_order=po, d=d, doff=doff, ptype=pt, edyn=ed)


def qdmf_export_flags(h, N):
    fl = np.zeros(N, np.uint8)
    _check(lib().qdmf_export_flags(h, _np(fl)), "qdmf_export_flags", h)
    return fl


def qdmf_export_front(h, s, f, p):
    panel = np.zeros((f, p), order="F")
    rows = np.zeros(f, np.int32)
    _check(lib().qdmf_export_front(h, int(s), _np(panel), _np(rows)), "qdmf_export_front", h)
    return panel, rows


def qdmf_graph_capture(h, theta_dev, rho, delta, prec, nsolves, nrhs, r7_dev, r1_dev, dx_dev, dy_dev):
    return _check(lib().qdmf_graph_capture(h, _dev(theta_dev), float(rho), float(delta), int(prec),
                                           int(nsolves), int(nrhs), _dev(r7_dev), _dev(r1_dev),
                                           _dev(dx_dev), _dev(dy_dev)), "qdmf_graph_capture", h)


def qdmf_graph_launch(h):
    return _check(lib().qdmf_graph_launch(h), "qdmf_graph_launch", h)


def qdmf_destroy(h):
    if h:
        lib().qdmf_destroy(h)


def qdmf_profile_kind(h, kind):
    return _check(lib().qdmf_profile_kind(h, int(kind)), "qdmf_profile_kind", h)


def qdmf_profile_read(h):
    n = C.c_int64()
    ms = C.c_double()
    fl = C.c_double()
    by = C.c_double()
    _check(lib().qdmf_profile_read(h, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)), "qdmf_profile_read", h)
    return dict(launches=n.value, total_ms=ms.value, flops=fl.value, bytes=by.value)


def qdmf_batch_analyse(h, lps, mode):
    """lps: list of dicts with m, n, colptr, rowidx (one per system)."""
    cnt = len(lps)
    m = np.array([lp["m"] for lp in lps], np.int32)
    n = np.array([lp["n"] for lp in lps], np.int32)
    cps = [np.ascontiguousarray(lp["colptr"], np.int64) for lp in lps]
    ris = [np.ascontiguousarray(lp["rowidx"], np.int32) for lp in lps]
    cpp = (C.c_void_p * cnt)(*[a.ctypes.data for a in cps])
    rip = (C.c_void_p * cnt)(*[a.ctypes.data if a.size else None for a in ris])
    return _check(lib().qdmf_batch_analyse(h, cnt, _np(m), _np(n), cpp, rip, int(mode)), "qdmf_batch_analyse", h)


def qdmf_batch_offsets(h, count):
    ro = np.zeros(count + 1, np.int64)
    co = np.zeros(count + 1, np.int64)
    _check(lib().qdmf_batch_offsets(h, _np(ro), _np(co)), "qdmf_batch_offsets", h)
    return ro, co


def qdmf_batch_factorise(h, theta_dev, rho, delta, prec=QDMF_FP64):
    r = np.ascontiguousarray(rho, np.float64)
    d = np.ascontiguousarray(delta, np.float64)
    return _check(lib().qdmf_batch_factorise(h, _dev(theta_dev), _np(r), _np(d), int(prec)),
                  "qdmf_batch_factorise", h)


def qdmf_batch_factorise_dev(h, theta_dev, rho_dev, delta_dev, prec=QDMF_FP64):
    return _check(lib().qdmf_batch_factorise_dev(h, _dev(theta_dev), _dev(rho_dev), _dev(delta_dev), int(prec)),
                  "qdmf_batch_factorise_dev", h)


def qdmf_batch_graph_capture(h, theta_dev, rho_dev, delta_dev, prec, nsolves, nrhs, r7_dev, r1_dev, dx_dev,
                             dy_dev):
    return _check(lib().qdmf_batch_graph_capture(h, _dev(theta_dev), _dev(rho_dev), _dev(delta_dev), int(prec),
                                                 int(nsolves), int(nrhs), _dev(r7_dev), _dev(r1_dev),
                                                 _dev(dx_dev), _dev(dy_dev)), "qdmf_batch_graph_capture", h)


def qdmf_peak_probe(device=0, stream=None):
    v = [C.c_double() for _ in range(4)]
    _check(lib().qdmf_peak_probe(int(device), stream, *[C.byref(x) for x in v]), "qdmf_peak_probe")
    return dict(mfma_f64_tflops=v[0].value, mfma_f32_tflops=v[1].value, valu_f64_tflops=v[2].value,
                hbm_gbs=v[3].value)


def qdmf_batch_stats(h, count, nrhs=0):
    inertia = np.zeros(3 * count, np.int64)
    be = np.zeros(max(1, count * nrhs))
    st = np.zeros(max(1, count * nrhs), np.int32)
    _check(lib().qdmf_batch_stats(h, _np(inertia), _np(be) if nrhs else None, _np(st) if nrhs else None),
           "qdmf_batch_stats", h)
    out = dict(inertia=inertia.reshape(count, 3))
    if nrhs:
        out["berr_nw"] = be.reshape(nrhs, count)
        out["steps"] = st.reshape(nrhs, count)
    return out


def qdmf_status_string(code):
    return lib().qdmf_status_string(int(code)).decode()


# ---- convenience wrapper -----------------------------------------------------------------

class Solver:
    """One analysed system on one GPU: analyse once, then factorise/solve per iteration.

    ``lp`` is a dict with m, n, colptr, rowidx, val, mode (see workloads.py); a quadratic
    program also has q_colptr, q_rowidx, q_val (Q's lower triangle).  Device buffers are
    torch tensors on ``cuda:device``; ``device=-1`` gives a host-only handle (analyse and
    symbolic information only).
    """

    def __init__(self, lp, device=0, stream=None, perm=None, systems=None, **opts):
        """systems: the list of independent systems whose block-diagonal concatenation is lp
        (workloads.concat_systems); they are analysed as a batch."""
        self.lp = lp
        self.device = device
        self.systems = systems
        self.opt = qdmf_default_options(**opts)
        if perm is not None:
            self.opt.ordering = QDMF_ORDER_USER
        if stream is None and device >= 0:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        self.h = qdmf_create(device, stream, self.opt)
        qp = lp.get("q_colptr") is not None
        if systems is not None:
            qdmf_batch_analyse(self.h, systems, lp["mode"])
        elif qp:
            qdmf_analyse_qp(self.h, lp["m"], lp["n"], lp["colptr"], lp["rowidx"], lp["q_colptr"], lp["q_rowidx"],
                            perm)
        else:
            qdmf_analyse(self.h, lp["m"], lp["n"], lp["colptr"], lp["rowidx"], lp["mode"], perm)
        self.sym = qdmf_symbolic(self.h)
        self.N = self.sym["N"]
        if device >= 0:
            qdmf_set_matrix(self.h, lp["val"])
            if qp:
                qdmf_set_hessian(self.h, lp["q_val"])

    def close(self):
        if getattr(self, "h", None):
            qdmf_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def factorise(self, theta_dev, rho, delta, prec=QDMF_FP64):
        qdmf_factorise(self.h, theta_dev, rho, delta, prec)

    def solve(self, r7_dev, r1_dev, dx_dev=None, dy_dev=None):
        import torch
        nrhs = r1_dev.shape[1] if r1_dev.dim() == 2 else 1
        dev = r1_dev.device
        if dx_dev is None:
            dx_dev = torch.empty((nrhs, self.lp["n"]), dtype=torch.float64, device=dev).T
        if dy_dev is None:
            dy_dev = torch.empty((nrhs, self.lp["m"]), dtype=torch.float64, device=dev).T
        qdmf_solve(self.h, nrhs, r7_dev, r1_dev, dx_dev, dy_dev)
        return dx_dev, dy_dev

    def solve_noalloc(self, r7_dev, r1_dev, dx_dev, dy_dev):
        """qdmf_solve_noalloc: the outputs are the caller's (nothing is allocated)."""
        nrhs = r1_dev.shape[1] if r1_dev.dim() == 2 else 1
        qdmf_solve_noalloc(self.h, nrhs, r7_dev, r1_dev, dx_dev, dy_dev)
        return dx_dev, dy_dev

    def factor_stats(self):
        return qdmf_factor_stats(self.h)

    def batch_stats(self, nrhs=0):
        return qdmf_batch_stats(self.h, len(self.systems) if self.systems else 1, nrhs)

    def solve_stats(self, nrhs=1):
        return qdmf_solve_stats(self.h, nrhs)

    def export_d(self):
        return qdmf_export_d(self.h, self.N)

    def export_flags(self):
        return qdmf_export_flags(self.h, self.N)

    def export_front(self, s):
        f = int(self.sym["sn_front"][s])
        p = int(self.sym["sn_ptr"][s + 1] - self.sym["sn_ptr"][s])
        return qdmf_export_front(self.h, s, f, p)


def to_device_colmajor(a, device="cuda"):
    """numpy (rows,) or (rows, cols) -> torch float64 tensor on ``device`` with
    column-major storage (leading dimension = rows), as the C ABI expects."""
    import torch
    a = np.asarray(a, np.float64)
    if a.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(a)).to(device)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to(device).T
