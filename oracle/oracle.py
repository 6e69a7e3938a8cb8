"""ctypes wrapper of the reference (oracle) implementation in ``qdmf_oracle.c``.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product library.  Builds ``liboracle.so`` with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "qdmf_oracle.c")

NE, AS = 0, 1
EF_LIFT, EF_PROP3, EF_SIGN = 1, 2, 4  # dynamic regularisation bits per pivot


def build(force=True):
    """Compile the oracle (plain C, -O2, no BLAS, single-threaded)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Opts(C.Structure):
    _fields_ = [("nb", C.c_int), ("alpha", C.c_double), ("eps_lift", C.c_double),
                ("presort", C.c_int), ("max_refine", C.c_int), ("target_berr", C.c_double),
                ("tau_big", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("nneg", C.c_int64), ("npos", C.c_int64), ("nzero", C.c_int64),
                ("n2x2", C.c_int64), ("nlift", C.c_int64), ("nprop3", C.c_int64),
                ("nsign", C.c_int64), ("nzskip", C.c_int64), ("max_edyn", C.c_double),
                ("large_reg", C.c_int), ("nbkd", C.c_int64)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_analyse.argtypes = [C.c_int, C.c_int, P, P, C.c_int, P, C.POINTER(P)]
        L.orc_analyse_qp.argtypes = [C.c_int, C.c_int, P, P, P, P, P, C.POINTER(P)]
        L.orc_factorise_qp.argtypes = [P, P, P, P, C.c_double, C.c_double, C.POINTER(Opts), C.POINTER(P)]
        L.orc_residual_qp.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, P, P, P, P, C.c_double,
                                      C.c_double, P, P, P, P, P, P]
        L.orc_sym_free.argtypes = [P]
        for nm in ("orc_sym_info", "orc_sym_perm", "orc_sym_parent", "orc_sym_colcount",
                   "orc_sym_snptr", "orc_sym_snparent"):
            getattr(L, nm).argtypes = [P, P]
        L.orc_sym_front_rows.argtypes = [P, P, P]
        L.orc_factorise.argtypes = [P, P, P, C.c_double, C.c_double, C.POINTER(Opts), C.POINTER(P)]
        L.orc_num_free.argtypes = [P]
        L.orc_num_stats.argtypes = [P, C.POINTER(Stats)]
        L.orc_num_knorm.argtypes = [P]
        L.orc_num_knorm.restype = C.c_double
        L.orc_num_export.argtypes = [P] * 7
        L.orc_num_eflags.argtypes = [P, P]
        L.orc_solve.argtypes = [P, P, C.c_int, P, P, P, P, P, P, P]
        L.orc_residual.argtypes = [C.c_int, C.c_int, P, P, P, C.c_int, P, C.c_double,
                                   C.c_double, P, P, P, P, P, P]
        L.orc_front_factor.argtypes = [C.c_int, C.c_int, P, P, P, P, C.c_double,
                                       C.POINTER(Opts), P, P, P, P, C.POINTER(Stats)]
        L.orc_default_opts.argtypes = [C.POINTER(Opts)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def default_opts(**kw):
    o = Opts()
    lib().orc_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _qp(lp):
    """Q's lower-triangle pattern of a quadratic program (lp keys q_colptr, q_rowidx) or None."""
    if lp.get("q_colptr") is None:
        return None, None
    return (np.ascontiguousarray(lp["q_colptr"], np.int64), np.ascontiguousarray(lp["q_rowidx"], np.int32))


class Sym:
    """Symbolic analysis: ordering, elimination tree, fundamental supernodes.  A quadratic
    program (AS only) carries Q's lower triangle in lp["q_colptr"], lp["q_rowidx"]."""

    def __init__(self, lp, perm=None):
        self.lp = lp
        self._cp = np.ascontiguousarray(lp["colptr"], np.int64)
        self._ri = np.ascontiguousarray(lp["rowidx"], np.int32)
        self._qcp, self._qri = _qp(lp)
        up = None if perm is None else np.ascontiguousarray(perm, np.int32)
        h = C.c_void_p()
        if self._qcp is None:
            rc = lib().orc_analyse(lp["m"], lp["n"], _p(self._cp), _p(self._ri), lp["mode"], _p(up),
                                   C.byref(h))
        else:
            if lp["mode"] != AS:
                raise ValueError("quadratic programs need the augmented system")
            rc = lib().orc_analyse_qp(lp["m"], lp["n"], _p(self._cp), _p(self._ri), _p(self._qcp),
                                      _p(self._qri), _p(up), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_analyse failed ({rc})")
        self.h = h
        info = np.zeros(5, np.int64)
        lib().orc_sym_info(h, _p(info))
        self.N, self.nsuper, self.nnzL, self.maxfront, self.flops = (int(v) for v in info)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_sym_free(self.h)
            self.h = None

    def perm(self):
        a = np.zeros(self.N, np.int32); lib().orc_sym_perm(self.h, _p(a)); return a

    def parent(self):
        a = np.zeros(self.N, np.int32); lib().orc_sym_parent(self.h, _p(a)); return a

    def colcount(self):
        a = np.zeros(self.N, np.int64); lib().orc_sym_colcount(self.h, _p(a)); return a

    def snptr(self):
        a = np.zeros(self.nsuper + 1, np.int32); lib().orc_sym_snptr(self.h, _p(a)); return a

    def snparent(self):
        a = np.zeros(self.nsuper, np.int32); lib().orc_sym_snparent(self.h, _p(a)); return a

    def front_rows(self):
        rp = np.zeros(self.nsuper + 1, np.int64)
        rows = np.zeros(max(1, self._rows_total()), np.int32)
        lib().orc_sym_front_rows(self.h, _p(rp), _p(rows))
        return rp, rows

    def _rows_total(self):
        snp = self.snptr()
        cc = self.colcount()
        # front of supernode s has (p + colcount(last) - 1) rows
        return int(sum((snp[s + 1] - snp[s]) + cc[snp[s + 1] - 1] - 1 for s in range(self.nsuper)))


class Num:
    """Numeric factorisation P (K_static + E_dyn) P^T = L D L^T.  qval: Q's lower values of a
    quadratic program (default lp["q_val"])."""

    def __init__(self, sym, aval, theta, rho, delta, opts=None, qval=None):
        self.sym = sym
        self.opts = opts or default_opts()
        self._a = np.ascontiguousarray(aval, np.float64)
        self._t = np.ascontiguousarray(theta, np.float64)
        h = C.c_void_p()
        if sym._qcp is None:
            rc = lib().orc_factorise(sym.h, _p(self._a), _p(self._t), float(rho), float(delta),
                                     C.byref(self.opts), C.byref(h))
        else:
            self._q = np.ascontiguousarray(sym.lp["q_val"] if qval is None else qval, np.float64)
            rc = lib().orc_factorise_qp(sym.h, _p(self._a), _p(self._q), _p(self._t), float(rho),
                                        float(delta), C.byref(self.opts), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_factorise failed ({rc})")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_num_free(self.h)
            self.h = None

    def stats(self):
        s = Stats(); lib().orc_num_stats(self.h, C.byref(s)); return s.asdict()

    def knorm(self):
        return lib().orc_num_knorm(self.h)

    def export(self, dense=True):
        N = self.sym.N
        fperm = np.zeros(N, np.int32)
        L = np.zeros((N, N), order="F") if dense else None
        d = np.zeros(N); doff = np.zeros(N); pt = np.zeros(N, np.int8); ed = np.zeros(N)
        lib().orc_num_export(self.h, _p(fperm), _p(L), _p(d), _p(doff), _p(pt), _p(ed))
        ef = np.zeros(N, np.int8)
        lib().orc_num_eflags(self.h, _p(ef))
        return dict(fperm=fperm, L=L, d=d, doff=doff, ptype=pt, edyn=ed, eflag=ef)

    def solve(self, r7, r1):
        lp = self.sym.lp
        m, n = lp["m"], lp["n"]
        r1 = np.asfortranarray(np.atleast_2d(np.asarray(r1, np.float64).T).T)
        nrhs = r1.shape[1]
        r7a = None if r7 is None else np.asfortranarray(np.atleast_2d(np.asarray(r7, np.float64).T).T)
        dx = np.zeros((n, nrhs), order="F"); dy = np.zeros((m, nrhs), order="F")
        bn = np.zeros(nrhs); bc = np.zeros(nrhs); st = np.zeros(nrhs, np.int32)
        lib().orc_solve(self.sym.h, self.h, nrhs, _p(r7a), _p(r1), _p(dx), _p(dy), _p(bn), _p(bc),
                        _p(st))
        return dict(dx=dx, dy=dy, berr_nw=bn, berr_cw=bc, steps=st)


def residual(lp, theta, rho, delta, x, b):
    """r = b - K_static x and the backward errors, from A, Theta, rho, delta (and Q of a
    quadratic program) directly."""
    cp = np.ascontiguousarray(lp["colptr"], np.int64)
    ri = np.ascontiguousarray(lp["rowidx"], np.int32)
    av = np.ascontiguousarray(lp["val"], np.float64)
    th = np.ascontiguousarray(theta, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    r = np.zeros_like(x)
    nw = C.c_double(); cw = C.c_double(); kn = C.c_double()
    qcp, qri = _qp(lp)
    if qcp is None:
        lib().orc_residual(lp["m"], lp["n"], _p(cp), _p(ri), _p(av), lp["mode"], _p(th), float(rho),
                           float(delta), _p(x), _p(b), _p(r), C.byref(nw), C.byref(cw), C.byref(kn))
    else:
        qv = np.ascontiguousarray(lp["q_val"], np.float64)
        rc = lib().orc_residual_qp(lp["m"], lp["n"], _p(cp), _p(ri), _p(av), lp["mode"], _p(qcp), _p(qri),
                                   _p(qv), _p(th), float(rho), float(delta), _p(x), _p(b), _p(r),
                                   C.byref(nw), C.byref(cw), C.byref(kn))
        if rc != 0:
            raise ValueError(f"orc_residual_qp failed ({rc})")
    return r, nw.value, cw.value, kn.value


def system_rhs(lp, r7, r1, theta):
    """Right-hand side b of the factorised system: AS [r7; r1]; NE r1 + A theta~ r7."""
    if lp["mode"] == AS:
        return np.concatenate([np.asarray(r7, np.float64).ravel(), np.asarray(r1, np.float64).ravel()])
    b = np.array(r1, np.float64).ravel()
    if r7 is not None:
        tt = 1.0 / (1.0 / np.asarray(theta) + lp["rho"])
        cp, ri, av = lp["colptr"], lp["rowidx"], lp["val"]
        r7 = np.asarray(r7, np.float64).ravel()
        for j in range(lp["n"]):
            for e in range(cp[j], cp[j + 1]):
                b[ri[e]] += av[e] * (tt[j] * r7[j])
    return b


def front_factor(F, p, sigma, shift, knorm, opts=None):
    """Partial LDL^T of one dense front.  Returns a dict with the factored front."""
    F = np.array(F, np.float64, order="F", copy=True)
    f = F.shape[0]
    sg = np.array(sigma, np.int8, copy=True)
    sh = np.array(shift, np.float64, copy=True)
    perm = np.zeros(f, np.int32)
    d = np.zeros(f); doff = np.zeros(f); pt = np.zeros(f, np.int8); ed = np.zeros(f)
    st = Stats()
    o = opts or default_opts()
    lib().orc_front_factor(f, p, _p(F), _p(sg), _p(sh), _p(perm), float(knorm), C.byref(o),
                           _p(d), _p(doff), _p(pt), _p(ed), C.byref(st))
    return dict(F=F, perm=perm, d=d[:p], doff=doff[:p], ptype=pt[:p], edyn=ed[:p],
                sigma=sg, shift=sh, stats=st.asdict())
