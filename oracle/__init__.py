"""Oracle for the resistive GRMHD IMEX-RK2 stage update (arXiv:2510.18968).

TEST INFRASTRUCTURE ONLY.  A plain, slow FP64 CPU implementation of the
discrete operator, written from the paper (see the header of
``rmhd_oracle.cpp`` for the equation each part follows).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The HIP library shares no code with it.

Arrays are numpy float64, field-major ``[nf, nz_p, ny_p, nx_p]`` (padded with
ghost cells, x fastest), the same layout the C-ABI library uses.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmhd_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_COPY, BC_GIVEN = 0, 1, 2
REC_MINMOD, REC_MC2, REC_WENO5 = 0, 1, 2
ST_OK, ST_WARN, ST_NOCONV, ST_UNPHYS = 0, 1, -3, -4


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["g++", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c++17",
               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out_dir: str) -> str:
    """Compile oracle/sanitize_main.cpp (the oracle's source plus a driver
    that calls every grid entry point on small grids) with the address and
    undefined-behaviour sanitizers, into out_dir; returns the executable."""
    exe = os.path.join(out_dir, "oracle_sanitized")
    src = os.path.join(os.path.dirname(_SRC), "sanitize_main.cpp")
    cmd = ["g++", "-O1", "-g", "-ffp-contract=off", "-fopenmp", "-std=c++17", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.dirname(_SRC), "-o", exe, src]
    subprocess.run(cmd, check=True)
    return exe


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("active", C.c_int32), ("ng", C.c_int32), ("bc", C.c_int32 * 3),
                ("recon", C.c_int32), ("c2p_maxit", C.c_int32), ("speed_mode", C.c_int32),
                ("sigma_model", C.c_int32),
                ("x0", C.c_double * 3), ("dx", C.c_double * 3),
                ("gamma_ad", C.c_double), ("kappa", C.c_double), ("c2p_tol", C.c_double),
                ("sigma0", C.c_double), ("sigma_exp", C.c_double), ("sigma_Datmo", C.c_double),
                ("rho_atmo", C.c_double), ("K_atmo", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp, ip, gp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(Grid)
        sig = {
            "orc_gamma_imex": (C.c_double, []),
            "orc_point_prim2con": (None, [dp, C.c_double, dp, dp]),
            "orc_point_metric": (None, [dp, dp, dp]),
            "orc_point_flux": (None, [dp, C.c_double, dp, C.c_double, C.c_int, dp]),
            "orc_point_hlle": (None, [dp, C.c_double, dp, dp, C.c_double, C.c_int, C.c_int, dp]),
            "orc_point_speeds": (None, [dp, C.c_int, C.c_int, dp, dp]),
            "orc_point_stiff": (None, [dp, dp, dp, dp, C.c_double, dp]),
            "orc_point_esolve": (None, [dp, dp, dp, dp, C.c_double, dp]),
            "orc_point_coupled": (C.c_int, [dp, C.c_double, dp, dp, C.c_double, C.c_double, dp, C.c_double,
                                            C.c_int, dp, dp, C.POINTER(C.c_int)]),
            "orc_point_recover_paper": (C.c_int, [dp, C.c_double, dp, dp, C.c_double, C.c_double, dp, C.c_double,
                                                  C.c_int, dp, dp, C.POINTER(C.c_int)]),
            "orc_recon": (None, [C.c_int, dp, dp, dp]),
            "orc_padded_cells": (C.c_long, [gp]),
            "orc_ghost_fill": (None, [gp, dp, C.c_int]),
            "orc_prim2con": (None, [gp, dp, dp, dp]),
            "orc_con2prim": (C.c_long, [gp, dp, dp, dp, dp, ip, ip]),
            "orc_explicit_rhs": (None, [gp, dp, dp, dp, dp]),
            "orc_stage1": (C.c_long, [gp, dp, C.c_double, dp, dp, dp, dp, dp, dp, ip, ip]),
            "orc_stage2": (C.c_long, [gp, dp, C.c_double, dp, dp, dp, dp, dp, dp, dp, dp, ip, ip]),
            "orc_final": (C.c_long, [gp, dp, C.c_double, dp, dp, dp, dp, dp, dp, dp, dp, ip, ip]),
            "orc_step": (C.c_long, [gp, dp, C.c_double, dp, dp, dp, ip]),
            "orc_step_tangent": (C.c_long, [gp, dp, C.c_double, dp, dp, dp, dp, dp, dp]),
            "orc_max_signal_speed": (C.c_double, [gp, dp]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int32))


SIGMA_FIELD, SIGMA_POWER, SIGMA_DYNAMO = 0, 1, 2
ATMO_FACTOR = 1.01


def make_grid(n, active, dx, bc, gamma_ad, recon=REC_WENO5, kappa=1.0, x0=(0.0, 0.0, 0.0), ng=3,
              c2p_tol=1e-14, c2p_maxit=500, speed_mode=0, sigma_model=0, sigma0=0.0, sigma_exp=0.0,
              sigma_Datmo=0.0, rho_atmo=0.0, K_atmo=0.0) -> Grid:
    """sigma_model 0: the given per-cell sigma field; 1: sigma0 D^sigma_exp
    (eq. sigma_evol); 2: sigma0 max(1 - sigma_Datmo/D, 0)^2 (eq.
    dynamo_sigma).  rho_atmo > 0: the step-end atmosphere (rho_atmo, p =
    K_atmo rho_atmo^Gamma, v = 0) below D = ATMO_FACTOR sqrt(gamma) rho_atmo."""
    g = Grid()
    for d in range(3):
        g.n[d] = int(n[d])
        g.bc[d] = int(bc[d])
        g.x0[d] = float(x0[d])
        g.dx[d] = float(dx[d])
    g.active, g.ng, g.recon = int(active), int(ng), int(recon)
    g.c2p_maxit, g.speed_mode = int(c2p_maxit), int(speed_mode)
    g.gamma_ad, g.kappa, g.c2p_tol = float(gamma_ad), float(kappa), float(c2p_tol)
    g.sigma_model, g.sigma0, g.sigma_exp, g.sigma_Datmo = int(sigma_model), float(sigma0), float(sigma_exp), \
        float(sigma_Datmo)
    g.rho_atmo, g.K_atmo = float(rho_atmo), float(K_atmo)
    return g


def padded_shape(g: Grid):
    gs = [g.ng if (g.active >> d) & 1 else 0 for d in range(3)]
    return (g.n[2] + 2 * gs[2], g.n[1] + 2 * gs[1], g.n[0] + 2 * gs[0])


def interior(g: Grid):
    gs = [g.ng if (g.active >> d) & 1 else 0 for d in range(3)]
    return (slice(gs[2], gs[2] + g.n[2]), slice(gs[1], gs[1] + g.n[1]), slice(gs[0], gs[0] + g.n[0]))


def gamma_imex() -> float:
    return lib().orc_gamma_imex()


# ---------------------------------------------------------------- pointwise
def point_prim2con(P, G, metric=None):
    U = np.zeros(14)
    lib().orc_point_prim2con(_p(None if metric is None else np.ascontiguousarray(metric, float)), G,
                             _p(np.ascontiguousarray(P, float)), _p(U))
    return U


def point_metric(metric):
    gi = np.zeros(9)
    sg = np.zeros(1)
    lib().orc_point_metric(_p(np.ascontiguousarray(metric, float)), _p(gi), _p(sg))
    return gi.reshape(3, 3), float(sg[0])


def point_flux(P, G, sigma, d, metric=None):
    F = np.zeros(14)
    lib().orc_point_flux(_p(None if metric is None else np.ascontiguousarray(metric, float)), G,
                         _p(np.ascontiguousarray(P, float)), sigma, d, _p(F))
    return F


def point_hlle(PL, PR, G, sigma, d, metric=None, mode=0):
    F = np.zeros(14)
    lib().orc_point_hlle(_p(None if metric is None else np.ascontiguousarray(metric, float)), G,
                         _p(np.ascontiguousarray(PL, float)), _p(np.ascontiguousarray(PR, float)), sigma, d, mode,
                         _p(F))
    return F


def point_speeds(metric, d, mode=0):
    """characteristic speeds (lambda_+, lambda_-) of the HLLE flux along d"""
    lp, lm = C.c_double(0), C.c_double(0)
    lib().orc_point_speeds(_p(np.ascontiguousarray(metric, float)), d, mode, C.byref(lp), C.byref(lm))
    return lp.value, lm.value


def point_stiff(v, Ec, Bc, sigma, metric=None):
    R = np.zeros(3)
    lib().orc_point_stiff(_p(None if metric is None else np.ascontiguousarray(metric, float)),
                          _p(np.ascontiguousarray(v, float)), _p(np.ascontiguousarray(Ec, float)),
                          _p(np.ascontiguousarray(Bc, float)), sigma, _p(R))
    return R


def point_esolve(v, Bc, Estar, c, metric=None):
    E = np.zeros(3)
    lib().orc_point_esolve(_p(None if metric is None else np.ascontiguousarray(metric, float)),
                           _p(np.ascontiguousarray(v, float)), _p(np.ascontiguousarray(Bc, float)),
                           _p(np.ascontiguousarray(Estar, float)), c, _p(E))
    return E


def point_coupled(U, Estar, adt, sigma, Pguess, G, metric=None, tol=1e-14, maxit=500):
    P = np.zeros(14)
    E = np.zeros(3)
    it = C.c_int(0)
    st = lib().orc_point_coupled(_p(None if metric is None else np.ascontiguousarray(metric, float)), G,
                                 _p(np.ascontiguousarray(U, float)), _p(np.ascontiguousarray(Estar, float)), adt,
                                 sigma, _p(np.ascontiguousarray(Pguess, float)), tol, maxit, _p(P), _p(E),
                                 C.byref(it))
    return P, E, st, it.value


def point_recover_paper(U, Estar, adt, sigma, Pguess, G, metric=None, tol=1e-14, maxit=500):
    """The paper's recovery iteration as printed (Picard in v, Newton in p)."""
    P = np.zeros(14)
    E = np.zeros(3)
    it = C.c_int(0)
    st = lib().orc_point_recover_paper(_p(None if metric is None else np.ascontiguousarray(metric, float)), G,
                                       _p(np.ascontiguousarray(U, float)), _p(np.ascontiguousarray(Estar, float)),
                                       adt, sigma, _p(np.ascontiguousarray(Pguess, float)), tol, maxit, _p(P), _p(E),
                                       C.byref(it))
    return P, E, st, it.value


def recon(method, f5):
    fm, fp = C.c_double(0), C.c_double(0)
    lib().orc_recon(method, _p(np.ascontiguousarray(f5, float)), C.byref(fm), C.byref(fp))
    return fm.value, fp.value


# --------------------------------------------------------------------- grid
def _chk(g, a, nf):
    shp = padded_shape(g)
    assert a.shape == (nf,) + shp, (a.shape, (nf,) + shp)
    return a


def ghost_fill(g, a):
    a = np.ascontiguousarray(a)
    lib().orc_ghost_fill(C.byref(g), _p(a), a.shape[0])
    return a


def prim2con(g, P, metric=None):
    _chk(g, P, 14)
    U = np.zeros_like(P)
    lib().orc_prim2con(C.byref(g), _p(metric), _p(P), _p(U))
    return U


def con2prim(g, U, Pguess, metric=None):
    P = np.array(Pguess, copy=True)
    st = np.zeros(padded_shape(g), np.int32)
    it = np.zeros(padded_shape(g), np.int32)
    nf = lib().orc_con2prim(C.byref(g), _p(metric), _p(U), _p(Pguess), _p(P), _ip(st), _ip(it))
    return P, st, it, nf


def explicit_rhs(g, P, sigma, metric=None):
    L = np.zeros_like(P)
    lib().orc_explicit_rhs(C.byref(g), _p(metric), _p(P), _p(sigma), _p(L))
    return L


def stage1(g, dt, sigma, Un, Pn, metric=None):
    P1 = np.array(Pn, copy=True)
    U1 = np.array(Un, copy=True)
    R1 = np.zeros((3,) + padded_shape(g))
    st = np.zeros(padded_shape(g), np.int32)
    it = np.zeros(padded_shape(g), np.int32)
    nf = lib().orc_stage1(C.byref(g), _p(metric), dt, _p(sigma), _p(Un), _p(Pn), _p(P1), _p(R1), _p(U1),
                          _ip(st), _ip(it))
    return dict(P1=P1, R1=R1, U1=U1, status=st, iters=it, nfail=nf)


def stage2(g, dt, sigma, Un, P1, R1, metric=None):
    U2 = np.array(Un, copy=True)
    P2 = np.array(P1, copy=True)
    R2 = np.zeros_like(R1)
    F1 = np.zeros_like(Un)
    st = np.zeros(padded_shape(g), np.int32)
    it = np.zeros(padded_shape(g), np.int32)
    nf = lib().orc_stage2(C.byref(g), _p(metric), dt, _p(sigma), _p(Un), _p(P1), _p(R1), _p(U2), _p(P2), _p(R2),
                          _p(F1), _ip(st), _ip(it))
    return dict(U2=U2, P2=P2, R2=R2, F1=F1, status=st, iters=it, nfail=nf)


def final(g, dt, sigma, Un, F1, P2, R1, R2, metric=None):
    U3 = np.array(Un, copy=True)
    P3 = np.array(P2, copy=True)
    st = np.zeros(padded_shape(g), np.int32)
    it = np.zeros(padded_shape(g), np.int32)
    nf = lib().orc_final(C.byref(g), _p(metric), dt, _p(sigma), _p(Un), _p(F1), _p(P2), _p(R1), _p(R2), _p(U3),
                         _p(P3), _ip(st), _ip(it))
    return dict(U=U3, P=P3, status=st, iters=it, nfail=nf)


def step(g, dt, sigma, U, P, metric=None, status=None):
    """One IMEX-SSP2(2,2,2) step in place; returns the number of failed cells.
    status ([Np] int32, optional): the final recovery's per-cell status
    (2: atmosphere)."""
    return lib().orc_step(C.byref(g), _p(metric), dt, _p(sigma), _p(U), _p(P), _ip(status))


def step_tangent(g, dt, sigma, U, dU, P, dsigma=None, metric=None):
    """One step in place on (U, P) in dual numbers: dU (in/out) is the
    directional derivative of U along the input direction (dU, dsigma).
    Returns (failed cells, dP)."""
    dP = np.zeros_like(P)
    nf = lib().orc_step_tangent(C.byref(g), _p(metric), dt, _p(sigma), _p(dsigma), _p(U), _p(dU), _p(P), _p(dP))
    return nf, dP


def max_signal_speed(g, metric=None):
    return lib().orc_max_signal_speed(C.byref(g), _p(metric))


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Thread count of the oracle's later parallel loops."""
    lib().orc_set_num_threads(int(n))
