"""Python wrapper of the FP64 CPU oracle (``z4c_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the GPU library; the only common module is the seeded input
generator (``paper_2311_04989_amd.workloads``), which holds no arithmetic of
the method.

The oracle's own Runge-Kutta tables are defined here (classic RK4 and the
Shu-Osher SSPRK(3,3) that the paper's "3rd order Runge-Kutta" is read as).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from paper_2311_04989_amd.workloads import NF, NM, NC, BLOCK_DTYPE, GHOST_NONE, \
    GHOST_PERIODIC, GHOST_NEIGHBOUR, GHOST_FROZEN

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "z4c_oracle.c")
LIB = os.path.join(HERE, "libz4c_oracle.so")
LIB_EXT = os.path.join(HERE, "libz4c_oracle_ext.so")
# FP32-arithmetic references of the right-hand side: float algebra with the
# stencil differences formed in double (mixed), or with the samples rounded to
# float first (naive).  They measure what FP32 arithmetic itself costs.
LIB_F32 = os.path.join(HERE, "libz4c_oracle_f32.so")
LIB_F32N = os.path.join(HERE, "libz4c_oracle_f32n.so")
_PATHS = {"f64": LIB, "ext": LIB_EXT, "f32": LIB_F32, "f32naive": LIB_F32N}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP, no FMA contraction), with
    double as working type, with x87 extended precision, and the two FP32
    references."""
    for path, extra in ((LIB, []), (LIB_EXT, ["-DORACLE_EXTENDED"]), (LIB_F32, ["-DORACLE_FP32"]),
                        (LIB_F32N, ["-DORACLE_FP32", "-DORACLE_NAIVE"])):
        if force or not os.path.exists(path):
            cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                   "-fPIC", "-shared", "-Wall"] + extra + ["-o", path + ".tmp", SRC, "-lm"]
            subprocess.check_call(cmd)
            os.replace(path + ".tmp", path)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int), ("ko_sigma", ctypes.c_double),
                ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double),
                ("eta", ctypes.c_double), ("lapse", ctypes.c_int), ("shift", ctypes.c_int),
                ("advect_gauge", ctypes.c_int), ("chi_floor", ctypes.c_double),
                ("alpha_floor", ctypes.c_double), ("advection", ctypes.c_int)]


class _RK(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("eps", ctypes.c_double), ("g1", ctypes.c_double),
                ("g2", ctypes.c_double), ("g3", ctypes.c_double), ("beta", ctypes.c_double),
                ("read_u1", ctypes.c_int), ("write_u1", ctypes.c_int)]


# Classic RK4 as 3-register stages:  u1 <- [u1] + delta u0 + eps dt k,
# u0' <- g1 u0 + g2 u1 + g3 u2 + beta dt k   (u2 = y_n, u0 = stage state).
RK4 = [
    dict(delta=1.0, eps=1.0 / 6.0, g1=0.0, g2=0.0, g3=1.0, beta=0.5, read_u1=0, write_u1=1),
    dict(delta=0.0, eps=1.0 / 3.0, g1=0.0, g2=0.0, g3=1.0, beta=0.5, read_u1=1, write_u1=1),
    dict(delta=0.0, eps=1.0 / 3.0, g1=0.0, g2=0.0, g3=1.0, beta=1.0, read_u1=1, write_u1=1),
    dict(delta=0.0, eps=1.0 / 6.0, g1=0.0, g2=1.0, g3=0.0, beta=0.0, read_u1=1, write_u1=0),
]
# SSPRK(3,3):  v1 = y + dt L(y);  v2 = 3/4 y + 1/4 v1 + 1/4 dt L(v1);
#              y' = 1/3 y + 2/3 v2 + 2/3 dt L(v2).   (u1 unused)
SSPRK3 = [
    dict(delta=0.0, eps=0.0, g1=1.0, g2=0.0, g3=0.0, beta=1.0, read_u1=0, write_u1=0),
    dict(delta=0.0, eps=0.0, g1=0.25, g2=0.0, g3=0.75, beta=0.25, read_u1=0, write_u1=0),
    dict(delta=0.0, eps=0.0, g1=2.0 / 3.0, g2=0.0, g3=1.0 / 3.0, beta=2.0 / 3.0,
         read_u1=0, write_u1=0),
]

_libs = {}


def lib(ext=False):
    """The FP64 oracle, or (ext=True) the same source in extended precision;
    ext may also name a build: "f64", "ext", "f32", "f32naive"."""
    ext = {False: "f64", True: "ext"}.get(ext, ext)
    if ext not in _libs:
        path = _PATHS[ext]
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_rhs.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_int, dp, dp,
                              dp, ctypes.c_int]
        L.orc_rk_stage.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_int, dp,
                                   dp, dp, dp, dp, ctypes.POINTER(_RK), ctypes.c_double,
                                   ctypes.c_int]
        L.orc_constraints.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_int,
                                      dp, dp, dp, dp, ctypes.c_int]
        L.orc_ghost_fill.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), dp, dp]
        L.orc_derivs.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, dp, dp]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_lopsided_weights.argtypes = [ctypes.c_int, dp]
        L.orc_sommerfeld.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp, dp, dp,
                                     ctypes.POINTER(_RK), ctypes.c_double]
        _libs[ext] = L
    return _libs[ext]


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(p) -> _Params:
    return _Params(int(p.fd_order), float(p.ko_sigma), float(p.kappa1), float(p.kappa2),
                   float(p.eta), int(p.lapse), int(p.shift), int(p.advect_gauge),
                   float(p.chi_floor), float(p.alpha_floor),
                   int(getattr(p, "advection", 0)))


def lopsided_weights(p: int) -> np.ndarray:
    """The oracle's lopsided first-derivative weights of order p (units 1/h)
    at offsets -p/2+1 .. p/2+1 (the stencil for beta > 0)."""
    w = np.zeros(p + 1)
    if lib().orc_lopsided_weights(int(p), _dp(w)) != 0:
        raise ValueError("order must be 4 or 6")
    return w


def max_threads() -> int:
    return int(lib().orc_max_threads())


def rhs(batch, u=None, params=None, nthreads: int = 0, ext=False) -> np.ndarray:
    """Right-hand side of all blocks; ghost entries of the result are 0.
    ext=True: extended precision; ext="f32" / "f32naive": the FP32-arithmetic
    references (mixed / naive differences)."""
    u = batch.u if u is None else u
    out = np.zeros_like(u)
    tab = batch.block_table()
    P = _params(params or batch.params)
    lib(ext).orc_rhs(ctypes.byref(P), tab.ctypes.data, len(batch.blocks), _dp(u),
                  _dp(batch.matter), _dp(out), nthreads)
    return out


def rk_stage(batch, u0, u0_out, u1, u2, coeffs: dict, dt: float, params=None,
             nthreads: int = 0, ext: bool = False):
    tab = batch.block_table()
    P = _params(params or batch.params)
    c = _RK(**coeffs)
    lib(ext).orc_rk_stage(ctypes.byref(P), tab.ctypes.data, len(batch.blocks), _dp(u0),
                       _dp(u0_out), _dp(u1), _dp(u2), _dp(batch.matter), ctypes.byref(c),
                       float(dt), nthreads)


def constraints(batch, u=None, params=None, nthreads: int = 0, want_fields: bool = True,
                ext: bool = False):
    """Returns (cons, norms): cons in the 8-field layout (None if not wanted),
    norms of shape (nblocks, 8, 2) = (L1, L2^2) with volume element dx dy dz."""
    u = batch.u if u is None else u
    tab = batch.block_table()
    P = _params(params or batch.params)
    cons = np.zeros(batch.total_c) if want_fields else None
    norms = np.zeros(len(batch.blocks) * 16)
    lib(ext).orc_constraints(ctypes.byref(P), tab.ctypes.data, len(batch.blocks), _dp(u),
                          _dp(batch.matter), _dp(cons), _dp(norms), nthreads)
    return cons, norms.reshape(len(batch.blocks), 8, 2)


def ghost_fill(batch, u, policy=None):
    policy = batch.ghost if policy is None else policy
    if policy == GHOST_NONE:
        return
    tab = batch.block_table()
    nbr = batch.neighbours
    if policy == GHOST_NEIGHBOUR:
        nbr = np.ascontiguousarray(nbr, dtype=np.int32)
        nptr = nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    else:
        nptr = None
    lib().orc_ghost_fill(int(policy), tab.ctypes.data, len(batch.blocks), nptr, _dp(u),
                         _dp(batch.frozen))


def derivs(block, field: np.ndarray, fd_order: int, ko_sigma: float = 1.0) -> np.ndarray:
    """Operator probe on one field of shape block.shape: returns (12, nz, ny, nx)
    = D1x D1y D1z D2xx D2xy D2xz D2yy D2yz D2zz KOx KOy KOz."""
    from paper_2311_04989_amd.workloads import Params
    tab = np.zeros(1, dtype=BLOCK_DTYPE)
    tab[0] = (0, 0, 0, block.npts, block.nx, block.ny, block.nz, block.ng,
              block.dx, block.dy, block.dz)
    f = np.ascontiguousarray(field, dtype=np.float64).reshape(-1)
    out = np.zeros(12 * block.ninterior)
    P = _params(Params(fd_order=fd_order, ko_sigma=ko_sigma))
    lib().orc_derivs(ctypes.byref(P), tab.ctypes.data, _dp(f), _dp(out))
    return out.reshape(12, block.nz, block.ny, block.nx)


def _sommerfeld(batch, u0, rhs, u0_out, u1, u2, coeffs, dt, params, ext):
    nbr = np.ascontiguousarray(batch.neighbours, dtype=np.int32)
    x0 = np.ascontiguousarray(batch.origins())
    tab = batch.block_table()
    P = _params(params or batch.params)
    c = _RK(**(coeffs or RK4[0]))
    lib(ext).orc_sommerfeld(ctypes.byref(P), tab.ctypes.data, len(batch.blocks),
                            nbr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(x0), _dp(u0),
                            _dp(rhs), _dp(u0_out), _dp(u1), _dp(u2), ctypes.byref(c), float(dt))


def sommerfeld_rhs(batch, u=None, params=None, ext=False) -> np.ndarray:
    """Radiative-law d_t u at the outer ghost points (neighbour entry -1) of
    every block; every other entry of the result is 0."""
    u = batch.u if u is None else u
    out = np.zeros_like(u)
    _sommerfeld(batch, u, out, None, None, None, None, 0.0, params, ext)
    return out


def sommerfeld_stage(batch, u0, u0_out, u1, u2, coeffs: dict, dt: float, params=None,
                     ext=False):
    """One Runge-Kutta stage of the outer ghost points by the radiative law
    (combination and enforcement as rk_stage); other points are untouched."""
    _sommerfeld(batch, u0, None, u0_out, u1, u2, coeffs, dt, params, ext)


def rk_step(batch, u, table=None, dt=None, params=None, nthreads: int = 0, ext: bool = False):
    """One full Runge-Kutta step of every block with the ghost policy of the
    batch applied after each stage (with batch.sommerfeld, the outer ghost
    points advance by the radiative law in every stage first).  Returns the
    new state (a new array)."""
    table = RK4 if table is None else table
    dt = batch.dt if dt is None else dt
    y = u
    u1 = np.zeros_like(u)
    cur = u
    for s, c in enumerate(table):
        nxt = cur.copy()   # ghosts carried over, interior overwritten
        rk_stage(batch, cur, nxt, u1, y, c, dt, params=params, nthreads=nthreads, ext=ext)
        if getattr(batch, "sommerfeld", False):
            if batch.frozen is not None:
                raise ValueError("radiative outer ghosts and a frozen array exclude each other")
            sommerfeld_stage(batch, cur, nxt, u1, y, c, dt, params=params, ext=ext)
        ghost_fill(batch, nxt)
        cur = nxt
    return cur
