"""Python binding of libz4c.so (argument marshalling only).

Every computation runs in the HIP kernels of the C-ABI library; this module
converts Python objects to the C structures of ``include/z4c.h`` and device
addresses (integers, e.g. ``torch.Tensor.data_ptr()``), raises on error
statuses, and fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libz4c.so")

OK, EINVAL, ENOGHOST, EALIGN, EHIP, ENOTSUP, ENOMEM, ENODEV = 0, -1, -2, -3, -4, -5, -6, -7
LAPSE_1PLUSLOG, LAPSE_HARMONIC, LAPSE_FROZEN = 0, 1, 2
SHIFT_GAMMADRIVER, SHIFT_FROZEN = 0, 1
ARITH_FP64, ARITH_FP32, ARITH_FP32_NAIVE = 0, 1, 2
ADVECT_CENTRED, ADVECT_LOPSIDED = 0, 1
GHOST_NONE, GHOST_PERIODIC, GHOST_NEIGHBOUR, GHOST_FROZEN = 0, 1, 2, 3
PLAN_NO_DEVICE = 1
STEP_STORED_GHOSTS, STEP_NO_FINAL_FILL, STEP_MONITOR, STEP_LEVEL_EXCHANGE = 1, 2, 4, 8
STEP_SOMMERFELD = 16


class Params(ctypes.Structure):
    _fields_ = [("fd_order", ctypes.c_int), ("ko_sigma", ctypes.c_double),
                ("kappa1", ctypes.c_double), ("kappa2", ctypes.c_double),
                ("eta", ctypes.c_double), ("lapse", ctypes.c_int), ("shift", ctypes.c_int),
                ("advect_gauge", ctypes.c_int), ("chi_floor", ctypes.c_double),
                ("alpha_floor", ctypes.c_double), ("arith", ctypes.c_int),
                ("advection", ctypes.c_int)]


class Block(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_longlong), ("moffset", ctypes.c_longlong),
                ("coffset", ctypes.c_longlong), ("field_stride", ctypes.c_longlong),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("ng", ctypes.c_int), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("dz", ctypes.c_double)]


class RKCoeffs(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("eps", ctypes.c_double), ("g1", ctypes.c_double),
                ("g2", ctypes.c_double), ("g3", ctypes.c_double), ("beta", ctypes.c_double),
                ("read_u1", ctypes.c_int), ("write_u1", ctypes.c_int)]


class Launch(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int), ("tile_z", ctypes.c_int),
                ("persistent", ctypes.c_int), ("waves", ctypes.c_int)]


class StepDesc(ctypes.Structure):
    _fields_ = [("regs", ctypes.c_void_p * 4), ("matter", ctypes.c_void_p),
                ("table", ctypes.POINTER(RKCoeffs)), ("nstages", ctypes.c_int),
                ("dt", ctypes.c_double), ("ghost_policy", ctypes.c_int),
                ("frozen", ctypes.c_void_p), ("flags", ctypes.c_int),
                ("cons", ctypes.c_void_p), ("norms", ctypes.c_void_p)]


# Classic RK4 in the library's three-register stage form.
RK4 = [(1.0, 1.0 / 6.0, 0.0, 0.0, 1.0, 0.5, 0, 1),
       (0.0, 1.0 / 3.0, 0.0, 0.0, 1.0, 0.5, 1, 1),
       (0.0, 1.0 / 3.0, 0.0, 0.0, 1.0, 1.0, 1, 1),
       (0.0, 1.0 / 6.0, 0.0, 1.0, 0.0, 0.0, 1, 0)]
# SSPRK(3,3) (Shu-Osher) in the same form; the accumulator is unused.
SSPRK3 = [(0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0, 0),
          (0.0, 0.0, 0.25, 0.0, 0.75, 0.25, 0, 0),
          (0.0, 0.0, 2.0 / 3.0, 0.0, 1.0 / 3.0, 2.0 / 3.0, 0, 0)]


class MBlock(ctypes.Structure):
    """z4c_mblock of include/z4c_matter.h."""
    _fields_ = [("vs_offset", ctypes.c_longlong), ("vm_offset", ctypes.c_longlong),
                ("vc_stride", ctypes.c_longlong), ("cg_offset", ctypes.c_longlong),
                ("cp_offset", ctypes.c_longlong), ("ca_offset", ctypes.c_longlong),
                ("cq_offset", ctypes.c_longlong), ("cf_offset", ctypes.c_longlong),
                ("cc_stride", ctypes.c_longlong), ("ncx", ctypes.c_int), ("ncy", ctypes.c_int),
                ("ncz", ctypes.c_int), ("ngv", ctypes.c_int), ("ngc", ctypes.c_int),
                ("pad", ctypes.c_int)]


class Fluid(ctypes.Structure):
    """z4c_fluid of include/z4c_matter.h."""
    _fields_ = [("mhd", ctypes.c_int), ("gamma_ad", ctypes.c_double),
                ("chi_floor", ctypes.c_double)]


class C2PParams(ctypes.Structure):
    """z4c_c2p_params of include/z4c_matter.h."""
    _fields_ = [("mhd", ctypes.c_int), ("gamma_ad", ctypes.c_double),
                ("chi_floor", ctypes.c_double), ("rho_atm", ctypes.c_double),
                ("p_atm", ctypes.c_double), ("f_thr", ctypes.c_double),
                ("ut_max", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int)]


class Transfer(ctypes.Structure):
    """z4c_transfer of include/z4c.h."""
    _fields_ = [("coarse", ctypes.c_int), ("fine", ctypes.c_int), ("c0", ctypes.c_int * 3),
                ("lo", ctypes.c_int * 3), ("hi", ctypes.c_int * 3)]


class Z4cError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"z4c status {status}: {message}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIBPATH)
        vp, st = ctypes.c_void_p, ctypes.c_int
        L.z4c_plan_create.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Block), ctypes.c_int,
                                      ctypes.c_int, ctypes.POINTER(vp)]
        L.z4c_plan_destroy.argtypes = [vp]
        L.z4c_plan_set_params.argtypes = [vp, ctypes.POINTER(Params)]
        L.z4c_plan_set_neighbours.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        L.z4c_plan_set_halo.argtypes = [vp, ctypes.c_int, vp]
        L.z4c_plan_set_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(Launch)]
        L.z4c_plan_get_launch.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.POINTER(Launch)]
        L.z4c_rhs.argtypes = [vp, vp, vp, vp, vp]
        L.z4c_rk_stage.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(RKCoeffs),
                                   ctypes.c_double, vp]
        L.z4c_constraints.argtypes = [vp, vp, vp, vp, vp, vp]
        L.z4c_constraints_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
        L.z4c_rk_stage_monitor.argtypes = [vp, vp, vp, vp, vp, vp, ctypes.POINTER(RKCoeffs),
                                           ctypes.c_double, vp, vp, vp]
        L.z4c_ghost_fill.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.z4c_step.argtypes = [vp, ctypes.POINTER(StepDesc), ctypes.POINTER(ctypes.c_int), vp]
        L.z4c_step_graph.argtypes = [vp, ctypes.POINTER(StepDesc), ctypes.POINTER(ctypes.c_int),
                                     vp]
        L.z4c_plan_autotune.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int, vp]
        L.z4c_set_tune_cache.argtypes = [ctypes.c_char_p]
        L.z4c_set_tune_cache.restype = st
        L.z4c_check_finite.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_longlong), vp]
        L.z4c_strerror.argtypes = [st]
        L.z4c_strerror.restype = ctypes.c_char_p
        L.z4c_last_error.restype = ctypes.c_char_p
        L.z4c_plan_tiles.argtypes = [vp]
        L.z4c_plan_tiles.restype = ctypes.c_longlong
        L.z4c_mplan_create.argtypes = [ctypes.POINTER(MBlock), ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(vp)]
        L.z4c_mplan_destroy.argtypes = [vp]
        L.z4c_metric_to_cc.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, vp, vp]
        L.z4c_adm_sources.argtypes = [vp, ctypes.POINTER(Fluid), ctypes.c_int, vp, vp, vp, vp]
        L.z4c_sources_to_vc.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        L.z4c_p2c.argtypes = [vp, ctypes.POINTER(C2PParams), ctypes.c_int, vp, vp, vp, vp]
        L.z4c_c2p.argtypes = [vp, ctypes.POINTER(C2PParams), ctypes.c_int, vp, vp, vp, vp, vp]
        L.z4c_xplan_create.argtypes = [vp, ctypes.POINTER(Transfer), ctypes.c_int,
                                       ctypes.POINTER(Transfer), ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(vp)]
        L.z4c_xplan_destroy.argtypes = [vp]
        L.z4c_prolongate.argtypes = [vp, vp, vp]
        L.z4c_level_transfers.argtypes = [vp, ctypes.POINTER(Loc), ctypes.c_int,
                                          ctypes.POINTER(Transfer), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(Transfer), ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_int)]
        L.z4c_restrict.argtypes = [vp, vp, vp]
        L.z4c_plan_set_level_exchange.argtypes = [vp, ctypes.POINTER(vp), ctypes.c_int]
        L.z4c_plan_set_sommerfeld.argtypes = [vp, vp]
        L.z4c_sommerfeld_rhs.argtypes = [vp, vp, vp, vp]
        L.z4c_sommerfeld_stage.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(RKCoeffs),
                                           ctypes.c_double, vp]
        L.z4c_plan_set_level_exchange.restype = st
        for name in ("z4c_xplan_create", "z4c_xplan_destroy", "z4c_prolongate", "z4c_restrict",
                     "z4c_level_transfers"):
            getattr(L, name).restype = st
        for name in ("z4c_mplan_create", "z4c_mplan_destroy", "z4c_metric_to_cc",
                     "z4c_adm_sources", "z4c_sources_to_vc", "z4c_p2c", "z4c_c2p"):
            getattr(L, name).restype = st
        for name in ("z4c_plan_create", "z4c_plan_destroy", "z4c_plan_set_params", "z4c_plan_set_halo",
                     "z4c_plan_set_neighbours", "z4c_plan_set_launch", "z4c_plan_get_launch",
                     "z4c_rhs", "z4c_rk_stage", "z4c_constraints", "z4c_constraints_noalloc",
                     "z4c_ghost_fill", "z4c_rk_stage_monitor",
                     "z4c_step", "z4c_step_graph", "z4c_plan_autotune", "z4c_check_finite"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def set_tune_cache(path):
    """Autotuning cache file of the process (None: no cache)."""
    _check(lib().z4c_set_tune_cache(None if path is None else str(path).encode()))


def _check(status: int):
    if status != OK:
        raise Z4cError(status, lib().z4c_last_error().decode())


def make_params(p, arith: int = ARITH_FP64) -> Params:
    """C parameters from any object with the scheme-parameter attributes."""
    return Params(int(p.fd_order), float(p.ko_sigma), float(p.kappa1), float(p.kappa2),
                  float(p.eta), int(p.lapse), int(p.shift), int(p.advect_gauge),
                  float(p.chi_floor), float(p.alpha_floor), int(arith),
                  int(getattr(p, "advection", ADVECT_CENTRED)))


def make_blocks(table: np.ndarray):
    """C block array from a structured numpy array with the z4c_block fields."""
    arr = (Block * len(table))()
    for i, r in enumerate(table):
        arr[i] = Block(int(r["offset"]), int(r["moffset"]), int(r["coffset"]),
                       int(r["field_stride"]), int(r["nx"]), int(r["ny"]), int(r["nz"]),
                       int(r["ng"]), float(r["dx"]), float(r["dy"]), float(r["dz"]))
    return arr


def _coeffs(c) -> RKCoeffs:
    if isinstance(c, RKCoeffs):
        return c
    if isinstance(c, dict):
        return RKCoeffs(c["delta"], c["eps"], c["g1"], c["g2"], c["g3"], c["beta"],
                        int(c["read_u1"]), int(c["write_u1"]))
    return RKCoeffs(*c)


def _stream(stream) -> int:
    if stream is None:
        return 0
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


def _ptr(x) -> int:
    if x is None:
        return 0
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x)


class Plan:
    """A validated set of MeshBlocks with device tables (z4c_plan)."""

    def __init__(self, params: Params, blocks, flags: int = 0):
        self._h = ctypes.c_void_p()
        self.nblocks = len(blocks)
        _check(lib().z4c_plan_create(ctypes.byref(params), blocks, self.nblocks, flags,
                                     ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().z4c_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tiles(self) -> int:
        return int(lib().z4c_plan_tiles(self._h))

    def set_params(self, params: Params):
        _check(lib().z4c_plan_set_params(self._h, ctypes.byref(params)))

    def set_neighbours(self, table: np.ndarray):
        t = np.ascontiguousarray(table, dtype=np.int32).reshape(-1)
        _check(lib().z4c_plan_set_neighbours(self._h, t.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int))))

    def set_halo(self, policy, frozen=None):
        _check(lib().z4c_plan_set_halo(self._h, int(policy), _ptr(frozen)))

    def set_level_exchange(self, xplans):
        """Transfer plans (XPlan) of the level jumps, coarsest pair first."""
        arr = (ctypes.c_void_p * max(1, len(xplans)))(*[x._h.value for x in xplans])
        self._levels = list(xplans)   # keep them alive while the plan uses them
        _check(lib().z4c_plan_set_level_exchange(self._h, arr, len(xplans)))

    def set_sommerfeld(self, origins):
        """Radiative outer boundary: coordinates of every block's interior
        point (0, 0, 0), shape (nblocks, 3); None removes it."""
        if origins is None:
            _check(lib().z4c_plan_set_sommerfeld(self._h, None))
            return
        o = np.ascontiguousarray(origins, dtype=np.float64).reshape(-1)
        if o.size != 3 * self.nblocks:
            raise ValueError("origins must hold 3 coordinates per block")
        _check(lib().z4c_plan_set_sommerfeld(self._h, o.ctypes.data))

    def sommerfeld_rhs(self, u, rhs, stream=None):
        _check(lib().z4c_sommerfeld_rhs(self._h, _ptr(u), _ptr(rhs), _stream(stream)))

    def sommerfeld_stage(self, u0_in, u0_out, u1, u2, coeffs, dt, stream=None):
        c = _coeffs(coeffs)
        _check(lib().z4c_sommerfeld_stage(self._h, _ptr(u0_in), _ptr(u0_out), _ptr(u1),
                                          _ptr(u2), ctypes.byref(c), float(dt), _stream(stream)))

    def set_launch(self, nx, ny, nz, tile=(8, 8, 8), persistent=0, waves=2):
        L = Launch(tile[0], tile[1], tile[2], persistent, waves)
        _check(lib().z4c_plan_set_launch(self._h, nx, ny, nz, ctypes.byref(L)))

    def get_launch(self, nx, ny, nz):
        L = Launch()
        _check(lib().z4c_plan_get_launch(self._h, nx, ny, nz, ctypes.byref(L)))
        return (L.tile_x, L.tile_y, L.tile_z), L.persistent, L.waves

    def rhs(self, u, matter, out, stream=None):
        _check(lib().z4c_rhs(self._h, _ptr(u), _ptr(matter), _ptr(out), _stream(stream)))

    def rk_stage(self, u0_in, u0_out, u1, u2, matter, coeffs, dt, stream=None):
        c = _coeffs(coeffs)
        _check(lib().z4c_rk_stage(self._h, _ptr(u0_in), _ptr(u0_out), _ptr(u1), _ptr(u2),
                                  _ptr(matter), ctypes.byref(c), float(dt), _stream(stream)))

    def rk_stage_monitor(self, u0_in, u0_out, u1, u2, matter, coeffs, dt, cons, norms,
                         stream=None):
        """rk_stage plus the constraints of u0_in (cons may be None; norms as
        in constraints), formed inside the stage kernel."""
        c = _coeffs(coeffs)
        _check(lib().z4c_rk_stage_monitor(self._h, _ptr(u0_in), _ptr(u0_out), _ptr(u1),
                                          _ptr(u2), _ptr(matter), ctypes.byref(c), float(dt),
                                          _ptr(cons), _ptr(norms), _stream(stream)))

    def constraints(self, u, matter, cons, norms, stream=None):
        _check(lib().z4c_constraints(self._h, _ptr(u), _ptr(matter), _ptr(cons), _ptr(norms),
                                     _stream(stream)))

    def constraints_noalloc(self, u, matter, cons, norms, stream=None):
        """constraints with the library's static scratch (allocates nothing)."""
        _check(lib().z4c_constraints_noalloc(self._h, _ptr(u), _ptr(matter), _ptr(cons),
                                             _ptr(norms), _stream(stream)))

    def ghost_fill(self, policy, u, frozen=None, stream=None):
        _check(lib().z4c_ghost_fill(self._h, int(policy), _ptr(u), _ptr(frozen),
                                    _stream(stream)))

    def _desc(self, regs, matter, table, dt, ghost, frozen, flags=0, cons=None, norms=None):
        tab = (RKCoeffs * len(table))(*[_coeffs(c) for c in table])
        d = StepDesc()
        for r in range(4):
            d.regs[r] = _ptr(regs[r]) if r < len(regs) else 0
        d.matter = _ptr(matter)
        d.table = tab
        d.nstages = len(table)
        d.dt = float(dt)
        d.ghost_policy = int(ghost)
        d.frozen = _ptr(frozen)
        d.flags = int(flags)
        d.cons = _ptr(cons)
        d.norms = _ptr(norms)
        return d, tab

    def step(self, regs, matter, table, dt, ghost, frozen=None, stream=None, graph=False,
             flags=0, cons=None, norms=None) -> int:
        """One Runge-Kutta step; returns the index of the register holding the
        new state.  With flags & STEP_MONITOR the constraints of the state on
        entry go to cons (or None) and norms."""
        d, tab = self._desc(regs, matter, table, dt, ghost, frozen, flags, cons, norms)
        res = ctypes.c_int(-1)
        fn = lib().z4c_step_graph if graph else lib().z4c_step
        _check(fn(self._h, ctypes.byref(d), ctypes.byref(res), _stream(stream)))
        return res.value

    def autotune(self, u0, u0_out, u1, matter, reps=3, stream=None):
        _check(lib().z4c_plan_autotune(self._h, _ptr(u0), _ptr(u0_out), _ptr(u1), _ptr(matter),
                                       int(reps), _stream(stream)))

    def check_finite(self, u, stream=None) -> int:
        n = ctypes.c_longlong(0)
        _check(lib().z4c_check_finite(self._h, _ptr(u), ctypes.byref(n), _stream(stream)))
        return n.value


def plan_for(batch, arith: int = ARITH_FP64, flags: int = 0) -> Plan:
    """Plan for a workload batch (its block table, parameters, neighbours)."""
    p = Plan(make_params(batch.params, arith), make_blocks(batch.block_table()), flags)
    if batch.neighbours is not None:
        p.set_neighbours(batch.neighbours)
        if getattr(batch, "sommerfeld", False):
            p.set_sommerfeld(batch.origins())
    return p


def make_mblocks(table: np.ndarray):
    """C z4c_mblock array from a structured numpy array with its fields."""
    arr = (MBlock * len(table))()
    names = [f[0] for f in MBlock._fields_]
    for i, r in enumerate(table):
        arr[i] = MBlock(*[int(r[n]) for n in names])
    return arr


class MPlan:
    """Matter-coupling plan (z4c_mplan): block table and tile lists on the
    device for z4c_metric_to_cc, z4c_adm_sources and z4c_sources_to_vc."""

    def __init__(self, table: np.ndarray, flags: int = 0):
        self._h = ctypes.c_void_p()
        blocks = make_mblocks(table)
        _check(lib().z4c_mplan_create(blocks, len(table), flags, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().z4c_mplan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def metric_to_cc(self, order, ext, u, geom, stream=None):
        _check(lib().z4c_metric_to_cc(self._h, int(order), int(ext), _ptr(u), _ptr(geom),
                                      _stream(stream)))

    def adm_sources(self, mhd, gamma_ad, chi_floor, ext, geom, prim, adm, stream=None):
        fl = Fluid(int(mhd), float(gamma_ad), float(chi_floor))
        _check(lib().z4c_adm_sources(self._h, ctypes.byref(fl), int(ext), _ptr(geom), _ptr(prim),
                                     _ptr(adm), _stream(stream)))

    def p2c(self, c, ext, geom, prim, cons, stream=None):
        _check(lib().z4c_p2c(self._h, ctypes.byref(c), int(ext), _ptr(geom), _ptr(prim),
                             _ptr(cons), _stream(stream)))

    def c2p(self, c, ext, geom, cons, prim, status=None, stream=None):
        _check(lib().z4c_c2p(self._h, ctypes.byref(c), int(ext), _ptr(geom), _ptr(cons),
                             _ptr(prim), _ptr(status), _stream(stream)))

    def sources_to_vc(self, order, adm, matter, stream=None):
        _check(lib().z4c_sources_to_vc(self._h, int(order), _ptr(adm), _ptr(matter),
                                       _stream(stream)))


def c2p_params(mhd=1, gamma_ad=2.0, chi_floor=1e-6, rho_atm=1e-13, p_atm=None, f_thr=1.0,
               ut_max=20.0, tol=1e-15, max_iter=100) -> C2PParams:
    """C2P parameters; p_atm defaults to the polytrope p = 100 rho^Gamma at rho_atm."""
    if p_atm is None:
        p_atm = 100.0 * rho_atm ** gamma_ad
    return C2PParams(int(mhd), float(gamma_ad), float(chi_floor), float(rho_atm), float(p_atm),
                     float(f_thr), float(ut_max), float(tol), int(max_iter))


def mplan_for(mbatch, flags: int = 0) -> MPlan:
    return MPlan(mbatch.table(), flags)


class Loc(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("o", ctypes.c_int * 3)]


def level_transfers(plan: "Plan", locs, coarse_level: int):
    """z4c_level_transfers: (prolongations, restrictions) of the level jump
    coarse_level -> coarse_level + 1 as lists of dicts (coarse, fine, c0, lo,
    hi), from locs = [(level, (ox, oy, oz)), ...] per block of the plan."""
    L = (Loc * len(locs))()
    for b, (lev, o) in enumerate(locs):
        L[b] = Loc(int(lev), (ctypes.c_int * 3)(*[int(v) for v in o]))
    np_, nr = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().z4c_level_transfers(plan._h, L, int(coarse_level), None, 0, ctypes.byref(np_),
                                     None, 0, ctypes.byref(nr)))
    P = (Transfer * max(np_.value, 1))()
    R = (Transfer * max(nr.value, 1))()
    _check(lib().z4c_level_transfers(plan._h, L, int(coarse_level), P, np_.value,
                                     ctypes.byref(np_), R, nr.value, ctypes.byref(nr)))
    conv = lambda t: dict(coarse=t.coarse, fine=t.fine, c0=list(t.c0), lo=list(t.lo),  # noqa: E731
                          hi=list(t.hi))
    return [conv(P[k]) for k in range(np_.value)], [conv(R[k]) for k in range(nr.value)]


def make_transfers(items):
    """C z4c_transfer array from dicts with coarse, fine, c0, lo, hi."""
    arr = (Transfer * max(len(items), 1))()
    for k, t in enumerate(items):
        arr[k] = Transfer(int(t["coarse"]), int(t["fine"]), (ctypes.c_int * 3)(*t["c0"]),
                          (ctypes.c_int * 3)(*t["lo"]), (ctypes.c_int * 3)(*t["hi"]))
    return arr


class XPlan:
    """Transfers between refinement levels (z4c_xplan) over the blocks of a
    Plan, which must stay alive as long as the XPlan."""

    def __init__(self, plan: Plan, prolong, restrict, order: int, flags: int = 0):
        self._h = ctypes.c_void_p()
        self._plan = plan
        p, r = make_transfers(prolong), make_transfers(restrict)
        _check(lib().z4c_xplan_create(plan._h, p, len(prolong), r, len(restrict), int(order),
                                      int(flags), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            lib().z4c_xplan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prolongate(self, u, stream=None):
        _check(lib().z4c_prolongate(self._h, _ptr(u), _stream(stream)))

    def restrict(self, u, stream=None):
        _check(lib().z4c_restrict(self._h, _ptr(u), _stream(stream)))
