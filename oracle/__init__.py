"""ctypes wrapper around the CPU FP64 oracle (``mcc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg.  It imports nothing from the GPU package.

All arrays are numpy; velocities are updated in place, as in the C code.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcc_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

TA77 = 0
N97 = 1
ORDER_N = 0
NXN = 1
DUPLICITY = 2
HARD_SPHERE = 2   # method: isotropic collisions with probability 1 - exp(-s)

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc, FP64, no floating-point contraction."""
    if force or not os.path.exists(LIB_PATH) or (
            os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-std=gnu11", "-O2", "-ffp-contract=off",
                               "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-o",
                               tmp, _SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32, i64, u32, u64, f64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_shuffle.argtypes = [i32, u32, u64, u64, i32, i32, P]
        L.oracle_shuffle.restype = None
        L.oracle_n97_M.argtypes = [f64]
        L.oracle_n97_M.restype = f64
        L.oracle_n97_L.argtypes = [f64]
        L.oracle_n97_L.restype = f64
        L.oracle_n97_A.argtypes = [f64]
        L.oracle_n97_A.restype = f64
        L.oracle_sample_angle.argtypes = [i32, f64, f64, f64, P]
        L.oracle_sample_angle.restype = f64
        L.oracle_rotate.argtypes = [P, f64, f64, f64, P]
        L.oracle_rotate.restype = None
        L.oracle_energy_pair_nr.argtypes = [f64, f64, f64, P, P]
        L.oracle_energy_pair_nr.restype = None
        L.oracle_energy_pair_rel.argtypes = [f64, f64, f64, f64, P, P]
        L.oracle_energy_pair_rel.restype = C.c_int
        L.oracle_rel_kecm.argtypes = [f64, f64, P, P, f64]
        L.oracle_rel_kecm.restype = f64
        L.oracle_scatter_pair.argtypes = [i32, i32, f64, f64, f64, f64, f64, f64, f64,
                                          u64, u64, u32, i32, u32, f64, f64, f64, f64,
                                          f64, f64, P, P]
        L.oracle_scatter_pair.restype = None
        L.oracle_collide_sorted.argtypes = (
            [i64, i32, i32, P, P, P, i32, P, P, P, P, P, P, P, f64, f64, f64, u64, u64,
             i32, i32, i32, i32, i32, i32, i32, f64, f64, f64, P, i32, P, P, P, P, i32])
        L.oracle_collide_sorted.restype = C.c_int
        L.oracle_collide.argtypes = (
            [i64, P, P, i32, i32, P, P, i32, P, P, P, P, P, P, P, f64, f64, f64, u64, u64,
             i32, i32, i32, i32, i32, i32, i32, f64, f64, f64, P, P, P, P, i32])
        L.oracle_collide.restype = C.c_int
        L.oracle_collide_sorted_traced.argtypes = (
            [i64, i32, i32, P, P, P, i32, P, P, P, P, P, P, f64, f64, f64, u64, u64,
             i32, i32, i32, f64, f64, P, P, P, P])
        L.oracle_collide_sorted_traced.restype = C.c_int
        L.oracle_bin.argtypes = [i64, P, P, i32, i32, P, P]
        L.oracle_bin.restype = C.c_int
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's cell loop (default 1).  Cells are independent
    and every random number is keyed by its cell, so results are the same,
    bit for bit, for every thread count."""
    lib().oracle_set_threads(int(n))


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def philox(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.array(ctr, dtype=np.uint32)
    k = np.array(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def shuffle(n: int, cell: int, seed: int, step: int, coll: int, slot: int) -> np.ndarray:
    out = np.zeros(max(n, 1), dtype=np.int32)
    lib().oracle_shuffle(n, cell, seed, step, coll, slot, _p(out))
    return out[:n]


def n97_M(A: float) -> float:
    return lib().oracle_n97_M(A)


def n97_A(s: float) -> float:
    return lib().oracle_n97_A(s)


def sample_angle(method: int, s: float, u0: float, u1: float) -> Tuple[float, float]:
    st = C.c_double(0.0)
    oc = lib().oracle_sample_angle(method, s, u0, u1, C.byref(st))
    return oc, st.value


def rotate(u, st: float, oc: float, phi: float) -> np.ndarray:
    u = _f64(u)
    du = np.zeros(3)
    lib().oracle_rotate(_p(u), st, oc, phi, _p(du))
    return du


def energy_pair_nr(m1, m2, U, v1, v2):
    v1 = _f64(v1).copy()
    v2 = _f64(v2).copy()
    lib().oracle_energy_pair_nr(m1, m2, U, _p(v1), _p(v2))
    return v1, v2


def energy_pair_rel(m1, m2, U, c, u1, u2):
    u1 = _f64(u1).copy()
    u2 = _f64(u2).copy()
    ok = lib().oracle_energy_pair_rel(m1, m2, U, c, _p(u1), _p(u2))
    return bool(ok), u1, u2


def rel_kecm(m1, m2, u1, u2, c):
    return lib().oracle_rel_kecm(m1, m2, _p(_f64(u1)), _p(_f64(u2)), c)


def scatter_pair(vi, vj, *, mi, qi, mj, qj, wi, wj, nmin, dt, lnL, method=N97,
                 relativistic=False, s_factor=1.0, dV=1.0, eps0=1.0, c=math.inf,
                 seed=1, step=0, cell=0, coll=0, pair=0):
    vi = _f64(vi).copy()
    vj = _f64(vj).copy()
    lib().oracle_scatter_pair(method, int(relativistic), s_factor, nmin, dV, dt, lnL,
                              eps0, c, seed, step, cell, coll, pair, mi, qi, mj, qj,
                              wi, wj, _p(vi), _p(vj))
    return vi, vj


class OracleError(RuntimeError):
    pass


def _coll_arrays(collisions):
    ca = np.array([c[0] for c in collisions], dtype=np.int32)
    cb = np.array([c[1] for c in collisions], dtype=np.int32)
    return ca, cb


def _sigma(cross_section, collisions):
    """Per-collision cross-sections: the argument, else the third entry of
    (a, b, sigma) collision tuples, else none."""
    n_coll = len(collisions)
    if cross_section is None:
        if n_coll and all(len(c) > 2 for c in collisions):
            return _f64([c[2] for c in collisions]).copy()
        return None
    sg = _f64(np.broadcast_to(np.asarray(cross_section, dtype=np.float64), (n_coll,)))
    return sg.copy()


def collide_sorted(offsets, mass, charge, collisions, w, vx, vy, vz, *, dt,
                   coulomb_log, seed, step, method=N97, relativistic=False,
                   correction=True, sort_by_weight=True, max_passes=1,
                   keep_on_fail=False, f_E=0.05, eps0=1.0, c=math.inf,
                   cell_volume=1.0, cells: Optional[Sequence[int]] = None,
                   n_cells: Optional[int] = None, pairing: int = ORDER_N,
                   cross_section=None, uniform23: bool = False) -> dict:
    """One step on (cell, species)-grouped arrays; vx, vy, vz updated in place.
    pairing: ORDER_N (Sec. 3.2), NXN (every pair once, Sec. 3.1) or
    DUPLICITY (order-N pairs, inter-species s with N_max / D, the variant the
    paper attributes to Higginson et al.).
    method HARD_SPHERE needs cross_section (one per collision, or a scalar):
    charges, coulomb_log and eps0 are then unused.
    uniform23: draw the angle, Box-Muller phase and azimuth uniforms from the
    top 23 bits of their words, (k + 1/2) 2^-23, as the FP32-kinematics form
    does (the acceptance keeps the 32-bit uniform)."""
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    mass = _f64(mass)
    charge = _f64(charge)
    S = mass.shape[0]
    if n_cells is None:
        n_cells = (offsets.shape[0] - 1) // S
    for a in (w, vx, vy, vz):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    ca, cb = _coll_arrays(collisions)
    cv = None
    cvs = float(cell_volume) if np.isscalar(cell_volume) else 0.0
    if not np.isscalar(cell_volume):
        cv = _f64(cell_volume)
    cl = None if cells is None else np.ascontiguousarray(cells, dtype=np.int32)
    sg = _sigma(cross_section, collisions)
    counters = np.zeros(4, dtype=np.int64)
    diag = np.zeros(2)
    ccp = np.zeros(max(n_cells, 1), dtype=np.int32)
    if not math.isfinite(c):
        c = 0.0 if not relativistic else c
    rc = lib().oracle_collide_sorted(
        w.shape[0], n_cells, S, _p(offsets), _p(mass), _p(charge), len(collisions),
        _p(ca), _p(cb), _p(w), _p(vx), _p(vy), _p(vz), _p(cv), cvs, dt, coulomb_log,
        seed, step, method, int(pairing), int(relativistic), int(correction),
        int(sort_by_weight), max_passes, int(keep_on_fail), f_E, eps0, c, _p(cl),
        0 if cl is None else cl.shape[0], _p(counters), _p(diag), _p(ccp), _p(sg),
        int(uniform23))
    if rc != 0:
        raise OracleError("oracle_collide_sorted returned %d" % rc)
    return dict(pairs=int(counters[0]), corr_pairs=int(counters[1]),
                failed=int(counters[2]), collisions=int(counters[3]),
                max_rel_dP=float(diag[0]), max_rel_dE=float(diag[1]),
                cell_corr_pairs=ccp[:n_cells])


def collide(cells, species, n_cells, mass, charge, collisions, w, vx, vy, vz, *, dt,
            coulomb_log, seed, step, method=N97, relativistic=False, correction=True,
            sort_by_weight=True, max_passes=1, keep_on_fail=False, f_E=0.05, eps0=1.0,
            c=math.inf, cell_volume=1.0, pairing: int = ORDER_N, cross_section=None,
            uniform23: bool = False) -> dict:
    """One step on particles in any order; vx, vy, vz updated in place."""
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    species = np.ascontiguousarray(species, dtype=np.int32)
    mass = _f64(mass)
    charge = _f64(charge)
    S = mass.shape[0]
    ca, cb = _coll_arrays(collisions)
    sg = _sigma(cross_section, collisions)
    cv = None
    cvs = float(cell_volume) if np.isscalar(cell_volume) else 0.0
    if not np.isscalar(cell_volume):
        cv = _f64(cell_volume)
    counters = np.zeros(4, dtype=np.int64)
    diag = np.zeros(2)
    ccp = np.zeros(max(n_cells, 1), dtype=np.int32)
    if not math.isfinite(c):
        c = 0.0 if not relativistic else c
    rc = lib().oracle_collide(
        w.shape[0], _p(cells), _p(species), n_cells, S, _p(mass), _p(charge),
        len(collisions), _p(ca), _p(cb), _p(w), _p(vx), _p(vy), _p(vz), _p(cv), cvs,
        dt, coulomb_log, seed, step, method, int(pairing), int(relativistic),
        int(correction), int(sort_by_weight), max_passes, int(keep_on_fail), f_E, eps0, c,
        _p(counters), _p(diag), _p(ccp), _p(sg), int(uniform23))
    if rc != 0:
        raise OracleError("oracle_collide returned %d" % rc)
    return dict(pairs=int(counters[0]), corr_pairs=int(counters[1]),
                failed=int(counters[2]), collisions=int(counters[3]),
                max_rel_dP=float(diag[0]), max_rel_dE=float(diag[1]),
                cell_corr_pairs=ccp[:n_cells])


def bin_particles(cells, species, n_cells, n_species):
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    species = np.ascontiguousarray(species, dtype=np.int32)
    off = np.zeros(n_cells * n_species + 1, dtype=np.int64)
    perm = np.zeros(max(cells.shape[0], 1), dtype=np.int64)
    rc = lib().oracle_bin(cells.shape[0], _p(cells), _p(species), n_cells, n_species,
                          _p(off), _p(perm))
    if rc != 0:
        raise OracleError("oracle_bin returned %d" % rc)
    return off, perm[:cells.shape[0]]


def run_workload(wl, steps: int = 1, first_step: int = 0, cells=None, **over) -> dict:
    """Advance a workload (from the input-generator module) by `steps` steps."""
    kw = dict(dt=wl.dt, coulomb_log=wl.coulomb_log, seed=wl.seed, method=wl.method,
              relativistic=wl.relativistic, c=wl.c, eps0=wl.eps0,
              cell_volume=wl.cell_volume, f_E=wl.f_E)
    kw.update(over)
    st = None
    for k in range(steps):
        st = collide_sorted(wl.offsets, wl.mass, wl.charge, wl.collisions, wl.w,
                            wl.vx, wl.vy, wl.vz, step=first_step + k, cells=cells,
                            n_cells=wl.n_cells, **kw)
    return st


def n97_L(A: float) -> float:
    return lib().oracle_n97_L(A)


def collide_sorted_traced(wl, step=0, sort_by_weight=True):
    """One step of a workload with post-scatter / post-momentum states and the
    energy violation and its partition recorded (test hook)."""
    n = wl.n
    vps = np.zeros(3 * n)
    vpm = np.zeros(3 * n)
    nc = len(wl.collisions)
    dE = np.zeros(wl.n_cells * nc)
    dEs = np.zeros(2 * wl.n_cells * nc)
    ca, cb = _coll_arrays(wl.collisions)
    c = wl.c if wl.relativistic else 0.0
    rc = lib().oracle_collide_sorted_traced(
        n, wl.n_cells, wl.n_species, _p(wl.offsets), _p(_f64(wl.mass)),
        _p(_f64(wl.charge)), nc, _p(ca), _p(cb), _p(wl.w), _p(wl.vx), _p(wl.vy),
        _p(wl.vz), float(wl.cell_volume), wl.dt, wl.coulomb_log, wl.seed, step,
        wl.method, int(wl.relativistic), int(sort_by_weight), wl.f_E, c, _p(vps),
        _p(vpm), _p(dE), _p(dEs))
    if rc != 0:
        raise OracleError("oracle_collide_sorted_traced returned %d" % rc)
    return dict(vps=vps.reshape(3, n), vpm=vpm.reshape(3, n),
                dE=dE.reshape(wl.n_cells, nc), dEs=dEs.reshape(wl.n_cells, nc, 2))
