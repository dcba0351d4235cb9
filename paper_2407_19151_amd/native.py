"""ctypes binding of libmcc_hip.so (include/mcc.h): argument marshalling only.

Every step of the collision path runs in the library's HIP kernels; this
module turns torch device tensors into pointers and the current torch stream
into the library's stream.  If the library is missing it raises; there is no
fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import sys
from typing import Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcc_hip.so")

MCC_TA77, MCC_N97, MCC_HARD_SPHERE = 0, 1, 2
MCC_FP64, MCC_FP32_KINEMATICS = 0, 1
MCC_FAIL_RESET, MCC_FAIL_KEEP = 0, 1
MCC_PAIRING_ORDER_N, MCC_PAIRING_NXN, MCC_PAIRING_DUPLICITY = 0, 1, 2
MCC_MAX_SPECIES = 8
MCC_MAX_COLLISIONS = 32
MCC_MAX_CELL = 32768

STATUS = {0: "ok", -1: "invalid argument", -2: "device out of memory",
          -3: "HIP runtime error", -4: "unsupported combination",
          -5: "device-side data check failed"}

EXPORTS = ["mcc_default_params", "mcc_status_string", "mcc_create", "mcc_set_stream",
           "mcc_set_variant",
           "mcc_destroy", "mcc_device_error", "mcc_collide_sorted", "mcc_collide",
           "mcc_bin", "mcc_rebin", "mcc_rebin_out", "mcc_plan_create", "mcc_plan_run",
           "mcc_plan_describe",
           "mcc_plan_destroy", "mcc_sample_angles", "mcc_plan_run_bucket",
           "mcc_collide_sorted_jvp", "mcc_collide_adjoint", "mcc_collide_sorted_noalloc"]


class mcc_species(C.Structure):
    _fields_ = [("mass", C.c_double), ("charge", C.c_double)]


class mcc_collision(C.Structure):
    _fields_ = [("a", C.c_int32), ("b", C.c_int32), ("cross_section", C.c_double)]


class mcc_params(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("relativistic", C.c_int32),
                ("moment_correction", C.c_int32), ("sort_by_weight", C.c_int32),
                ("max_passes", C.c_int32), ("on_failure", C.c_int32),
                ("diagnostics", C.c_int32), ("pairing", C.c_int32), ("f_E", C.c_double),
                ("eps0", C.c_double), ("c", C.c_double)]


class mcc_stats(C.Structure):
    _fields_ = [("pairs", C.c_ulonglong), ("corr_pairs", C.c_ulonglong),
                ("failed", C.c_ulonglong), ("collisions", C.c_ulonglong),
                ("max_rel_dP", C.c_double), ("max_rel_dE", C.c_double)]


class MCCError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__("%s failed: %s (%d)" % (fn, STATUS.get(code, "unknown"), code))
        self.code = code


_lib = None


def _hip_runtimes():
    """Files of the HIP runtime (libamdhip64) mapped into this process."""
    out = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    out.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return out


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmcc_hip.so not found at %s: run __graft_entry__.build() "
                           "(or python -m paper_2407_19151_amd.build)" % path)
    # torch ships its own HIP runtime with the same soname as the system one;
    # loading torch first makes this library bind to that runtime, so the
    # process holds one HIP runtime and torch's allocations and streams are
    # valid here
    import torch  # noqa: F401
    L = C.CDLL(path)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError("two HIP runtimes are mapped in this process (%s): this library and "
                           "torch would hold separate devices, streams and allocations; import "
                           "torch before loading libmcc_hip.so" % ", ".join(sorted(runtimes)))
    P, i32, i64, u64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
    L.mcc_default_params.argtypes = [C.POINTER(mcc_params)]
    L.mcc_default_params.restype = None
    L.mcc_status_string.argtypes = [C.c_int]
    L.mcc_status_string.restype = C.c_char_p
    L.mcc_create.argtypes = [C.POINTER(P), C.c_int, P]
    L.mcc_create.restype = C.c_int
    L.mcc_set_stream.argtypes = [P, P]
    L.mcc_set_stream.restype = C.c_int
    L.mcc_destroy.argtypes = [P]
    L.mcc_destroy.restype = None
    L.mcc_set_variant.argtypes = [P, i32, i32]
    L.mcc_set_variant.restype = C.c_int
    L.mcc_device_error.argtypes = [P, C.POINTER(i32)]
    L.mcc_device_error.restype = C.c_int
    step_args = [P, P, P, P, P, f64, C.POINTER(mcc_species), i32, C.POINTER(mcc_collision),
                 f64, f64, u64, u64, C.POINTER(mcc_params), P, P]
    L.mcc_collide_sorted.argtypes = [P, i64, i32, i32, P] + step_args
    L.mcc_collide_sorted.restype = C.c_int
    L.mcc_collide_sorted_noalloc.argtypes = [P, i64, i32, i32, P] + step_args
    L.mcc_collide_sorted_noalloc.restype = C.c_int
    L.mcc_collide.argtypes = [P, i64, P, P, i32, i32] + step_args
    L.mcc_collide.restype = C.c_int
    L.mcc_collide_sorted_jvp.argtypes = [P, i64, i32, i32, P, P, P, P, P, P, P, P, P, f64,
                                         C.POINTER(mcc_species), i32, C.POINTER(mcc_collision),
                                         f64, f64, f64, u64, u64, C.POINTER(mcc_params), i32, P]
    L.mcc_collide_sorted_jvp.restype = C.c_int
    L.mcc_collide_adjoint.argtypes = [P, i64, i32, i32, P, P, P, P, P, P, P, P, P, f64,
                                      C.POINTER(mcc_species), i32, C.POINTER(mcc_collision),
                                      f64, f64, u64, u64, C.POINTER(mcc_params), P]
    L.mcc_collide_adjoint.restype = C.c_int
    L.mcc_bin.argtypes = [P, i64, P, P, i32, i32, P, P]
    L.mcc_rebin.argtypes = [P, i64, i32, i32, P, P, P, P, P, P, P, P]
    L.mcc_rebin.restype = C.c_int
    L.mcc_rebin_out.argtypes = [P, i64, i32, i32, P, P, P, P, P, P, P, P, P, P, P, P]
    L.mcc_rebin_out.restype = C.c_int
    L.mcc_bin.restype = C.c_int
    L.mcc_plan_create.argtypes = [P, C.POINTER(P), i64, i32, i32, P, P, P, P, P, P, f64,
                                  C.POINTER(mcc_species), i32, C.POINTER(mcc_collision), f64,
                                  f64, u64, C.POINTER(mcc_params), P, P, i32]
    L.mcc_plan_create.restype = C.c_int
    L.mcc_plan_run.argtypes = [P, u64, i32]
    L.mcc_plan_run.restype = C.c_int
    L.mcc_plan_run_bucket.argtypes = [P, i32, u64]
    L.mcc_plan_run_bucket.restype = C.c_int
    L.mcc_plan_describe.argtypes = [P, C.c_char_p, C.c_size_t]
    L.mcc_plan_describe.restype = C.c_int
    L.mcc_sample_angles.argtypes = [P, i32, i32, i64, P, P, P, P, P, P]
    L.mcc_sample_angles.restype = C.c_int
    L.mcc_plan_destroy.argtypes = [P]
    L.mcc_plan_destroy.restype = None
    _lib = L
    return L


def _check(fn: str, rc: int):
    if rc != 0:
        raise MCCError(fn, rc)


def make_params(method: int = MCC_N97, precision: int = MCC_FP64, relativistic: bool = False,
                moment_correction: bool = True, sort_by_weight: bool = True,
                max_passes: int = 1, on_failure: int = MCC_FAIL_RESET,
                diagnostics: bool = False, f_E: float = 0.05, eps0: float = 1.0,
                c: float = 0.0, pairing: int = 0) -> mcc_params:
    p = mcc_params()
    load().mcc_default_params(C.byref(p))
    p.method = int(method)
    p.precision = int(precision)
    p.relativistic = int(bool(relativistic))
    p.moment_correction = int(bool(moment_correction))
    p.sort_by_weight = int(bool(sort_by_weight))
    p.max_passes = int(max_passes)
    p.on_failure = int(on_failure)
    p.diagnostics = int(bool(diagnostics))
    p.pairing = int(pairing)
    p.f_E = float(f_E)
    p.eps0 = float(eps0)
    p.c = float(c) if (c is not None and math.isfinite(c)) else 0.0
    return p


def _species(mass: Sequence[float], charge: Sequence[float]):
    arr = (mcc_species * len(mass))()
    for i, (m, q) in enumerate(zip(mass, charge)):
        arr[i].mass = float(m)
        arr[i].charge = float(q)
    return arr


def _collisions(coll: Sequence[Tuple]):
    """(a, b) or (a, b, cross_section); the cross-section is read by the
    hard-sphere method only."""
    arr = (mcc_collision * max(len(coll), 1))()
    for i, c in enumerate(coll):
        arr[i].a = int(c[0])
        arr[i].b = int(c[1])
        arr[i].cross_section = float(c[2]) if len(c) > 2 else 0.0
    return arr


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _expect(t, dtype, n, name):
    """Arguments handed to the library as raw pointers: right type and size,
    dense, and on the GPU (the library reads them as flat device arrays)."""
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if n is not None and t.numel() != n:
        raise ValueError("%s must have %d elements" % (name, n))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)


def _cur_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Context:
    """One library context on the current torch device, following the
    current torch stream at every call."""

    def __init__(self, device: Optional[int] = None):
        import torch
        self.L = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check("mcc_create", self.L.mcc_create(C.byref(h), self.device,
                                                   C.c_void_p(_cur_stream())))
        self.h = h

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.L.mcc_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be torn down (and
        # module globals such as sys cleared: hence the bound default)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        _check("mcc_set_stream", self.L.mcc_set_stream(self.h, C.c_void_p(_cur_stream())))

    def set_variant(self, bucket: int, variant: int):
        """Kernel variant for a cell-size bucket (-1: default)."""
        _check("mcc_set_variant", self.L.mcc_set_variant(self.h, int(bucket), int(variant)))

    def device_error(self) -> int:
        code = C.c_int32(0)
        _check("mcc_device_error", self.L.mcc_device_error(self.h, C.byref(code)))
        return code.value

    def _common(self, weights, vx, vy, vz, cell_volume, mass, charge, collisions, params,
                stats, cell_corr_pairs, n_cells):
        import torch
        n = vx.numel()
        for t, nm in ((weights, "weights"), (vx, "vx"), (vy, "vy"), (vz, "vz")):
            _expect(t, torch.float64, n, nm)
        if isinstance(cell_volume, torch.Tensor):
            _expect(cell_volume, torch.float64, n_cells, "cell_volume")
            cv, cvs = _ptr(cell_volume), 0.0
        else:
            cv, cvs = None, float(cell_volume)
        if stats is not None:
            _expect(stats, torch.uint8, C.sizeof(mcc_stats), "stats")
        if cell_corr_pairs is not None:
            _expect(cell_corr_pairs, torch.int32, n_cells, "cell_corr_pairs")
        sp = _species(mass, charge)
        co = _collisions(collisions)
        p = params if params is not None else make_params()
        return n, cv, cvs, sp, co, p

    def collide_sorted(self, offsets, weights, vx, vy, vz, *, n_cells: int, mass, charge,
                       collisions, dt: float, coulomb_log: float, seed: int, step: int,
                       params: Optional[mcc_params] = None, cell_volume=1.0, stats=None,
                       cell_corr_pairs=None):
        """mcc_collide_sorted on device tensors (velocities updated in place)."""
        import torch
        n, cv, cvs, sp, co, p = self._common(weights, vx, vy, vz, cell_volume, mass, charge,
                                             collisions, params, stats, cell_corr_pairs, n_cells)
        _expect(offsets, torch.int64, n_cells * len(mass) + 1, "offsets")
        self._stream()
        rc = self.L.mcc_collide_sorted(
            self.h, n, n_cells, len(mass), _ptr(offsets), _ptr(weights), _ptr(vx), _ptr(vy),
            _ptr(vz), cv, cvs, sp, len(collisions), co, float(dt), float(coulomb_log),
            int(seed), int(step), C.byref(p), _ptr(stats), _ptr(cell_corr_pairs))
        _check("mcc_collide_sorted", rc)

    def collide_sorted_noalloc(self, offsets, weights, vx, vy, vz, *, n_cells: int, mass,
                               charge, collisions, dt: float, coulomb_log: float, seed: int,
                               step: int, params: Optional[mcc_params] = None,
                               cell_volume=1.0, stats=None, cell_corr_pairs=None):
        """mcc_collide_sorted_noalloc: the sorted step with no device allocation."""
        import torch
        n, cv, cvs, sp, co, p = self._common(weights, vx, vy, vz, cell_volume, mass, charge,
                                             collisions, params, stats, cell_corr_pairs, n_cells)
        _expect(offsets, torch.int64, n_cells * len(mass) + 1, "offsets")
        self._stream()
        rc = self.L.mcc_collide_sorted_noalloc(
            self.h, n, n_cells, len(mass), _ptr(offsets), _ptr(weights), _ptr(vx), _ptr(vy),
            _ptr(vz), cv, cvs, sp, len(collisions), co, float(dt), float(coulomb_log),
            int(seed), int(step), C.byref(p), _ptr(stats), _ptr(cell_corr_pairs))
        _check("mcc_collide_sorted_noalloc", rc)

    def collide_sorted_jvp(self, offsets, weights, vx, vy, vz, tx, ty, tz, *, n_cells: int,
                           mass, charge, collisions, dt: float, coulomb_log: float,
                           coulomb_log_tangent: float, seed: int, step: int,
                           params: Optional[mcc_params] = None, cell_volume=1.0,
                           update_primal: bool = True, stats=None):
        """mcc_collide_sorted_jvp: the step and its tangent (tx, ty, tz in place)."""
        import torch
        n, cv, cvs, sp, co, p = self._common(weights, vx, vy, vz, cell_volume, mass, charge,
                                             collisions, params, stats, None, n_cells)
        _expect(offsets, torch.int64, n_cells * len(mass) + 1, "offsets")
        for name, t in (("tx", tx), ("ty", ty), ("tz", tz)):
            _expect(t, torch.float64, n, name)
        self._stream()
        rc = self.L.mcc_collide_sorted_jvp(
            self.h, n, n_cells, len(mass), _ptr(offsets), _ptr(weights), _ptr(vx), _ptr(vy),
            _ptr(vz), _ptr(tx), _ptr(ty), _ptr(tz), cv, cvs, sp, len(collisions), co, float(dt),
            float(coulomb_log), float(coulomb_log_tangent), int(seed), int(step), C.byref(p),
            int(bool(update_primal)), _ptr(stats))
        _check("mcc_collide_sorted_jvp", rc)

    def collide_adjoint(self, offsets, weights, vx, vy, vz, gx, gy, gz, *, n_cells: int,
                        mass, charge, collisions, dt: float, coulomb_log: float, seed: int,
                        step: int, params: Optional[mcc_params] = None, cell_volume=1.0,
                        g_coulomb_log=None):
        """mcc_collide_adjoint: (gx, gy, gz) <- g J in place for the step from
        (vx, vy, vz); g_coulomb_log (1-element float64 device tensor or None)
        receives g dv'/dlnL."""
        import torch
        n, cv, cvs, sp, co, p = self._common(weights, vx, vy, vz, cell_volume, mass, charge,
                                             collisions, params, None, None, n_cells)
        _expect(offsets, torch.int64, n_cells * len(mass) + 1, "offsets")
        for name, t in (("gx", gx), ("gy", gy), ("gz", gz)):
            _expect(t, torch.float64, n, name)
        if g_coulomb_log is not None:
            _expect(g_coulomb_log, torch.float64, 1, "g_coulomb_log")
        self._stream()
        rc = self.L.mcc_collide_adjoint(
            self.h, n, n_cells, len(mass), _ptr(offsets), _ptr(weights), _ptr(vx), _ptr(vy),
            _ptr(vz), _ptr(gx), _ptr(gy), _ptr(gz), cv, cvs, sp, len(collisions), co, float(dt),
            float(coulomb_log), int(seed), int(step), C.byref(p), _ptr(g_coulomb_log))
        _check("mcc_collide_adjoint", rc)

    def collide(self, cells, species_id, weights, vx, vy, vz, *, n_cells: int, mass, charge,
                collisions, dt: float, coulomb_log: float, seed: int, step: int,
                params: Optional[mcc_params] = None, cell_volume=1.0, stats=None,
                cell_corr_pairs=None):
        """mcc_collide on particles in any order (velocities updated in place)."""
        import torch
        n, cv, cvs, sp, co, p = self._common(weights, vx, vy, vz, cell_volume, mass, charge,
                                             collisions, params, stats, cell_corr_pairs, n_cells)
        _expect(cells, torch.int32, n, "cells")
        _expect(species_id, torch.int32, n, "species_id")
        self._stream()
        rc = self.L.mcc_collide(
            self.h, n, _ptr(cells), _ptr(species_id), n_cells, len(mass), _ptr(weights),
            _ptr(vx), _ptr(vy), _ptr(vz), cv, cvs, sp, len(collisions), co, float(dt),
            float(coulomb_log), int(seed), int(step), C.byref(p), _ptr(stats),
            _ptr(cell_corr_pairs))
        _check("mcc_collide", rc)

    def sample_angles(self, method: int, precision: int, s, a0, a1):
        """mcc_sample_angles on device tensors: returns (oc, st, A)."""
        import torch
        n = s.numel()
        _expect(s, torch.float64, n, "s")
        _expect(a0, torch.int32, n, "a0")
        _expect(a1, torch.int32, n, "a1")
        oc = torch.empty(n, dtype=torch.float64, device=s.device)
        st = torch.empty_like(oc)
        A = torch.empty_like(oc)
        self._stream()
        _check("mcc_sample_angles", self.L.mcc_sample_angles(
            self.h, int(method), int(precision), n, _ptr(s), _ptr(a0), _ptr(a1), _ptr(oc),
            _ptr(st), _ptr(A)))
        return oc, st, A

    def bin(self, cells, species_id, n_cells: int, n_species: int):
        """mcc_bin: (offsets int64[n_cells*S+1], perm int32[n]) on the device."""
        import torch
        n = cells.numel()
        _expect(cells, torch.int32, n, "cells")
        _expect(species_id, torch.int32, n, "species_id")
        off = torch.empty(n_cells * n_species + 1, dtype=torch.int64, device=cells.device)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=cells.device)
        self._stream()
        _check("mcc_bin", self.L.mcc_bin(self.h, n, _ptr(cells), _ptr(species_id), n_cells,
                                         n_species, _ptr(off), _ptr(perm)))
        return off, perm[:n]

    def rebin(self, offsets, cells_new, n_cells: int, n_species: int, w=None, vx=None,
              vy=None, vz=None):
        """mcc_rebin: (offsets_new, perm) on the device; w, vx, vy, vz (all or
        none) are permuted in place."""
        import torch
        n = cells_new.numel()
        _expect(cells_new, torch.int32, n, "cells_new")
        _expect(offsets, torch.int64, n_cells * n_species + 1, "offsets")
        pay = (w, vx, vy, vz)
        if any(a is not None for a in pay):
            for a, name in zip(pay, ("w", "vx", "vy", "vz")):
                _expect(a, torch.float64, n, name)
        off = torch.empty(n_cells * n_species + 1, dtype=torch.int64, device=cells_new.device)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=cells_new.device)
        self._stream()
        _check("mcc_rebin", self.L.mcc_rebin(self.h, n, n_cells, n_species, _ptr(offsets),
                                             _ptr(cells_new), _ptr(off), _ptr(perm),
                                             *(_ptr(a) for a in pay)))
        return off, perm[:n]

    def rebin_out(self, offsets, cells_new, n_cells: int, n_species: int, w, vx, vy, vz,
                  w_out, vx_out, vy_out, vz_out):
        """mcc_rebin_out: (offsets_new, perm) on the device; w, vx, vy, vz are
        gathered into w_out, vx_out, vy_out, vz_out in the new order."""
        import torch
        n = cells_new.numel()
        _expect(cells_new, torch.int32, n, "cells_new")
        _expect(offsets, torch.int64, n_cells * n_species + 1, "offsets")
        pay = (w, vx, vy, vz, w_out, vx_out, vy_out, vz_out)
        for a, name in zip(pay, ("w", "vx", "vy", "vz", "w_out", "vx_out", "vy_out", "vz_out")):
            _expect(a, torch.float64, n, name)
        off = torch.empty(n_cells * n_species + 1, dtype=torch.int64, device=cells_new.device)
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=cells_new.device)
        self._stream()
        _check("mcc_rebin_out", self.L.mcc_rebin_out(self.h, n, n_cells, n_species,
                                                     _ptr(offsets), _ptr(cells_new), _ptr(off),
                                                     _ptr(perm), *(_ptr(a) for a in pay)))
        return off, perm[:n]


def new_stats(device=None):
    """A zeroed device mcc_stats buffer (uint8 bytes)."""
    import torch
    return torch.zeros(C.sizeof(mcc_stats), dtype=torch.uint8,
                       device=device if device is not None else "cuda")


def read_stats(stats) -> dict:
    """Decode a device mcc_stats buffer (synchronizes through .cpu())."""
    raw = bytes(stats.cpu().numpy().tobytes())
    s = mcc_stats.from_buffer_copy(raw)
    return dict(pairs=s.pairs, corr_pairs=s.corr_pairs, failed=s.failed,
                collisions=s.collisions, max_rel_dP=s.max_rel_dP, max_rel_dE=s.max_rel_dE)


class Plan:
    """mcc_plan: one particle population, size-bucketed work lists, autotuned
    threads-per-cell, one step captured in a HIP graph."""

    def __init__(self, ctx: Context, offsets, weights, vx, vy, vz, *, n_cells: int, mass,
                 charge, collisions, dt: float, coulomb_log: float, seed: int,
                 params: Optional[mcc_params] = None, cell_volume=1.0, stats=None,
                 cell_corr_pairs=None, autotune: bool = True):
        import torch
        self.ctx = ctx
        n, cv, cvs, sp, co, p = ctx._common(weights, vx, vy, vz, cell_volume, mass, charge,
                                            collisions, params, stats, cell_corr_pairs, n_cells)
        _expect(offsets, torch.int64, n_cells * len(mass) + 1, "offsets")
        # keep the bound tensors alive for the plan's lifetime
        self._keep = (offsets, weights, vx, vy, vz, cell_volume, stats, cell_corr_pairs)
        ctx._stream()
        h = C.c_void_p()
        rc = ctx.L.mcc_plan_create(ctx.h, C.byref(h), n, n_cells, len(mass), _ptr(offsets),
                                   _ptr(weights), _ptr(vx), _ptr(vy), _ptr(vz), cv, cvs, sp,
                                   len(collisions), co, float(dt), float(coulomb_log),
                                   int(seed), C.byref(p), _ptr(stats), _ptr(cell_corr_pairs),
                                   int(bool(autotune)))
        _check("mcc_plan_create", rc)
        self.h = h

    def run(self, first_step: int, n_steps: int = 1):
        self.ctx._stream()
        _check("mcc_plan_run", self.ctx.L.mcc_plan_run(self.h, int(first_step), int(n_steps)))

    def run_bucket(self, bucket: int, step: int):
        """Launch the kernel of one size bucket alone for one step."""
        self.ctx._stream()
        _check("mcc_plan_run_bucket",
               self.ctx.L.mcc_plan_run_bucket(self.h, int(bucket), int(step)))

    def describe(self) -> str:
        buf = C.create_string_buffer(8192)
        _check("mcc_plan_describe", self.ctx.L.mcc_plan_describe(self.h, buf, 8192))
        return buf.value.decode()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.ctx.L.mcc_plan_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
