"""ctypes binding of libpamd.so (the C ABI in include/pamd.h).

Argument marshalling only: every step of the PAMD path runs in the HIP
kernels of the library.  PyTorch provides the device buffers and the stream.
Raises ``RuntimeError`` when the library has not been built (no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpamd.so")
CHECK_LIB_PATH = os.path.join(_HERE, "libpamd_check.so")   # resampling indices verified on the device

PAMD_OK, PAMD_ERR_ARG, PAMD_ERR_HIP, PAMD_ERR_CAPACITY, PAMD_ERR_NONFINITE, PAMD_ERR_STATE, PAMD_ERR_INTERNAL = range(7)
PAMD_FP64, PAMD_FP32 = 0, 1
PAMD_RESAMPLE_NEAREST, PAMD_RESAMPLE_MULTINOMIAL, PAMD_RESAMPLE_NONE = 0, 1, 2
PAMD_THERMOSTAT_ANDERSEN, PAMD_THERMOSTAT_LANGEVIN = 0, 1
PAMD_LAYOUT_AUTO, PAMD_LAYOUT_TILE, PAMD_LAYOUT_WIDE = 0, 1, 2
LAYOUTS = {"auto": PAMD_LAYOUT_AUTO, "tile": PAMD_LAYOUT_TILE, "wide": PAMD_LAYOUT_WIDE}
THERMOSTATS = {"andersen": PAMD_THERMOSTAT_ANDERSEN, "langevin": PAMD_THERMOSTAT_LANGEVIN}
RESAMPLING_MODES = {"nearest": PAMD_RESAMPLE_NEAREST, "multinomial": PAMD_RESAMPLE_MULTINOMIAL,
                    "none": PAMD_RESAMPLE_NONE}
PAMD_FORCE_CHUNK = 256
MAX_ATOMS = 320
TILE_ATOMS = 80
WIDE_LJ_CLASSES = 25   # distinct (sigma, epsilon) pairs of one molecule in the wide layout


class PamdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pamd error {code}: {msg}")
        self.code = code


class pamd_system(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32), ("n_bonds", C.c_int32), ("n_angles", C.c_int32),
        ("n_dihedrals", C.c_int32),
        ("mass", C.c_void_p), ("charge", C.c_void_p), ("sigma", C.c_void_p), ("epsilon", C.c_void_p),
        ("bond_idx", C.c_void_p), ("bond_k", C.c_void_p), ("bond_r0", C.c_void_p),
        ("angle_idx", C.c_void_p), ("angle_k", C.c_void_p), ("angle_theta0", C.c_void_p),
        ("dih_idx", C.c_void_p), ("dih_k", C.c_void_p), ("dih_n", C.c_void_p), ("dih_delta", C.c_void_p),
        ("scale14_lj", C.c_double), ("scale14_coul", C.c_double), ("coulomb_k", C.c_double),
        ("dielectric", C.c_int32), ("reserved", C.c_int32), ("kB", C.c_double), ("x_init", C.c_void_p),
    ]


class pamd_params(C.Structure):
    _fields_ = [
        ("R_target", C.c_int64), ("R_cap", C.c_int64), ("T0", C.c_double), ("dt", C.c_double),
        ("nu", C.c_double), ("seed", C.c_uint64), ("precision", C.c_int32),
        ("waves_per_block", C.c_int32), ("V_target", C.c_double), ("T_final", C.c_double),
        ("resampling", C.c_int32), ("thermostat", C.c_int32), ("layout", C.c_int32),
        ("wide_waves_per_block", C.c_int32),
    ]


class pamd_obs(C.Structure):
    _fields_ = [
        ("T", C.c_double), ("T_prev", C.c_double), ("lnQ_last", C.c_double), ("sum_lnQ", C.c_double),
        ("V_last", C.c_double), ("E_mean", C.c_double), ("E2_mean", C.c_double), ("K_mean", C.c_double),
        ("T_measured", C.c_double), ("Cv", C.c_double), ("R", C.c_int64), ("families", C.c_int64),
        ("temp_index", C.c_int64), ("step", C.c_int64), ("error", C.c_int32), ("reserved", C.c_int32),
    ]


class pamd_run_scalars(C.Structure):
    _fields_ = [("T", C.c_double), ("T_prev", C.c_double), ("sum_lnQ", C.c_double),
                ("lnQ_last", C.c_double), ("R", C.c_int64), ("step", C.c_uint32),
                ("temp_index", C.c_uint32)]


EXPORTS = ["pamd_query_sizes", "pamd_init", "pamd_md_steps", "pamd_resample", "pamd_observables",
           "pamd_graph_capture", "pamd_graph_launch", "pamd_set_schedule",
           "pamd_get_forces", "pamd_get_state", "pamd_set_state", "pamd_get_counts",
           "pamd_launch_info", "pamd_run_launch", "pamd_destroy", "pamd_last_error",
           "pamd_nn_query_sizes", "pamd_nn_create", "pamd_nn_set_weights", "pamd_nn_get_weights",
           "pamd_nn_forces", "pamd_nn_forces_static",
           "pamd_nn_loss_grad", "pamd_nn_train_step", "pamd_nn_destroy", "pamd_nn_last_error",
           "pamd_export_configs", "pamd_mts_query_sizes", "pamd_set_mts", "pamd_fp32_fma_rate", "pamd_valu_issue_rates",
           "pamd_family_error", "pamd_binning_error", "pamd_wham", "pamd_wham_average"]
NN_PARAMS = 49537
NN_FEATURES, NN_HIDDEN, NN_TYPES = 256, 128, 8
NN_STATIC_ROWS = 16000      # configuration-atom rows of pamd_nn_forces_static
_NO_STATUS = ("pamd_destroy", "pamd_last_error", "pamd_nn_destroy", "pamd_nn_last_error")

_lib = None
_other_libs: Dict[str, object] = {}


def load_library(path: str = LIB_PATH):
    """Load libpamd.so (built by ``python -m paper_1806_06016_amd.build``), or
    another build of it such as CHECK_LIB_PATH."""
    global _lib
    if path == LIB_PATH and _lib is not None:
        return _lib
    if path != LIB_PATH and path in _other_libs:
        return _other_libs[path]
    # torch first: libpamd then binds to the HIP runtime torch already loaded
    # (one runtime per process)
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1806_06016_amd.build` "
                           "(the PAMD path has no fallback)")
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    P = C.POINTER
    lib.pamd_query_sizes.argtypes = [vp, i32, vp, P(C.c_size_t), P(C.c_size_t)]
    lib.pamd_init.argtypes = [vp, i32, vp, vp, C.c_size_t, vp, C.c_size_t, vp, P(vp)]
    lib.pamd_md_steps.argtypes = [vp, i32, vp]
    lib.pamd_resample.argtypes = [vp, vp, vp, vp]
    lib.pamd_observables.argtypes = [vp, vp, vp]
    lib.pamd_graph_capture.argtypes = [vp, i32, i32, i32, i32, vp]
    lib.pamd_graph_launch.argtypes = [vp, i32, vp]
    lib.pamd_set_schedule.argtypes = [vp, i32, vp, i32, vp]
    lib.pamd_get_forces.argtypes = [vp, i32, i64, i32, vp, vp, vp]
    lib.pamd_get_state.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.pamd_set_state.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.pamd_get_counts.argtypes = [vp, i32, vp, P(i64), vp]
    lib.pamd_launch_info.argtypes = [vp, P(i32), P(i32), P(i32)]
    lib.pamd_run_launch.argtypes = [vp, i32, P(i32), P(i32), P(i32), P(i32)]
    lib.pamd_destroy.argtypes = [vp]
    lib.pamd_destroy.restype = None
    lib.pamd_last_error.argtypes = [vp]
    lib.pamd_last_error.restype = C.c_char_p
    lib.pamd_nn_query_sizes.argtypes = [i32, i64, P(C.c_size_t)]
    lib.pamd_nn_create.argtypes = [vp, vp, i64, vp, C.c_size_t, vp, P(vp)]
    lib.pamd_nn_set_weights.argtypes = [vp, vp, vp]
    lib.pamd_nn_get_weights.argtypes = [vp, vp, vp]
    lib.pamd_nn_forces.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.pamd_nn_forces_static.argtypes = [vp, i64, vp, vp, vp, vp]
    lib.pamd_nn_loss_grad.argtypes = [vp, i64, vp, vp, vp, vp, vp]
    lib.pamd_nn_train_step.argtypes = [vp, i64, vp, vp, C.c_float, vp, vp]
    lib.pamd_nn_destroy.argtypes = [vp]
    lib.pamd_nn_destroy.restype = None
    lib.pamd_nn_last_error.argtypes = [vp]
    lib.pamd_nn_last_error.restype = C.c_char_p
    lib.pamd_export_configs.argtypes = [vp, i32, i64, i64, vp, vp, vp]
    lib.pamd_mts_query_sizes.argtypes = [vp, P(C.c_size_t)]
    lib.pamd_set_mts.argtypes = [vp, vp, i32, vp, C.c_size_t, vp]
    lib.pamd_fp32_fma_rate.argtypes = [vp, vp, vp]
    lib.pamd_valu_issue_rates.argtypes = [vp, i32, vp, vp, vp]
    lib.pamd_family_error.argtypes = [vp, vp, i64, vp]
    lib.pamd_binning_error.argtypes = [vp, i64, i64, vp]
    lib.pamd_wham.argtypes = [i32, vp, vp, vp, vp, i32, C.c_double, vp]
    lib.pamd_wham_average.argtypes = [i32, vp, vp, vp, vp, C.c_double, vp, vp]
    for name in EXPORTS:
        if name not in _NO_STATUS:
            getattr(lib, name).restype = i32
    if path == LIB_PATH:
        _lib = lib
    else:
        _other_libs[path] = lib
    return lib


class pamd_family_stats(C.Structure):
    _fields_ = [("mean", C.c_double), ("naive_se", C.c_double), ("family_se", C.c_double),
                ("rho_t", C.c_double), ("family_entropy", C.c_double), ("families", C.c_int64)]


def _host_check(st: int, what: str):
    if st != PAMD_OK:
        raise PamdError(st, what)


def family_error(O, ancestor) -> Dict:
    """Population mean of O with its naive and family (common-ancestor) errors,
    rho_t and the family entropy (host, FP64)."""
    O = np.ascontiguousarray(O, np.float64)
    a = np.ascontiguousarray(ancestor, np.int32)
    assert O.shape == a.shape and O.ndim == 1
    out = pamd_family_stats()
    _host_check(load_library().pamd_family_error(_ptr(O), _ptr(a), len(O), C.byref(out)), "family_error")
    return {k: getattr(out, k) for k, _ in pamd_family_stats._fields_}


def binning_error(O, bin_size: int) -> float:
    O = np.ascontiguousarray(O, np.float64)
    se = C.c_double()
    _host_check(load_library().pamd_binning_error(_ptr(O), len(O), int(bin_size), C.byref(se)), "binning_error")
    return se.value


def _wham_args(beta, samples):
    b = np.ascontiguousarray(beta, np.float64)
    n = np.ascontiguousarray([len(s) for s in samples], np.int64)
    E = np.ascontiguousarray(np.concatenate([np.asarray(s, np.float64) for s in samples]))
    assert len(b) == len(n)
    return b, n, E


def wham(beta, samples, lnZ0, max_iter: int = 1000, tol: float = 1e-10):
    """Refined ln Z [L] and the iteration count (see pamd_wham)."""
    b, n, E = _wham_args(beta, samples)
    lnZ = np.ascontiguousarray(lnZ0, np.float64).copy()
    it = C.c_int32()
    _host_check(load_library().pamd_wham(len(b), _ptr(b), _ptr(n), _ptr(E), _ptr(lnZ), int(max_iter), float(tol),
                                         C.byref(it)), "wham")
    return lnZ, it.value


def wham_average(beta_q: float, beta, samples, lnZ):
    b, n, E = _wham_args(beta, samples)
    z = np.ascontiguousarray(lnZ, np.float64)
    e1, e2 = C.c_double(), C.c_double()
    _host_check(load_library().pamd_wham_average(len(b), _ptr(b), _ptr(n), _ptr(E), _ptr(z), float(beta_q),
                                                 C.byref(e1), C.byref(e2)), "wham_average")
    return e1.value, e2.value


def fp32_fma_rate() -> float:
    """TFLOP/s of independent FP32 FMAs on the current GPU (the ceiling of this
    library's FP32 VALU-bound kernels, built without packed FP32)."""
    import torch
    lib = load_library()
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    out = C.c_double()
    st = lib.pamd_fp32_fma_rate(C.c_void_p(sink.data_ptr()), C.byref(out),
                                C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != PAMD_OK:
        raise PamdError(st, "FMA-rate calibration failed")
    return out.value


VALU_FORMS = ("v_fma_f32 (VGPR operands)", "v_fma_f32 (one SGPR operand)", "v_fmac_f32_e32", "v_mul_f32_e32",
              "v_add_f32 (DPP row-rotated source)", "v_mov_b32 (DPP row rotation)", "v_rcp_f32")


def valu_issue_rates(waves_per_simd: int = 4) -> Dict:
    """Shader cycles per wave64 instruction per SIMD of single VALU
    instruction forms (pamd_valu_issue_rates) and the measured shader clock."""
    import torch
    lib = load_library()
    sink = torch.zeros(4, dtype=torch.float32, device="cuda")
    cyc = (C.c_double * len(VALU_FORMS))()
    ghz = C.c_double()
    st = lib.pamd_valu_issue_rates(C.c_void_p(sink.data_ptr()), int(waves_per_simd), cyc, C.byref(ghz),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != PAMD_OK:
        raise PamdError(st, "VALU issue-rate calibration failed")
    return {"waves_per_simd": int(waves_per_simd), "clock_ghz": ghz.value,
            "cycles_per_instr": {name: cyc[f] for f, name in enumerate(VALU_FORMS)}}


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def make_system_struct(sysd, keep: list) -> pamd_system:
    """Fill a pamd_system from an input-system object (numpy arrays)."""
    def f64(a):
        a = np.ascontiguousarray(a, np.float64)
        keep.append(a)
        return a.ctypes.data

    def i32(a):
        a = np.ascontiguousarray(a, np.int32)
        keep.append(a)
        return a.ctypes.data

    s = pamd_system()
    s.n_atoms = int(sysd.n_atoms)
    s.n_bonds, s.n_angles, s.n_dihedrals = len(sysd.bonds), len(sysd.angles), len(sysd.dihedrals)
    s.mass, s.charge, s.sigma, s.epsilon = (f64(sysd.mass), f64(sysd.charge), f64(sysd.sigma),
                                            f64(sysd.epsilon))
    s.bond_idx, s.bond_k, s.bond_r0 = i32(sysd.bonds), f64(sysd.bond_k), f64(sysd.bond_r0)
    s.angle_idx, s.angle_k, s.angle_theta0 = i32(sysd.angles), f64(sysd.angle_k), f64(sysd.angle_theta0)
    s.dih_idx, s.dih_k, s.dih_n, s.dih_delta = (i32(sysd.dihedrals), f64(sysd.dih_k), i32(sysd.dih_n),
                                                f64(sysd.dih_delta))
    s.scale14_lj, s.scale14_coul = float(sysd.scale14_lj), float(sysd.scale14_coul)
    s.coulomb_k, s.dielectric, s.kB = float(sysd.coulomb_k), int(sysd.dielectric), float(sysd.kB)
    s.x_init = f64(sysd.x_init)
    return s


class Pamd:
    """One PAMD context: n_runs independent populations on the current GPU."""

    def __init__(self, systems: Sequence, R_target: int, T0: float, dt: float, nu: float, seed: int,
                 precision: int = PAMD_FP32, R_cap: Optional[int] = None, V_target: float = 0.1,
                 T_final: Optional[float] = None, waves_per_block: int = 0, stream=None,
                 resampling="nearest", thermostat: str = "andersen", layout="auto", wide_waves: int = 0,
                 library: Optional[str] = None):
        """resampling: "nearest", "multinomial" or "none" for every run, or one
        mode per run (a sequence).  thermostat: "andersen" (nu = collision
        frequency) or "langevin" (nu = friction gamma), one for the context.
        layout: "auto", "tile" or "wide" for every run, or one per run.
        waves_per_block / wide_waves: workgroup size of the register-tile and
        of the batched wide kernel (0: automatic).  library: path of the
        library build to run (default libpamd.so; CHECK_LIB_PATH: the
        bounds-checked resampling)."""
        import torch
        self.torch = torch
        self.lib = load_library(library or LIB_PATH)
        if not torch.cuda.is_available():
            raise RuntimeError("the PAMD library needs a ROCm GPU")
        self.systems = list(systems)
        self.n_runs = len(self.systems)
        self.n_atoms = [int(s.n_atoms) for s in self.systems]
        if R_cap is None:
            R_cap = max(int(np.ceil(1.02 * R_target)), R_target + 64)
        self.R_cap = int(R_cap)
        self.R_target = int(R_target)
        self.fp32 = int(precision) == PAMD_FP32
        self._keep: list = []
        S = pamd_system * self.n_runs
        P = pamd_params * self.n_runs
        self._sys = S(*[make_system_struct(s, self._keep) for s in self.systems])
        prm = []
        for r in range(self.n_runs):
            p = pamd_params()
            p.R_target, p.R_cap = self.R_target, self.R_cap
            p.T0, p.dt, p.nu, p.seed = float(T0), float(dt), float(nu), int(seed)
            p.precision = int(precision)
            p.waves_per_block = int(waves_per_block)
            p.V_target = float(V_target)
            p.T_final = float(T_final if T_final is not None else T0)
            mode = resampling if isinstance(resampling, str) else resampling[r]
            p.resampling = RESAMPLING_MODES[mode]
            p.thermostat = THERMOSTATS[thermostat]
            p.layout = LAYOUTS[layout if isinstance(layout, str) else layout[r]]
            p.wide_waves_per_block = int(wide_waves)
            prm.append(p)
        self._prm = P(*prm)
        sb, wb = C.c_size_t(), C.c_size_t()
        st = self.lib.pamd_query_sizes(C.byref(self._sys), self.n_runs, C.byref(self._prm), C.byref(sb), C.byref(wb))
        if st == PAMD_ERR_ARG:
            def wide(r):   # the library's layout choice of run r
                lay = layout if isinstance(layout, str) else layout[r]
                if not self.fp32 or lay == "tile":
                    return False
                return lay == "wide" or any(n > TILE_ATOMS for n in self.n_atoms)
            many = [r for r, sd in enumerate(self.systems) if wide(r) and len(
                set(zip(np.asarray(sd.sigma).tolist(), np.asarray(sd.epsilon).tolist()))) > WIDE_LJ_CLASSES]
            if many:
                raise PamdError(st, f"runs {many}: the wide layout takes at most {WIDE_LJ_CLASSES} distinct "
                                    "(sigma, epsilon) pairs per molecule")
        self._check(st, None)
        self.state_bytes, self.work_bytes = sb.value, wb.value
        self.d_state = torch.empty(self.state_bytes + 256, dtype=torch.uint8, device="cuda")
        self.d_work = torch.empty(self.work_bytes + 256, dtype=torch.uint8, device="cuda")
        self._sp = (self.d_state.data_ptr() + 255) // 256 * 256
        self._wp = (self.d_work.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = C.c_void_p()
        st = self.lib.pamd_init(C.byref(self._sys), self.n_runs, C.byref(self._prm), self._sp,
                                self.state_bytes, self._wp, self.work_bytes, self._s(), C.byref(ctx))
        self.ctx = ctx
        self._check(st, ctx)

    # -- helpers ------------------------------------------------------------
    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _check(self, st: int, ctx):
        if st != PAMD_OK:
            msg = self.lib.pamd_last_error(ctx).decode() if ctx else "invalid arguments"
            raise PamdError(st, msg)

    def last_error(self) -> str:
        return self.lib.pamd_last_error(self.ctx).decode()

    def launch_info(self) -> Dict[str, int]:
        w, b, l = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.pamd_launch_info(self.ctx, C.byref(w), C.byref(b), C.byref(l)), self.ctx)
        return dict(waves_per_block=w.value, blocks=b.value, lds_bytes=l.value)

    def run_launch(self, run: int) -> Dict:
        """Layout ("tile" / "wide") and launch shape of the kernel advancing `run`."""
        lay, w, b, l = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.pamd_run_launch(self.ctx, int(run), C.byref(lay), C.byref(w), C.byref(b), C.byref(l)),
                    self.ctx)
        return dict(layout={PAMD_LAYOUT_TILE: "tile", PAMD_LAYOUT_WIDE: "wide"}[lay.value], waves_per_block=w.value,
                    blocks=b.value, lds_bytes=l.value)

    # -- PAMD steps -----------------------------------------------------------
    def md_steps(self, n: int) -> None:
        self._check(self.lib.pamd_md_steps(self.ctx, int(n), self._s()), self.ctx)

    def resample(self, T_next: Optional[Sequence[float]] = None, uniforms=None) -> None:
        """T_next: per-run temperatures (0 or None: adaptive, < 0: next entry of
        the device schedule).  uniforms: optional torch float64 CUDA tensor
        [n_runs, R_cap]: the rounding uniforms of slot j (mode "nearest") or the
        uniforms of draws k < R_target (mode "multinomial")."""
        tn = None
        if T_next is not None:
            tn = (C.c_double * self.n_runs)(*[float(t) for t in T_next])
        up = None
        if uniforms is not None:
            assert uniforms.is_cuda and uniforms.dtype == self.torch.float64
            assert uniforms.numel() >= self.n_runs * self.R_cap and uniforms.is_contiguous()
            up = uniforms.data_ptr()
        self._check(self.lib.pamd_resample(self.ctx, tn, up, self._s()), self.ctx)

    def set_schedule(self, run: int, temps: Sequence[float]) -> None:
        t = np.ascontiguousarray(np.asarray(temps, np.float64))
        self._check(self.lib.pamd_set_schedule(self.ctx, run, _ptr(t), len(t), self._s()), self.ctx)

    def graph_capture(self, n_steps: int, mode: str = "adaptive", slot: int = 0,
                      parts: str = "both") -> None:
        """Capture a HIP graph into `slot`: parts "resample", "md" or "both"
        (one temperature step: resample + n_steps MD steps); mode "adaptive"
        or "schedule" (device schedule) for the resampling."""
        torch = self.torch
        if getattr(self, "_cap_stream", None) is None:
            self._cap_stream = torch.cuda.Stream()
        self._cap_stream.wait_stream(self.stream)
        m = {"adaptive": 0, "schedule": 1}[mode]
        pm = {"resample": 1, "md": 2, "both": 3}[parts]
        self._check(self.lib.pamd_graph_capture(self.ctx, int(slot), pm, int(n_steps), m,
                                                C.c_void_p(self._cap_stream.cuda_stream)), self.ctx)
        self.stream.wait_stream(self._cap_stream)

    def graph_launch(self, slot: int = 0) -> None:
        self._check(self.lib.pamd_graph_launch(self.ctx, int(slot), self._s()), self.ctx)

    def observables(self) -> List[Dict]:
        out = (pamd_obs * self.n_runs)()
        self._check(self.lib.pamd_observables(self.ctx, out, self._s()), self.ctx)
        return [{k: getattr(o, k) for k, _ in pamd_obs._fields_} for o in out]

    # -- inspection -------------------------------------------------------------
    def get_forces(self, run: int = 0, r0: int = 0, count: Optional[int] = None):
        n = self.n_atoms[run]
        st = self.get_state(run, want_xv=False)
        R = st["R"]
        count = R - r0 if count is None else count
        F = np.zeros((count, n, 3))
        E = np.zeros(count)
        for c0 in range(0, count, PAMD_FORCE_CHUNK):
            c = min(PAMD_FORCE_CHUNK, count - c0)
            Fc = np.zeros((c, n, 3))
            Ec = np.zeros(c)
            self._check(self.lib.pamd_get_forces(self.ctx, run, r0 + c0, c, _ptr(Fc), _ptr(Ec), self._s()),
                        self.ctx)
            F[c0:c0 + c] = Fc
            E[c0:c0 + c] = Ec
        return F, E

    def get_state(self, run: int = 0, want_xv: bool = True, after_error: bool = False) -> Dict:
        """Population and scalars of `run`.  With after_error, a context stopped
        by PAMD_ERR_CAPACITY or PAMD_ERR_NONFINITE still returns its state (key
        "error" holds the code) instead of raising."""
        n = self.n_atoms[run]
        sc = pamd_run_scalars()
        x = np.zeros((self.R_cap, n, 3)) if want_xv else None
        v = np.zeros((self.R_cap, n, 3)) if want_xv else None
        Ep = np.zeros(self.R_cap)
        Ek = np.zeros(self.R_cap)
        anc = np.zeros(self.R_cap, np.int32)
        st = self.lib.pamd_get_state(self.ctx, run, _ptr(x), _ptr(v), _ptr(Ep), _ptr(Ek), _ptr(anc), C.byref(sc),
                                     self._s())
        if not (after_error and st in (PAMD_ERR_CAPACITY, PAMD_ERR_NONFINITE)):
            self._check(st, self.ctx)
        R = int(sc.R)
        d = dict(R=R, T=sc.T, T_prev=sc.T_prev, sum_lnQ=sc.sum_lnQ, lnQ_last=sc.lnQ_last, step=int(sc.step),
                 temp_index=int(sc.temp_index), E_pot=Ep[:R].copy(), E_kin=Ek[:R].copy(),
                 ancestor=anc[:R].copy(), error=int(st))
        if want_xv:
            d["x"] = x[:R].copy()
            d["v"] = v[:R].copy()
        return d

    def set_state(self, run: int, x: np.ndarray, v: np.ndarray, T: float, step: int = 0, temp_index: int = 0,
                  E_pot: Optional[np.ndarray] = None, ancestor: Optional[np.ndarray] = None,
                  T_prev: Optional[float] = None, sum_lnQ: float = 0.0, lnQ_last: float = 0.0) -> None:
        x = np.ascontiguousarray(x, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        R = x.shape[0]
        sc = pamd_run_scalars()
        sc.T, sc.T_prev, sc.sum_lnQ, sc.lnQ_last = float(T), float(T_prev or T), float(sum_lnQ), float(lnQ_last)
        sc.R, sc.step, sc.temp_index = R, int(step), int(temp_index)
        Ep = None if E_pot is None else np.ascontiguousarray(E_pot, np.float64)
        an = None if ancestor is None else np.ascontiguousarray(ancestor, np.int32)
        self._check(self.lib.pamd_set_state(self.ctx, run, _ptr(x), _ptr(v), _ptr(Ep), _ptr(an), C.byref(sc),
                                            self._s()), self.ctx)

    # -- learned multiple-time-step surrogate ------------------------------------
    def export_configs(self, run: int = 0, r0: int = 0, count: Optional[int] = None):
        """Positions and exact nonbonded forces of replicas [r0, r0 + count) as
        CUDA float32 tensors [count, n, 3] (FP32 contexts)."""
        torch = self.torch
        n = self.n_atoms[run]
        if count is None:
            count = self.get_state(run, want_xv=False)["R"] - r0
        x = torch.empty((count, n, 3), dtype=torch.float32, device="cuda")
        f = torch.empty((count, n, 3), dtype=torch.float32, device="cuda")
        self._check(self.lib.pamd_export_configs(self.ctx, run, int(r0), int(count), x.data_ptr(), f.data_ptr(),
                                                 self._s()), self.ctx)
        return x, f

    def set_mts(self, nn: Optional["PamdNN"], outer_ratio: int = 4) -> None:
        """Attach surrogate `nn` (r-RESPA, outer step outer_ratio * dt) or detach
        (None).  The per-run r-RESPA buffers are a torch allocation of the size
        the library asks for."""
        if nn is None:
            self._check(self.lib.pamd_set_mts(self.ctx, None, 0, None, 0, self._s()), self.ctx)
            self._mts_nn, self._mts_mem = None, None
            return
        nb = C.c_size_t()
        self._check(self.lib.pamd_mts_query_sizes(self.ctx, C.byref(nb)), self.ctx)
        mem = self.torch.empty(nb.value + 256, dtype=self.torch.uint8, device="cuda")
        ptr = (mem.data_ptr() + 255) // 256 * 256
        self._check(self.lib.pamd_set_mts(self.ctx, nn.handle, int(outer_ratio), C.c_void_p(ptr), nb.value,
                                          self._s()), self.ctx)
        self._mts_nn, self._mts_mem = nn, mem

    def get_counts(self, run: int = 0) -> np.ndarray:
        c = np.zeros(self.R_cap, np.int32)
        n = C.c_int64()
        self._check(self.lib.pamd_get_counts(self.ctx, run, _ptr(c), C.byref(n), self._s()), self.ctx)
        return c[:n.value].copy()

    def close(self) -> None:
        if getattr(self, "ctx", None):
            self.lib.pamd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack_params(w: Dict[str, np.ndarray]) -> np.ndarray:
    """Flat FP32 parameter vector (W1, b1, W2, b2, w3, b3) from a weight dict."""
    v = np.concatenate([np.asarray(w[k], np.float64).ravel() for k in ("W1", "b1", "W2", "b2", "w3", "b3")])
    assert v.size == NN_PARAMS
    return np.ascontiguousarray(v, np.float32)


def unpack_params(v: np.ndarray) -> Dict[str, np.ndarray]:
    v = np.asarray(v)
    F, H = NN_FEATURES, NN_HIDDEN
    o = np.cumsum([0, F * H, H, H * H, H, H, 1])
    return {"W1": v[o[0]:o[1]].reshape(F, H), "b1": v[o[1]:o[2]], "W2": v[o[2]:o[3]].reshape(H, H),
            "b2": v[o[3]:o[4]], "w3": v[o[4]:o[5]], "b3": v[o[5]:o[6]]}


class PamdNN:
    """The learned surrogate of one molecule (pamd_nn_* calls).  Configuration
    arrays are CUDA float32 tensors [n_conf, n, 3]."""

    def __init__(self, sysd, atom_type: Sequence[int], max_conf: int = 256, stream=None,
                 library: Optional[str] = None):
        """max_conf: the largest batch of forces / loss_grad / train_step; the
        parameters and workspace are one torch allocation of the size the
        library asks for.  library: another build of libpamd (default: the
        in-tree one)."""
        import torch
        self.torch = torch
        self.lib = load_library(library or LIB_PATH)
        if not torch.cuda.is_available():
            raise RuntimeError("the PAMD library needs a ROCm GPU")
        self._keep: list = []
        self._sys = make_system_struct(sysd, self._keep)
        self.n = int(sysd.n_atoms)
        t = np.ascontiguousarray(np.asarray(atom_type, np.int32))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.max_conf = int(max_conf)
        nb = C.c_size_t()
        st = self.lib.pamd_nn_query_sizes(self.n, self.max_conf, C.byref(nb))
        if st != PAMD_OK:
            raise PamdError(st, "pamd_nn_query_sizes: atom count or max_conf out of range")
        self._mem = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (self._mem.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        st = self.lib.pamd_nn_create(C.byref(self._sys), _ptr(t), self.max_conf, C.c_void_p(ptr), nb.value,
                                     self._s(), C.byref(h))
        if st != PAMD_OK:
            raise PamdError(st, "pamd_nn_create failed")
        self.handle = h

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _check(self, st: int):
        if st != PAMD_OK:
            raise PamdError(st, self.lib.pamd_nn_last_error(self.handle).decode())

    def set_weights(self, w) -> None:
        v = pack_params(w) if isinstance(w, dict) else np.ascontiguousarray(w, np.float32)
        self._check(self.lib.pamd_nn_set_weights(self.handle, _ptr(v), self._s()))

    def get_weights(self) -> Dict[str, np.ndarray]:
        v = np.zeros(NN_PARAMS, np.float32)
        self._check(self.lib.pamd_nn_get_weights(self.handle, _ptr(v), self._s()))
        return unpack_params(v)

    def forces(self, x):
        torch = self.torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        B = x.shape[0]
        F = torch.empty_like(x)
        E = torch.empty(B, dtype=torch.float32, device=x.device)
        self._check(self.lib.pamd_nn_forces(self.handle, B, x.data_ptr(), F.data_ptr(), E.data_ptr(), self._s()))
        return E, F

    def forces_static(self, x, F=None, E=None):
        """forces() through the allocation-free entry point (fixed library
        staging, n_conf * n <= NN_STATIC_ROWS); F and E may be given."""
        torch = self.torch
        assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()
        B = x.shape[0]
        F = torch.empty_like(x) if F is None else F
        E = torch.empty(B, dtype=torch.float32, device=x.device) if E is None else E
        self._check(self.lib.pamd_nn_forces_static(self.handle, B, x.data_ptr(), F.data_ptr(), E.data_ptr(),
                                                   self._s()))
        return E, F

    def loss_grad(self, x, F_target, want_grad: bool = True):
        torch = self.torch
        assert x.is_contiguous() and F_target.is_contiguous() and x.shape == F_target.shape
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        g = torch.empty(NN_PARAMS, dtype=torch.float32, device=x.device) if want_grad else None
        self._check(self.lib.pamd_nn_loss_grad(self.handle, x.shape[0], x.data_ptr(), F_target.data_ptr(),
                                               loss.data_ptr(), None if g is None else g.data_ptr(), self._s()))
        return loss, g

    def train_step(self, x, F_target, lr: float, loss=None) -> None:
        assert x.is_contiguous() and F_target.is_contiguous() and x.shape == F_target.shape
        self._check(self.lib.pamd_nn_train_step(self.handle, x.shape[0], x.data_ptr(), F_target.data_ptr(),
                                                float(lr), None if loss is None else loss.data_ptr(), self._s()))

    def close(self) -> None:
        if getattr(self, "handle", None):
            self.lib.pamd_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
