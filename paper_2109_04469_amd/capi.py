"""ctypes declarations of libpic's C ABI (include/pic.h). Marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_EHIP, PIC_ECAPACITY, PIC_EUNSTABLE, PIC_ETABLE, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
FLAG_NO_FIELD, FLAG_FIXED_E, FLAG_NO_COLL, FLAG_IMMOBILE_IONS, FLAG_RECORD, FLAG_THOMAS = 1, 2, 4, 8, 16, 32
NCOUNTERS = 16
NTIMERS = 10
TIMER_NAMES = ["field", "electron", "ion", "sort", "e_decide", "e_emit", "e_rare", "i_decide",
               "i_emit", "i_rare"]
COUNTER_NAMES = [
    "steps", "e_pushed", "i_pushed", "e_absorbed", "e_reflected", "i_absorbed", "se_emitted",
    "e_candidates", "e_elastic", "e_excitation", "e_ionization", "i_candidates", "i_isotropic",
    "i_backward", "reflect_lost", "beyond_table",
]


class PicParams(ctypes.Structure):
    _fields_ = [
        ("gap_m", ctypes.c_double), ("pressure_pa", ctypes.c_double),
        ("gas_temp_k", ctypes.c_double), ("rf_voltage_v", ctypes.c_double),
        ("rf_freq_hz", ctypes.c_double),
        ("steps_per_cycle", ctypes.c_int32), ("n_cells", ctypes.c_int32),
        ("weight", ctypes.c_double), ("area_m2", ctypes.c_double),
        ("reflection", ctypes.c_double), ("gamma_see", ctypes.c_double),
        ("see_temp_ev", ctypes.c_double),
        ("capacity", ctypes.c_int64 * 2),
        ("ion_subcycle", ctypes.c_int32), ("sort_interval", ctypes.c_int32),
        ("seed", ctypes.c_uint32), ("run", ctypes.c_uint32),
        ("eepf_bins", ctypes.c_int32),
        ("eepf_emax_ev", ctypes.c_double), ("eepf_halfwidth_m", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


class PicXsec(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("dv_e", ctypes.c_double), ("dv_i", ctypes.c_double),
        ("sigma_e", ctypes.POINTER(ctypes.c_double) * 3),
        ("sigma_i", ctypes.POINTER(ctypes.c_double) * 2),
        ("exc_threshold_ev", ctypes.c_double), ("ion_threshold_ev", ctypes.c_double),
    ]


class PicDerived(ctypes.Structure):
    _fields_ = [
        ("n_x", ctypes.c_int32), ("n_tiles_max", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("gas_density", ctypes.c_double),
        ("nu_max", ctypes.c_double * 2), ("p_coll", ctypes.c_double * 2),
    ]


class PicMomentsOut(ctypes.Structure):
    _fields_ = [
        ("n_e", ctypes.POINTER(ctypes.c_double)), ("n_i", ctypes.POINTER(ctypes.c_double)),
        ("mean_energy_e", ctypes.POINTER(ctypes.c_double)), ("eepf", ctypes.POINTER(ctypes.c_double)),
        ("steps_averaged", ctypes.c_int64),
    ]


_D2 = ctypes.c_double * 2
_I2 = ctypes.c_int64 * 2
_DP = ctypes.POINTER(ctypes.c_double)


class PicPassTrial(ctypes.Structure):
    _fields_ = [
        ("pipeline", ctypes.c_int), ("decide_block", ctypes.c_int), ("decide_wg_per_cu", ctypes.c_int),
        ("emit_wg_per_cu", ctypes.c_int), ("us_per_step", ctypes.c_double),
    ]


class PicWallOut(ctypes.Structure):
    _fields_ = [
        ("arrivals", _I2 * 2), ("absorbed", _I2 * 2), ("flux", _D2 * 2), ("absorbed_flux", _D2 * 2),
        ("mean_energy_ev", _D2 * 2), ("fedf", (_DP * 2) * 2), ("fedf_emax_ev", _D2),
        ("fedf_bins", ctypes.c_int32), ("ionizations", ctypes.c_int64),
        ("ionization_rate", ctypes.c_double), ("steps_averaged", ctypes.c_int64),
    ]


class PicMonitors(ctypes.Structure):
    _fields_ = [
        ("omega_pe_dt", ctypes.c_double), ("p_coll", _D2), ("n_e_max", ctypes.c_double),
        ("n_e_center", ctypes.c_double), ("mean_energy_center_ev", ctypes.c_double),
        ("lambda_d_m", ctypes.c_double), ("dx_over_lambda_d", ctypes.c_double),
        ("n_d", ctypes.c_double), ("steps_averaged", ctypes.c_int64),
    ]


_lib = None


def load():
    """Loads the in-tree libpic.so; fails loudly if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__; __graft_entry__.build()')")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    L.pic_workspace_bytes.argtypes = [ctypes.POINTER(PicParams), ctypes.POINTER(PicXsec), ctypes.POINTER(u64)]
    L.pic_init.argtypes = [ctypes.POINTER(PicParams), ctypes.POINTER(PicXsec), P, u64, P, ctypes.POINTER(P)]
    L.pic_set_state.argtypes = [P, ctypes.c_int, P, P, P, P, i64, i64]
    L.pic_get_state.argtypes = [P, ctypes.c_int, P, P, P, P, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.pic_step.argtypes = [P, i64]
    L.pic_step_many.argtypes = [ctypes.POINTER(P), ctypes.c_int, i64, i64]
    L.pic_batch_workspace_bytes.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(u64)]
    L.pic_batch_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P, u64, ctypes.POINTER(P)]
    L.pic_batch_step.argtypes = [P, i64]
    L.pic_batch_free.argtypes = [P]
    L.pic_batch_free.restype = None
    L.pic_load_profile.argtypes = [P, ctypes.c_int, i64, P, P, ctypes.c_int, i64]
    f32 = ctypes.c_float
    L.pic_mlp_workspace_bytes.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(u64)]
    L.pic_mlp_init.argtypes = [ctypes.c_int] * 5 + [P, u64, P, ctypes.POINTER(P)]
    L.pic_mlp_num_params.argtypes = [P, ctypes.POINTER(i64)]
    L.pic_mlp_set_params.argtypes = [P, P]
    L.pic_mlp_get_params.argtypes = [P, P]
    L.pic_mlp_forward.argtypes = [P, P, ctypes.c_int, P]
    L.pic_mlp_grad.argtypes = [P, P, P, ctypes.c_int]
    L.pic_mlp_get_grad.argtypes = [P, P]
    L.pic_mlp_get_loss.argtypes = [P, ctypes.POINTER(f32)]
    L.pic_mlp_adam.argtypes = [P, f32, f32, f32, f32, f32]
    L.pic_mlp_train_step.argtypes = [P, P, P, ctypes.c_int, f32, f32, f32, f32, f32]
    L.pic_mlp_free.argtypes = [P]
    L.pic_mlp_free.restype = None
    L.pic_mlp_forward_static.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, P, P]
    L.pic_sync.argtypes = [P]
    L.pic_set_field.argtypes = [P, P]
    L.pic_get_field.argtypes = [P, P, P, P, P, P]
    L.pic_measure.argtypes = [P, ctypes.c_int]
    L.pic_moments.argtypes = [P, ctypes.POINTER(PicMomentsOut), ctypes.c_int]
    L.pic_wall_moments.argtypes = [P, ctypes.POINTER(PicWallOut)]
    L.pic_get_monitors.argtypes = [P, ctypes.POINTER(PicMonitors)]
    L.pic_set_launch.argtypes = [P, ctypes.c_int, ctypes.c_int]
    L.pic_set_pipeline.argtypes = [P, ctypes.c_int]
    L.pic_set_decide_block.argtypes = [P, ctypes.c_int]
    L.pic_tune.argtypes = [P, i64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.pic_tune_pass.argtypes = [P, i64, ctypes.POINTER(PicPassTrial), ctypes.c_int,
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.pic_get_counters.argtypes = [P, P]
    L.pic_get_decisions.argtypes = [P, ctypes.c_int, P, i64, ctypes.POINTER(i64)]
    L.pic_get_derived.argtypes = [P, ctypes.POINTER(PicDerived)]
    L.pic_free.argtypes = [P]
    L.pic_free.restype = None
    L.pic_strerror.argtypes = [ctypes.c_int]
    L.pic_strerror.restype = ctypes.c_char_p
    L.pic_timing.argtypes = [P, ctypes.c_int]
    L.pic_get_timing.argtypes = [P, P, P, ctypes.c_int]
    L.pic_selftest_philox.argtypes = [P, P, P, i64, P]
    L.pic_selftest_sqrt.argtypes = [P, P, i64, P]
    L.pic_selftest_copy.argtypes = [P, P, i64, P]
    for name in ("pic_workspace_bytes", "pic_init", "pic_set_state", "pic_get_state", "pic_step",
                 "pic_step_many", "pic_batch_workspace_bytes", "pic_batch_create", "pic_batch_step",
                 "pic_load_profile", "pic_wall_moments", "pic_get_monitors", "pic_set_launch", "pic_set_pipeline", "pic_set_decide_block", "pic_tune", "pic_tune_pass", "pic_mlp_workspace_bytes", "pic_mlp_init", "pic_mlp_num_params",
                 "pic_mlp_set_params", "pic_mlp_get_params", "pic_mlp_forward", "pic_mlp_grad",
                 "pic_mlp_get_grad", "pic_mlp_get_loss", "pic_mlp_adam", "pic_mlp_train_step",
                 "pic_mlp_forward_static",
                 "pic_sync", "pic_set_field", "pic_get_field", "pic_measure", "pic_moments",
                 "pic_get_counters", "pic_get_decisions", "pic_get_derived",
                 "pic_selftest_philox", "pic_selftest_sqrt", "pic_selftest_copy", "pic_timing",
                 "pic_get_timing"):
        getattr(L, name).restype = ctypes.c_int
    _ = i32
    _lib = L
    return L


class PicError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = load().pic_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def check(status, what=""):
    if status != PIC_OK:
        raise PicError(status, what)
