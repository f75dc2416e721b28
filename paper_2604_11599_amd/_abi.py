"""ctypes declarations of libqsv's C ABI (include/qsv.h, include/qsv_plan.h).

Argument marshalling only: every step of the simulation runs in the library.
Importing this module fails loudly when the built library is missing; there is
no fallback implementation.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqsv.so")

QSV_OK, QSV_ERR_ARG, QSV_ERR_PARSE, QSV_ERR_UNSUPPORTED = 0, -1, -2, -3
QSV_ERR_NOMEM, QSV_ERR_DEVICE, QSV_ERR_FORCED_ZERO_PROB, QSV_ERR_LIMIT = -4, -5, -6, -7
QSV_FLAG_PROFILE, QSV_FLAG_DEVICE_PTRS, QSV_FLAG_NULL_STREAM, QSV_FLAG_TUNED_PLANS = 1, 2, 4, 8
QSV_RUN_SHARE_TRAJ = 1
QSV_RUN_COMPLEX64 = 2
QSV_RUN_GRAPH = 4
STATUS_NAMES = {0: "QSV_OK", -1: "QSV_ERR_ARG", -2: "QSV_ERR_PARSE", -3: "QSV_ERR_UNSUPPORTED",
                -4: "QSV_ERR_NOMEM", -5: "QSV_ERR_DEVICE", -6: "QSV_ERR_FORCED_ZERO_PROB",
                -7: "QSV_ERR_LIMIT"}
PLAN_MAX_STEPS, PLAN_MAX_GATES = 4096, 65536
NOALLOC_SCRATCH_BYTES = 64 << 20


class Config(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("arena", C.c_void_p),
                ("arena_bytes", C.c_size_t), ("flags", C.c_uint32)]


class ProgramDesc(C.Structure):
    _fields_ = [("n_qubits", C.c_uint32), ("n_clbits", C.c_uint32), ("n_params", C.c_uint32),
                ("n_instr", C.c_uint32), ("n_pred", C.c_uint32), ("reserved", C.c_uint32),
                ("instr", C.c_void_p), ("pred", C.c_void_p), ("n_code", C.c_uint32), ("reserved2", C.c_uint32),
                ("code", C.c_void_p), ("n_lin", C.c_uint32), ("n_derived", C.c_uint32), ("lin", C.c_void_p),
                ("n_noise", C.c_uint32), ("reserved3", C.c_uint32), ("noise", C.c_void_p)]


class ProgramInfo(C.Structure):
    _fields_ = [("n_qubits", C.c_uint32), ("n_clbits", C.c_uint32), ("n_params", C.c_uint32),
                ("max_events", C.c_uint32), ("n_passes", C.c_uint32), ("n_sites", C.c_uint32),
                ("is_unitary", C.c_uint8)]


class RunOpts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("shot_offset", C.c_uint64), ("forced", C.c_void_p),
                ("forced_len", C.c_uint32), ("flags", C.c_uint32), ("state_out", C.c_void_p),
                ("readout_error", C.c_double), ("reset_error", C.c_double), ("depolarizing", C.c_double)]


class ShotResults(C.Structure):
    _fields_ = [("creg", C.c_void_p), ("record", C.c_void_p), ("n_events", C.c_void_p),
                ("record_prob", C.c_void_p), ("shot_status", C.c_void_p)]


class Request(C.Structure):
    _fields_ = [("prog", C.c_void_p), ("theta", C.c_void_p), ("n_shots", C.c_uint64),
                ("opts", RunOpts), ("out", ShotResults)]


class PauliSum(C.Structure):
    _fields_ = [("n_terms", C.c_uint32), ("reserved", C.c_uint32), ("coeff", C.c_void_p),
                ("pauli", C.c_void_p)]


class PlanStats(C.Structure):
    _fields_ = [("n_steps", C.c_uint32), ("n_passes", C.c_uint32), ("n_sites", C.c_uint32),
                ("n_gates", C.c_uint32), ("n_events", C.c_uint32), ("max_record", C.c_uint32),
                ("is_unitary", C.c_uint8), ("init_step", C.c_uint8), ("reserved", C.c_uint8 * 6),
                ("step_kind", C.c_uint8 * PLAN_MAX_STEPS), ("step_mask", C.c_uint64 * PLAN_MAX_STEPS),
                ("step_count", C.c_uint32 * PLAN_MAX_STEPS), ("gate_instr", C.c_uint32 * PLAN_MAX_GATES),
                ("gate_regs", C.c_uint64 * PLAN_MAX_GATES), ("n_phases", C.c_uint32), ("n_dense_phases", C.c_uint32),
                ("n_mfma_sweep_passes", C.c_uint32)]


class PlanOptions(C.Structure):
    _fields_ = [("tile_bits", C.c_uint32), ("low_bits", C.c_uint32), ("dense_min_cost", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("best", PlanOptions), ("deflt", PlanOptions), ("best_ms", C.c_double), ("default_ms", C.c_double),
                ("n_candidates", C.c_uint32), ("reserved", C.c_uint32), ("arch", C.c_char * 64)]


class Profile(C.Structure):
    _fields_ = [("pass_launches", C.c_uint64), ("pass_ms", C.c_double),
                ("pass_uncond_launches", C.c_uint64), ("pass_uncond_ms", C.c_double),
                ("pass_uncond_bytes", C.c_double), ("pass_uncond_flops", C.c_double),
                ("site_launches", C.c_uint64), ("site_ms", C.c_double),
                ("other_launches", C.c_uint64), ("other_ms", C.c_double),
                ("ham_launches", C.c_uint64), ("ham_ms", C.c_double), ("ham_bytes", C.c_double),
                ("sweep_launches", C.c_uint64), ("sweep_ms", C.c_double), ("sweep_bytes", C.c_double),
                ("persistent_launches", C.c_uint64), ("persistent_ms", C.c_double),
                ("persistent_bytes", C.c_double)]


# name -> (restype, argtypes); the ABI surface the tests check for.
SIGNATURES = {
    "qsv_create": (C.c_int32, [C.POINTER(Config), C.POINTER(C.c_void_p)]),
    "qsv_destroy": (None, [C.c_void_p]),
    "qsv_last_error": (C.c_char_p, [C.c_void_p]),
    "qsv_load_program": (C.c_int32, [C.c_void_p, C.POINTER(ProgramDesc), C.POINTER(C.c_void_p)]),
    "qsv_program_info_get": (C.c_int32, [C.c_void_p, C.POINTER(ProgramInfo)]),
    "qsv_program_free": (None, [C.c_void_p]),
    "qsv_run_shots": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(RunOpts),
                                  C.POINTER(ShotResults)]),
    "qsv_run_shots_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(RunOpts),
                                          C.POINTER(ShotResults)]),
    "qsv_run_batch": (C.c_int32, [C.c_void_p, C.POINTER(Request), C.c_uint32]),
    "qsv_expval": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(PauliSum),
                               C.c_void_p]),
    "qsv_expval_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(PauliSum),
                                    C.c_void_p, C.c_void_p]),
    "qsv_plan_inspect": (C.c_int32, [C.POINTER(ProgramDesc), C.c_uint32, C.POINTER(PlanStats)]),
    "qsv_server_create": (C.c_int32, [C.c_void_p, C.c_size_t, C.c_uint32, C.POINTER(C.c_void_p)]),
    "qsv_server_destroy": (None, [C.c_void_p]),
    "qsv_submit": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64,
                               C.POINTER(C.c_uint64)]),
    "qsv_submit_expval_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(PauliSum),
                                           C.POINTER(C.c_uint64)]),
    "qsv_server_step": (C.c_int32, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]),
    "qsv_poll": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int32)]),
    "qsv_fetch_shots": (C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(ShotResults)]),
    "qsv_fetch_expval_grad": (C.c_int32, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p]),
    "qsv_profile_read": (C.c_int32, [C.c_void_p, C.POINTER(Profile)]),
    "qsv_diag_copy": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "qsv_profile_reset": (C.c_int32, [C.c_void_p]),
    "qsv_autotune": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                 C.POINTER(TuneReport)]),
    "qsv_program_plan_get": (C.c_int32, [C.c_void_p, C.POINTER(PlanOptions)]),
    "qsv_program_replan": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(PlanOptions)]),
    "qsv_tune_lookup": (C.c_int32, [C.c_void_p, C.c_uint32, C.c_uint32, C.POINTER(PlanOptions),
                                    C.POINTER(C.c_int32)]),
    "qsv_tune_export": (C.c_int32, [C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "qsv_tune_import": (C.c_int32, [C.c_char_p]),
    "qsv_context_fork": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "qsv_expval_grad_each": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    "qsv_server_profile": (C.c_int32, [C.c_void_p, C.POINTER(Profile)]),
}


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libqsv.so is not built at {path}; run __graft_entry__.build() first")
    # One HIP runtime per process: torch ships its own libamdhip64 under the
    # same soname. Loaded first, it is the runtime libqsv binds to as well;
    # loaded after libqsv had pulled in the system runtime, torch would bring a
    # second runtime that finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB
