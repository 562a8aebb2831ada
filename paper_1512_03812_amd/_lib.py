"""ctypes declarations of the C ABI in include/schwinger_hmc.h (argument marshalling only)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libschwinger_hmc.so")

HMC_OK, HMC_E_INVAL, HMC_E_NOMEM, HMC_E_NOCONV, HMC_E_HIP, HMC_E_NAN = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {0: "HMC_OK", -1: "HMC_E_INVAL", -2: "HMC_E_NOMEM", -3: "HMC_E_NOCONV",
               -4: "HMC_E_HIP", -5: "HMC_E_NAN"}
(LEAPFROG, OMELYAN_5STAGE, FORCE_GRADIENT, NESTED_FG, ADAPTED_NESTED_FG, NESTED_LEAPFROG,
 NESTED_5STAGE, OMELYAN_11STAGE) = range(8)
SCHEMES = {"leapfrog": LEAPFROG, "omelyan": OMELYAN_5STAGE, "force_gradient": FORCE_GRADIENT,
           "nested_fg": NESTED_FG, "adapted_nested_fg": ADAPTED_NESTED_FG,
           "nested_leapfrog": NESTED_LEAPFROG, "nested_omelyan": NESTED_5STAGE,
           "omelyan_11stage": OMELYAN_11STAGE}
PREC_FP64, PREC_MIXED = 0, 1
PRECISIONS = {"fp64": PREC_FP64, "mixed": PREC_MIXED}
FORCE_GAUGE, FORCE_FERMION, FORCE_TOTAL = 0, 1, 2
FORCE_SETS = {"gauge": FORCE_GAUGE, "fermion": FORCE_FERMION, "total": FORCE_TOTAL}
FG_SHIFT, FG_EXACT = 0, 1
FG_MODES = {"shift": FG_SHIFT, "exact": FG_EXACT}
FIELD_Q, FIELD_P, FIELD_PHI, FIELD_CHI, FIELD_XI, FIELD_F, FIELD_ZETA = range(7)


class CGInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("reliable_updates", ctypes.c_int), ("pad", ctypes.c_int),
                ("rel_resid", ctypes.c_double), ("rel_resid_true", ctypes.c_double)]


class TrajInfo(ctypes.Structure):
    _fields_ = [("dH", ctypes.c_double), ("H0", ctypes.c_double), ("H1", ctypes.c_double),
                ("plaquette", ctypes.c_double), ("u", ctypes.c_double),
                ("accepted", ctypes.c_int), ("status", ctypes.c_int),
                ("n_force_evals", ctypes.c_int), ("n_solves", ctypes.c_int),
                ("n_dinv", ctypes.c_int), ("pad", ctypes.c_int),
                ("n_cg_iters", ctypes.c_longlong)]


class TuneSchedule(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("n_outer", ctypes.c_int), ("n_inner", ctypes.c_int),
                ("pad", ctypes.c_int), ("tau", ctypes.c_double)]


class TuneInfo(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("persistent_limit", ctypes.c_int),
                ("step_variant", ctypes.c_int), ("check_interval", ctypes.c_int),
                ("groups", ctypes.c_int), ("candidates", ctypes.c_int),
                ("reliable_delta", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("traj_ms", ctypes.c_double)]


STEP_VARIANTS = {"plain": 0, "two_sites": 1, "resident": 2, "waves8": 3}


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong), ("timed_launches", ctypes.c_longlong),
                ("timed_ms", ctypes.c_double), ("timed_bytes", ctypes.c_double),
                ("sample_every", ctypes.c_int), ("fused", ctypes.c_int),
                ("all_bytes", ctypes.c_double)]


# name -> (restype, argtypes)
_P, _I, _D, _U32, _U64, _SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint32,
                               ctypes.c_uint64, ctypes.c_size_t)
SIGNATURES = {
    "hmc_init": (_I, [_P, _I, _D, _D, _U64]),
    "hmc_init_ex": (_I, [_P, _I, _I, _D, _D, _U64]),
    "hmc_batch_init": (_I, [_P, _I, _P, _P, _P, _P, _U64]),
    "hmc_workspace_bytes": (_SZ, [_P]),
    "hmc_bind": (_I, [_P, _P, _SZ, _P]),
    "hmc_field": (_I, [_P, _I, _P, _P]),
    "hmc_mark_links_changed": (_I, [_P]),
    "hmc_geometry": (_I, [_P, _P, _P, _P, _P, _P]),
    "hmc_pack_links": (_I, [_P, _P, _P]),
    "hmc_unpack_links": (_I, [_P, _P, _P]),
    "hmc_pack_spinor": (_I, [_P, _P, _P]),
    "hmc_unpack_spinor": (_I, [_P, _P, _P]),
    "hmc_cold_start": (_I, [_P]),
    "hmc_hot_start": (_I, [_P]),
    "hmc_set_trajectory_counter": (_I, [_P, _U32]),
    "hmc_get_trajectory_counter": (_U32, [_P]),
    "hmc_set_solver": (_I, [_P, _D, _I, _D]),
    "hmc_set_quenched": (_I, [_P, _I]),
    "hmc_set_check_interval": (_I, [_P, _I]),
    "hmc_set_persistent_limit": (_I, [_P, _I]),
    "hmc_set_fused_cg": (_I, [_P, _I]),
    "hmc_set_cg_groups": (_I, [_P, _I]),
    "hmc_set_block_size": (_I, [_P, _I]),
    "hmc_autotune": (_I, [_P, _I, _D, _P, _P]),
    "hmc_set_step_variant": (_I, [_P, _I]),
    "hmc_dslash": (_I, [_P, _P, _P]),
    "hmc_dslash_dagger": (_I, [_P, _P, _P]),
    "hmc_cg_solve": (_I, [_P, _P, _P, _D, _I, _I, _P]),
    "hmc_cg_solve_noalloc": (_I, [_P, _P, _P, _D, _I, _P]),
    "hmc_fermion_force": (_I, [_P, _P, _P, _D, _I, _I, _P, _P]),
    "hmc_fermion_force_chixi": (_I, [_P, _P, _P, _P]),
    "hmc_total_force_chixi": (_I, [_P, _P, _P, _P]),
    "hmc_gauge_force": (_I, [_P, _P]),
    "hmc_actions": (_I, [_P, _P, _D, _P, _P, _P]),
    "hmc_update_links": (_I, [_P, _D]),
    "hmc_update_momenta": (_I, [_P, _D, _P]),
    "hmc_fg_shifted_force": (_I, [_P, _D, _I, _P, _P, _I, _P]),
    "hmc_hessian_vector": (_I, [_P, _I, _P, _P, _P, _I, _P]),
    "hmc_force_gradient_term": (_I, [_P, _I, _P, _P, _I, _P]),
    "hmc_set_fg_mode": (_I, [_P, _I]),
    "hmc_set_graph": (_I, [_P, _I]),
    "hmc_trajectory": (_I, [_P, _I, _D, _I, _I, _I, _P]),
    "hmc_trajectories_concurrent": (_I, [_P, _I, _I, _D, _I, _I, _I, _P, _P]),
    "hmc_integrate": (_I, [_P, _I, _D, _I, _I, _I, _P]),
    "hmc_refresh": (_I, [_P]),
    "hmc_set_timing": (_I, [_P, _I]),
    "hmc_get_kernel_stats": (_I, [_P, _I, _P]),
    "hmc_stream_copy": (_I, [_P, _P, _P, _SZ]),
    "hmc_last_error": (ctypes.c_char_p, [_P]),
    "hmc_destroy": (_I, [_P]),
}

_lib = None


def load():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "libschwinger_hmc.so is missing: build it first (python -m paper_1512_03812_amd.build "
                "or __graft_entry__.build()); there is no fallback implementation")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols():
    return sorted(SIGNATURES)
