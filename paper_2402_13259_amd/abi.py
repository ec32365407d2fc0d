"""ctypes declarations of the C ABI in include/eulerq.h: constants, structs and the argument
and result types of every exported function.  Declarations only: `configure(lib)` applies them
to a loaded library.  The binding uses it for libeulerq.so; the sanitizer tests for the same
sources built for the host.
"""
import ctypes as C

EQ_OK, EQ_EINVAL, EQ_ENOTDAG, EQ_ENOMEM, EQ_EDEVICE, EQ_EOVERFLOW = 0, -1, -2, -3, -4, -5
EQ_BACKWARD, EQ_FORWARD = 0, 1
EQ_DEP_EXACT, EQ_DEP_NAIVE = 0, 1
EQ_SHAPE_CONST, EQ_SHAPE_SINUSOID = 0, 1
EQ_KERNEL_AUTO, EQ_KERNEL_TILE, EQ_KERNEL_SWEEP = 0, 1, 2
STAT_TILE_REPS = 32       # EQ_STAT_TILE_REPS: replications per statistics tile of the sums
EQ_NOALLOC_SCRATCH_BYTES = 64 << 20   # static scratch of eq_sim_run_noalloc

EXPORTS = ["eq_net_create", "eq_net_destroy", "eq_net_set_staffing", "eq_net_set_params", "eq_sim_run_host", "eq_net_tables", "eq_net_levels", "eq_sim_workspace_bytes",
           "eq_sim_run", "eq_sim_run_noalloc", "eq_sim_tune", "eq_sim_run_pair", "eq_stats_reduce", "eq_stats_reduce_pair",
           "eq_sim_run_record", "eq_sojourn", "eq_sim_check", "eq_batch_create", "eq_batch_destroy",
           "eq_batch_layout", "eq_batch_run", "eq_batch_tune", "eq_batch_check", "eq_sim_run_scores", "eq_cost_reduce",
           "eq_grad_reduce", "eq_grad_reduce_reach", "eq_net_reach", "eq_selftest_math", "eq_selftest_sample", "eq_selftest_score", "eq_selftest_valu_peak", "eq_selftest_philox",
           "eq_last_error"]



class eq_arrivals(C.Structure):
    """eq_arrivals of eulerq.h: sources, base rates and the arrival shape (constant, sinusoid, piecewise)."""
    _fields_ = [("n_src", C.c_int32), ("src", C.c_void_p), ("lambda0", C.c_void_p), ("shape_kind", C.c_int32),
                ("amp", C.c_double), ("period", C.c_double), ("phase", C.c_double), ("n_knots", C.c_int32),
                ("knot_t", C.c_void_p), ("knot_shape", C.c_void_p)]


class eq_run_desc(C.Structure):
    """eq_run_desc of eulerq.h: scheme, departure rule, step, steps, seed, network id, replications, kernel."""
    _fields_ = [("scheme", C.c_int32), ("dep_mode", C.c_int32), ("dt", C.c_float), ("n_steps", C.c_int32),
                ("seed", C.c_uint64), ("net_id", C.c_uint32), ("rep0", C.c_int32), ("reps", C.c_int32),
                ("kernel", C.c_int32), ("tile_reps", C.c_int32), ("block", C.c_int32)]


class eq_batch_desc(C.Structure):
    """eq_batch_desc of eulerq.h: the run shape shared by every network of a batch."""
    _fields_ = [("scheme", C.c_int32), ("dep_mode", C.c_int32), ("dt", C.c_float), ("seed", C.c_uint64),
                ("reps", C.c_int32), ("waves_per_block", C.c_int32), ("use_graph", C.c_int32)]


_vp, _i32, _i64, _u32, _u64, _f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_float
_sig = {
    "eq_net_create": ([_i32, _vp, _vp, _vp, _vp, _vp, C.POINTER(eq_arrivals), C.POINTER(_vp)], C.c_int),
    "eq_net_destroy": ([_vp], None),
    "eq_net_set_staffing": ([_vp, _i32, _vp, _vp, _i32], C.c_int),
    "eq_net_set_params": ([_vp, _vp, _vp], C.c_int),
    "eq_sim_run_host": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp], C.c_int),
    "eq_net_tables": ([_vp, _f32, _i32, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_net_levels": ([_vp, _vp], C.c_int),
    "eq_sim_workspace_bytes": ([_vp, C.POINTER(eq_run_desc)], C.c_size_t),
    "eq_sim_run": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _vp], C.c_int),
    "eq_sim_run_noalloc": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _vp], C.c_int),
    "eq_sim_tune": ([_vp, C.POINTER(eq_run_desc), _i32, _vp, _vp, C.POINTER(eq_run_desc)], C.c_int),
    "eq_stats_reduce": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_sim_run_pair": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_sim_run_record": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "eq_sojourn": ([_vp, C.POINTER(eq_run_desc), _i32, _i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp], C.c_int),
    "eq_stats_reduce_pair": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_sim_check": ([_vp, _vp], C.c_int),
    "eq_batch_create": ([_i32, _vp, C.POINTER(_vp)], C.c_int),
    "eq_batch_destroy": ([_vp], None),
    "eq_batch_layout": ([_vp, _i32, _vp, _vp], C.c_int),
    "eq_batch_run": ([_vp, C.POINTER(eq_batch_desc), _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_batch_tune": ([_vp, C.POINTER(eq_batch_desc), _vp, _vp, _f32, _vp, _vp, _vp, C.POINTER(_i32)], C.c_int),
    "eq_batch_check": ([_vp, _vp], C.c_int),
    "eq_selftest_math": ([_i32, _vp, _vp, _i64, _vp], C.c_int),
    "eq_selftest_sample": ([_i32, _i64, _u64, _u32, _u32, _u32, _u32, _i32, _i32, _f32, _f32, _f32, _f32, _vp, _vp],
                           C.c_int),
    "eq_sim_run_scores": ([_vp, C.POINTER(eq_run_desc), _vp, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_cost_reduce": ([_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_grad_reduce": ([_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_grad_reduce_reach": ([_vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp], C.c_int),
    "eq_net_reach": ([_vp, _vp], C.c_int),
    "eq_selftest_score": ([_i32, _i64, _u64, _u32, _u32, _u32, _u32, _i32, _i32, _f32, _f32, _vp, _vp, _vp],
                          C.c_int),
    "eq_selftest_valu_peak": ([_i32, _i32, _vp, _vp], C.c_int),
    "eq_selftest_philox": ([_i64, _vp, _vp, _vp, _vp], C.c_int),
    "eq_last_error": ([], C.c_char_p),
}


def configure(lib) -> dict:
    """Set argtypes / restype of every exported function on `lib`; returns {name: function}."""
    out = {}
    for name, (args, res) in _sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
        out[name] = f
    return out
