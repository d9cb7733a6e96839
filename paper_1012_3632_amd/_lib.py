"""ctypes binding of libflb.so (argument marshalling only).

Every call goes straight to the C ABI declared in include/flb.h; no step of the
method runs in Python.  Importing this module fails loudly if the library has
not been built (``python paper_1012_3632_amd/build.py``).
"""

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflb.so")

FLB_D2Q9, FLB_D3Q19 = 0, 1
FLB_FP32, FLB_FP64 = 0, 1
FLB_IDEAL, FLB_LANDAU = 0, 1

STATUS = {0: "FLB_OK", -1: "FLB_ERR_INVALID_ARG", -2: "FLB_ERR_HIP", -3: "FLB_ERR_NONFINITE",
          -4: "FLB_ERR_UNSUPPORTED", -5: "FLB_ERR_STATE"}


class FLBError(RuntimeError):
    def __init__(self, status, func, msg):
        self.status = status
        super().__init__(f"{func}: {STATUS.get(status, status)}: {msg}")


class flb_params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int32), ("precision", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("force_model", C.c_int32), ("eta", C.c_int32), ("noise_rho_local", C.c_int32),
        ("rho0", C.c_double), ("kT", C.c_double),
        ("rate_bulk", C.c_double), ("rate_shear", C.c_double), ("rate_ghost", C.c_double),
        ("a", C.c_double), ("b", C.c_double), ("rho_c", C.c_double), ("kappa", C.c_double),
        ("seed", C.c_uint64), ("step0", C.c_uint64),
        ("replica", C.c_uint32), ("reserved", C.c_uint32),
    ]


class flb_interface(C.Structure):
    _fields_ = [("y_ref", C.c_double), ("sign", C.c_int32), ("half_window", C.c_int32)]


class flb_modeq_params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32), ("reserved", C.c_int32),
        ("rho0", C.c_double), ("kT", C.c_double), ("cs2_0", C.c_double), ("kappa", C.c_double),
        ("rate_bulk", C.c_double), ("rate_shear", C.c_double), ("rate_ghost", C.c_double),
        ("seed", C.c_uint64),
    ]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python paper_1012_3632_amd/build.py)")

lib = C.CDLL(LIB_PATH)

P = C.POINTER
vp = C.c_void_p
PROTOS = {
    "flb_query_sizes": [P(flb_params), P(C.c_size_t), P(C.c_size_t), P(C.c_size_t)],
    "flb_init": [P(flb_params), vp, vp, vp, vp, vp, vp, P(vp)],
    "flb_step": [vp, C.c_int64, C.c_int32, vp],
    "flb_set_check": [vp, C.c_int64, vp],
    "flb_state": [vp, P(vp), P(vp), P(C.c_uint64)],
    "flb_seek": [vp, C.c_uint64, vp],
    "flb_moments": [vp, P(C.c_double), P(C.c_double), P(C.c_int64), vp],
    "flb_reset_stats": [vp, vp],
    "flb_fields": [vp, vp, vp],
    "flb_noise_words": [P(flb_params), C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64,
                        C.c_uint64, vp, vp],
    "flb_lattice_tables": [C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_double),
                           P(C.c_double), P(C.c_double), P(C.c_int32)],
    "flb_graph_capture": [vp, C.c_int64, C.c_int32, vp],
    "flb_graph_launch": [vp, vp],
    "flb_adjoint_step": [vp, vp, vp, vp, P(C.c_double), C.c_uint64, vp],
    "flb_adjoint_density_seed": [vp, vp, vp, vp],
    "flb_adjoint_segment": [vp, vp, vp, vp, C.c_uint64, C.c_uint64, P(C.c_double), vp],
    "flb_adjoint_segment_bytes": [vp, C.c_int64, P(C.c_size_t)],
    "flb_density": [vp, vp, vp, vp],
    "flb_mode_fields": [vp, vp, vp],
    "flb_spectrum_work_bytes": [vp, P(C.c_size_t)],
    "flb_mode_spectrum": [vp, vp, vp, vp],
    "flb_field_spectrum": [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp],
    "flb_interface_heights": [vp, P(flb_interface), C.c_int32, C.c_double, C.c_double,
                              C.c_double, vp, vp],
    "flb_destroy": [vp],
    "flb_batch_query_sizes": [P(flb_params), C.c_int32, P(C.c_int32), P(C.c_size_t),
                              P(C.c_size_t), P(C.c_size_t)],
    "flb_batch_init": [P(flb_params), C.c_int32, P(C.c_int32), P(C.c_uint64), vp, vp, vp, vp,
                       vp, P(vp)],
    "flb_batch_step": [vp, C.c_int64, C.c_int32, vp],
    "flb_batch_moments": [vp, P(C.c_double), P(C.c_double), P(C.c_int64), vp],
    "flb_batch_state": [vp, P(vp), P(vp), P(C.c_uint64)],
    "flb_batch_reset_stats": [vp, vp],
    "flb_batch_graph_capture": [vp, C.c_int64, C.c_int32, vp],
    "flb_batch_graph_launch": [vp, vp],
    "flb_batch_destroy": [vp],
    "flb_autotune": [vp, C.c_int32, P(C.c_int32), P(C.c_double), vp],
    "flb_set_launch": [vp, C.c_int32],
    "flb_launch_configs": [vp, P(C.c_int32), P(C.c_int32)],
    "flb_launch_shape": [vp, C.c_int32, P(C.c_int32)],
    "flb_noise_normals": [vp, C.c_uint64, C.c_uint64, C.c_uint64, vp, vp],
    "flb_adjoint_run": [vp, P(vp), C.c_int32, C.c_int64, C.c_int64, vp, vp, P(C.c_double), vp],
    "flb_adjoint_run_bytes": [vp, C.c_int64, P(C.c_size_t)],
    "flb_batch_autotune": [vp, C.c_int32, P(C.c_int32), P(C.c_double), vp],
    "flb_batch_set_pairs": [vp, C.c_uint64],
    "flb_batch_pairs": [vp, P(C.c_uint64), P(C.c_int32)],
    "flb_modeq_work_bytes": [P(flb_modeq_params), P(C.c_size_t)],
    "flb_modeq_step": [P(flb_modeq_params), vp, vp, C.c_uint64, vp, C.c_size_t, vp],
    "flb_modeq_run": [P(flb_modeq_params), vp, vp, C.c_uint64, C.c_int32, vp, C.c_size_t, vp],
    "flb_modeq_noise": [P(flb_modeq_params), C.c_uint64, vp, vp, C.c_size_t, vp],
    "flb_modeq_moments": [P(flb_modeq_params), vp, vp, vp],
    "flb_plane_stream_probe": [vp, vp, C.c_int32, C.c_uint64, C.c_int32, vp],
    "flb_modeq_step_noalloc": [P(flb_modeq_params), vp, vp, C.c_uint64, vp],
    "flb_modeq_static_work_bytes": [P(C.c_size_t)],
}

for _name, _args in PROTOS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int

lib.flb_strerror.argtypes = [C.c_int]
lib.flb_strerror.restype = C.c_char_p
lib.flb_last_error.argtypes = []
lib.flb_last_error.restype = C.c_char_p


def check(status, func):
    if status != 0:
        raise FLBError(status, func, lib.flb_last_error().decode(errors="replace"))


def call(name, *args):
    check(getattr(lib, name)(*args), name)


def declared_symbols(header=None):
    """Function names declared in include/flb.h (for the export check)."""
    import re
    header = header or os.path.join(HERE, "..", "include", "flb.h")
    txt = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:flb_status|const char\*)\s+(flb_\w+)\s*\(", txt, re.M)))
