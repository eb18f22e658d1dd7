"""ctypes loader of libddf.so and the argument types of its C ABI (include/ddf.h).

Nothing here computes: it only marshals pointers and sizes.  Loading fails loudly
when the library has not been built; there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddf.so")

c_f = ctypes.c_float
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u32 = ctypes.c_uint32
c_u64 = ctypes.c_uint64
c_sz = ctypes.c_size_t
c_p = ctypes.c_void_p
STATUS = ctypes.c_int32

DDF_OK, DDF_ERR_INVALID_ARG, DDF_ERR_UNSUPPORTED, DDF_ERR_WORKSPACE, DDF_ERR_HIP = 0, 1, 2, 3, 4
PREC_FP32, PREC_BF16, PREC_FP8 = 0, 1, 2


class DdfNet(ctypes.Structure):
    _fields_ = [("width", c_i32), ("depth", c_i32), ("precision", c_i32), ("packed", c_p)]


class DdfPaperNet(ctypes.Structure):
    _fields_ = [("depth", c_i32), ("precision", c_i32), ("packed", c_p)]


class DdfInstance(ctypes.Structure):
    _fields_ = [("R", c_f * 9), ("T", c_f * 3), ("net", c_i32)]


class DdfScene(ctypes.Structure):
    _fields_ = [("backend", c_i32), ("tris", c_p), ("m", c_i64), ("net", ctypes.POINTER(DdfNet)),
                ("n_nets", c_i32), ("nets", ctypes.POINTER(DdfNet)), ("n_instances", c_i32),
                ("instances", ctypes.POINTER(DdfInstance))]


class DdfRenderParams(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("spp", c_i32), ("bounces", c_i32), ("rr_start", c_i32),
                ("seed", ctypes.c_uint64), ("eps", c_f), ("eye", c_f * 3), ("target", c_f * 3), ("up", c_f * 3),
                ("vfov_deg", c_f), ("light_pos", c_f * 3), ("light_intensity", c_f * 3), ("albedo", c_f * 3),
                ("spp_chunk", c_i32)]


BACKEND_MESH, BACKEND_NET, BACKEND_MULTI = 0, 1, 2


class DdfLoss(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("delta", c_f)]


LOSSES = {"bce_l1": 0, "clamp": 1, "squish": 2}


class DdfDatasetParams(ctypes.Structure):
    _fields_ = [("s_fc", c_i32), ("s_dr", c_i32), ("s_p", c_i32), ("eps", c_f), ("face_first", c_i64),
                ("n_faces", c_i64)]

# name -> argument types (every entry point returns ddf_status unless listed in _RESTYPE)
SIGNATURES = {
    "ddf_abi_version": [],
    "ddf_last_error": [],
    "ddf_label_rays": [c_p, c_p, c_i64, c_p, c_i64, c_f, c_f, c_p, c_p, c_p, c_p],
    "ddf_assemble_rays": [c_p, c_p, c_i64, c_p, c_p],
    "ddf_packed_bytes": [c_i32, c_i32, c_i32, ctypes.POINTER(c_sz)],
    "ddf_pack_net": [c_p, c_i32, c_i32, c_i32, c_p, c_p, c_p],
    "ddf_fp8_scales": [ctypes.POINTER(DdfNet), c_p, c_p, c_i64, c_p, c_p],
    "ddf_forward": [ctypes.POINTER(DdfNet), c_p, c_i64, c_p, c_p, c_p],
    "ddf_query": [ctypes.POINTER(DdfNet), c_p, c_p, c_i64, c_p, c_p, c_p],
    "ddf_train_workspace_size": [c_i32, c_i32, c_i64, ctypes.POINTER(c_sz)],
    "ddf_backward": [ctypes.POINTER(DdfNet), c_p, c_i64, c_p, c_p, c_p, c_p, c_u32, c_p, c_sz, c_p],
    "ddf_loss_seeds": [c_p, c_p, c_p, c_i64, c_p, c_p, c_p, c_p, c_sz, c_p],
    "ddf_adam_step": [c_p, c_p, c_p, c_p, c_i64, c_i64, c_f, c_f, c_f, c_f, c_p],
    "ddf_render_workspace_size": [ctypes.POINTER(DdfScene), ctypes.POINTER(DdfRenderParams), ctypes.POINTER(c_sz)],
    "ddf_render_wavefront": [ctypes.POINTER(DdfScene), ctypes.POINTER(DdfRenderParams), c_p, c_p, c_p, c_p, c_p, c_sz,
                             c_p],
    "ddf_train_step": [ctypes.POINTER(DdfNet), c_p, c_p, c_p, c_i64, c_f, c_p, c_p, c_i64, c_p, c_p, c_p, c_sz, c_p],
    "ddf_train_step_chunked": [ctypes.POINTER(DdfNet), c_p, c_p, c_p, c_i64, c_f, c_p, c_p, c_i64, c_i64, c_p, c_p,
                               c_p, c_sz, c_p],
    "ddf_set_tuning": [c_i32, c_i32],
    "ddf_get_tuning": [c_i32, ctypes.POINTER(c_i32)],
    "ddf_loss_seeds_ex": [c_p, c_p, c_p, c_i64, ctypes.POINTER(DdfLoss), c_p, c_p, c_p, c_p, c_sz, c_p],
    "ddf_train_step_ex": [ctypes.POINTER(DdfNet), c_p, c_p, c_p, c_i64, c_f, c_p, c_p, c_i64, c_i64,
                          ctypes.POINTER(DdfLoss), c_p, c_p, c_p, c_sz, c_p],
    "ddf_eikonal_workspace_size": [c_i32, c_i32, c_i64, ctypes.POINTER(c_sz)],
    "ddf_train_step_eikonal": [ctypes.POINTER(DdfNet), c_p, c_p, c_p, c_i64, c_f, c_p, c_p, c_p, c_i64, c_f, c_f,
                               ctypes.POINTER(DdfLoss), c_p, c_p, c_p, c_sz, c_p],
    "ddf_udf_workspace_size": [c_i64, c_i64, ctypes.POINTER(c_sz)],
    "ddf_udf": [ctypes.POINTER(DdfNet), c_p, c_i64, c_p, c_i64, c_p, c_p, c_p, c_sz, c_p],
    "ddf_udf_noalloc": [ctypes.POINTER(DdfNet), c_p, c_i64, c_p, c_i64, c_p, c_p, c_p],
    "ddf_dataset_workspace_size": [ctypes.POINTER(DdfDatasetParams), ctypes.POINTER(c_sz)],
    "ddf_sample_dataset": [c_p, c_i64, ctypes.POINTER(DdfDatasetParams), c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p,
                           c_sz, c_p],
    "ddf_paper_param_count": [c_i32, ctypes.POINTER(c_i64)],
    "ddf_paper_packed_bytes": [c_i32, c_i32, ctypes.POINTER(c_sz)],
    "ddf_paper_pack": [c_p, c_i32, c_i32, c_p, c_p],
    "ddf_paper_forward": [ctypes.POINTER(DdfPaperNet), c_p, c_i64, c_p, c_p],
    "ddf_paper_workspace_size": [c_i32, c_i64, ctypes.POINTER(c_sz)],
    "ddf_paper_backward": [ctypes.POINTER(DdfPaperNet), c_p, c_p, c_i64, c_p, c_p, c_p, c_u32, c_p, c_sz, c_p],
    "ddf_paper_train_step": [ctypes.POINTER(DdfPaperNet), c_p, c_p, c_p, c_i64, c_f, c_p, c_p, c_i64,
                             ctypes.POINTER(DdfLoss), c_f, c_u64, c_p, c_p, c_p, c_sz, c_p],
}
# launch-shape knobs (DDF_TUNE_* in ddf.h)
TUNE_KNOBS = {"stream_wg_per_cu": 0, "cull_rays_per_block": 1, "grad_wg_per_cu": 2}
_RESTYPE = {"ddf_abi_version": c_i32, "ddf_last_error": ctypes.c_char_p}

_lib = None


class DdfError(RuntimeError):
    def __init__(self, func, status, msg):
        super().__init__("%s failed with status %d: %s" % (func, status, msg))
        self.status = status


def load():
    """Load libddf.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libddf.so is not built (%s); run __graft_entry__.build() or "
                           "python paper_2306_16142_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = _RESTYPE.get(name, STATUS)
    _lib = lib
    return lib


def call(name, *args):
    """Call an entry point and raise DdfError on a non-zero status."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st != DDF_OK:
        raise DdfError(name, st, lib.ddf_last_error().decode())
    return st


def exported_symbols():
    return list(SIGNATURES)
