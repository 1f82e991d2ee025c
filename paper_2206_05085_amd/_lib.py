"""ctypes loader for libdvgo.so (the gfx950 HIP library) and its C structs.

There is no fallback: if the library has not been built this raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdvgo.so")
ABI_VERSION = 6

VP = C.c_void_p
OK = 0
ERRORS = {-1: "ERR_NULL", -2: "ERR_SHAPE", -3: "ERR_RANGE", -4: "ERR_UNSORTED", -5: "ERR_WORKSPACE", -6: "ERR_HIP",
          -7: "ERR_UNSUPPORTED", -8: "ERR_ABI"}
COLOR_GRID, COLOR_SAMPLES, COLOR_NONE = 0, 1, 2
WARP_NONE, WARP_CONTRACT_INF, WARP_CONTRACT_L2 = 0, 1, 2
SAMPLE_BOX, SAMPLE_NDC = 0, 1
MLP_SPLIT_F16, MLP_F16 = 0, 1


class DvgoError(RuntimeError):
    def __init__(self, fn, code, detail):
        super().__init__(f"{fn} failed with {ERRORS.get(code, code)}: {detail}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("channels", C.c_int32), ("ch_stride", C.c_int32), ("xyz_min", C.c_float * 3),
                ("xyz_max", C.c_float * 3), ("data", VP), ("grad", VP), ("warp", C.c_int32), ("warp_b", C.c_float)]


class Samples(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_rays", C.c_int32), ("n_samples", C.c_int64),
                ("ray_offsets", VP), ("xyz", VP), ("delta", VP), ("s_mid", VP), ("s_len", VP)]


class RenderParams(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("act_shift", C.c_float), ("halt_T", C.c_float),
                ("bg", C.c_float * 3), ("color_mode", C.c_int32), ("want_dist", C.c_int32),
                ("ray_list", VP), ("n_list", C.c_int32), ("waves_per_block", C.c_int32), ("grid_waves", C.c_int32)]


class ColorMLP(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("in_feat", C.c_int32), ("n_freq", C.c_int32), ("hidden", C.c_int32),
                ("W1", VP), ("b1", VP), ("W2", VP), ("b2", VP), ("W3", VP), ("b3", VP),
                ("gW1", VP), ("gb1", VP), ("gW2", VP), ("gb2", VP), ("gW3", VP), ("gb3", VP),
                ("precision", C.c_int32), ("prepared", C.c_int32)]


class Rays(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_rays", C.c_int32), ("origins", VP), ("dirs", VP),
                ("t_near", VP), ("t_far", VP)]


class Proposal(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_bins", C.c_int32), ("hidden", C.c_int32), ("n_layers", C.c_int32),
                ("W", VP * 4), ("b", VP * 4), ("gW", VP * 4), ("gb", VP * 4)]


class Sampler(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("mode", C.c_int32), ("xyz_min", C.c_float * 3),
                ("xyz_max", C.c_float * 3), ("near", C.c_float), ("step", C.c_float), ("voxel", C.c_float),
                ("max_per_ray", C.c_int32), ("mask_shape", C.c_int32 * 3), ("mask", VP), ("ndc_fx", C.c_float),
                ("ndc_fy", C.c_float), ("ndc_planes", C.c_int32)]


_I32, _I64, _F, _SZP = C.c_int32, C.c_int64, C.c_float, C.POINTER(C.c_size_t)
_PR, _PQ, _PSM = C.POINTER(Rays), C.POINTER(Proposal), C.POINTER(Sampler)
_PG, _PS, _PP, _PM = C.POINTER(Grid), C.POINTER(Samples), C.POINTER(RenderParams), C.POINTER(ColorMLP)

SIGNATURES = {
    "dvgo_abi_version": (C.c_int, []),
    "dvgo_last_error": (C.c_char_p, []),
    "dvgo_act_shift": (C.c_int, [C.c_double, C.c_double, C.POINTER(C.c_double)]),
    "dvgo_set_debug": (C.c_int, [_I32]),
    "dvgo_validate_samples": (C.c_int, [_PS, VP]),
    "dvgo_render_state_size": (C.c_int, [_I32, _I64, _SZP]),
    "dvgo_render_forward": (C.c_int, [_PP, _PS, _PG, _PG, VP, VP, VP, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_render_backward": (C.c_int, [_PP, _PS, _PG, _PG, VP, VP, VP, C.c_size_t, VP, VP, VP, VP, VP, VP]),
    "dvgo_render_train": (C.c_int, [_PP, _PS, _PG, _PG, VP, VP, _F, VP, VP, VP, VP, C.c_size_t, VP, VP, VP]),
    "dvgo_ray_schedule": (C.c_int, [_I32, VP, VP, VP, VP]),
    "dvgo_render_autotune": (C.c_int, [_PP, _PS, _PG, _PG, VP, _I32, C.POINTER(_I32), C.POINTER(_I32),
                                       C.POINTER(C.c_float), VP]),
    "dvgo_distortion_workspace_size": (C.c_int, [_I32, _I64, _SZP]),
    "dvgo_distortion_loss": (C.c_int, [_I32, VP, _I64, VP, VP, VP, VP, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_distortion_loss_noalloc": (C.c_int, [_I32, VP, _I64, VP, VP, VP, VP, VP, VP, VP]),
    "dvgo_grid_adam_step": (C.c_int, [VP, VP, VP, VP, _I64, _F, _F, _F, _F, _I32, VP, _I32, _I32, VP]),
    "dvgo_counter_add": (C.c_int, [VP, _I32, VP]),
    "dvgo_grid_gather": (C.c_int, [_PG, _I64, VP, VP, VP]),
    "dvgo_grid_scatter": (C.c_int, [_PG, _I64, VP, VP, VP]),
    "dvgo_bin_workspace_size": (C.c_int, [_PG, _I64, _SZP]),
    "dvgo_grid_resample": (C.c_int, [_PG, _I32, _I32, _I32, VP, VP]),
    "dvgo_bin_samples": (C.c_int, [_PG, _I64, VP, VP, C.c_size_t, VP]),
    "dvgo_grid_scatter_binned": (C.c_int, [_PG, _I64, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_owner_workspace_size": (C.c_int, [_PG, _I64, _SZP]),
    "dvgo_owner_bin": (C.c_int, [_PG, _I64, VP, VP, C.c_size_t, VP]),
    "dvgo_grid_scatter_owned": (C.c_int, [_PG, _I64, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_grid_scatter_adam": (C.c_int, [_PG, _I64, VP, VP, VP, C.c_size_t, VP, VP, VP, _F, _F, _F, _F, _I32, VP,
                                         VP]),
    "dvgo_tv_add_grad": (C.c_int, [_PG, _F, _F, _I32, VP]),
    "dvgo_alpha": (C.c_int, [_PG, _I64, VP, VP, _F, VP, VP]),
    "dvgo_mlp_workspace_size": (C.c_int, [_PM, _I32, _I64, _SZP]),
    "dvgo_mlp_prepare": (C.c_int, [_PM, _I32, VP, VP, _I64, VP, C.c_size_t, VP]),
    "dvgo_mlp_forward": (C.c_int, [_PM, _I32, VP, VP, _I64, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_mlp_forward_gather": (C.c_int, [_PM, _I32, VP, VP, _I64, _PG, VP, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_mlp_backward": (C.c_int, [_PM, _I32, VP, VP, _I64, VP, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_mlp_backward_partials": (C.c_int, [_PM, _I32, VP, VP, _I64, VP, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_mlp_reduce_grads": (C.c_int, [_PM, _I32, _I64, VP, C.c_size_t, VP]),
    "dvgo_loss_head": (C.c_int, [_I32, VP, VP, VP, _F, VP, VP, VP, VP]),
    "dvgo_proposal_coarse": (C.c_int, [_PR, _PG, _F, _F, _F, VP, VP, VP]),
    "dvgo_proposal_forward": (C.c_int, [_PQ, _I32, VP, VP, VP, VP, VP]),
    "dvgo_proposal_workspace_size": (C.c_int, [_PQ, _I32, _SZP]),
    "dvgo_proposal_backward": (C.c_int, [_PQ, _I32, VP, VP, VP, VP, C.c_size_t, VP]),
    "dvgo_histogram": (C.c_int, [_I32, VP, VP, VP, _I32, _F, VP, VP]),
    "dvgo_resample_offsets": (C.c_int, [_PR, VP, _F, _I32, _I32, VP, VP]),
    "dvgo_resample": (C.c_int, [_PR, VP, VP, _F, VP, _I32, _I32, _F, VP, VP, VP, VP, VP]),
    "dvgo_resample_guarded_offsets": (C.c_int, [_PR, VP, VP, VP, _F, _I32, _I32, _F, VP, VP, VP]),
    "dvgo_resample_guarded": (C.c_int, [_PR, VP, VP, _F, VP, VP, VP, VP, VP]),
    "dvgo_sample_count": (C.c_int, [_PSM, _I32, VP, VP, VP, VP, VP, VP]),
    "dvgo_sample_emit": (C.c_int, [_PSM, _I32, VP, VP, VP, _I64, VP, VP, VP, VP, VP]),
    "dvgo_occupancy_update": (C.c_int, [_PG, _F, _F, _F, VP, VP]),
}

_lib = None


def lib():
    """Load libdvgo.so; raise if it is missing (there is no CPU or PyTorch fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2206_05085_amd.build` "
                               "(or __graft_entry__.build()) first")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        v = L.dvgo_abi_version()
        if v != ABI_VERSION:
            raise RuntimeError(f"libdvgo ABI version {v} != binding version {ABI_VERSION}")
        _lib = L
    return _lib


def call(name, *args):
    rc = getattr(lib(), name)(*args)
    if rc != OK:
        detail = lib().dvgo_last_error().decode(errors="replace")
        raise DvgoError(name, rc, detail)
    return rc
