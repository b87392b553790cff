"""Thin ctypes binding of libntc.so (C ABI in include/ntc.h).

Argument marshalling only: every step of decoding and training runs in the HIP
kernels of libntc.so.  PyTorch provides device memory and streams.  Importing this
module fails loudly if the library has not been built
(``python -m paper_2305_17105_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libntc.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_17105_amd.build`")
_lib = C.CDLL(LIB_PATH)

OK, E_INVALID, E_UNSUPPORTED, E_WORKSPACE, E_HIP = range(5)
F32, F16, FP8_E4M3 = 0, 1, 2
ACT_RELU, ACT_HARDGELU = 0, 1
FILTER_BILINEAR, FILTER_TRILINEAR, FILTER_STOCHASTIC = 1, 2, 3
PE_SINCOS, PE_TRIANGLE = 0, 1
MAX_LEVELS, MAX_MIPS = 8, 16

QUERY_DTYPE = np.dtype([("u", "<f4"), ("v", "<f4"), ("lod", "<i4")])
MIXED_QUERY_DTYPE = np.dtype([("u", "<f4"), ("v", "<f4"), ("lod", "<i4"), ("material", "<i4")])


class Material(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("channels", C.c_int32), ("num_mips", C.c_int32),
        ("c0", C.c_int32), ("c1", C.c_int32), ("b0", C.c_int32), ("b1", C.c_int32),
        ("grid_shift", C.c_int32), ("hidden", C.c_int32), ("activation", C.c_int32), ("posenc", C.c_int32),
        ("lod_input", C.c_int32),
        ("num_levels", C.c_int32), ("input_width", C.c_int32),
        ("mip_w", C.c_int32 * MAX_MIPS), ("mip_h", C.c_int32 * MAX_MIPS), ("level_of_mip", C.c_int32 * MAX_MIPS),
        ("g0_w", C.c_int32 * MAX_LEVELS), ("g0_h", C.c_int32 * MAX_LEVELS),
        ("g1_w", C.c_int32 * MAX_LEVELS), ("g1_h", C.c_int32 * MAX_LEVELS),
        ("g0_offset", C.c_int64 * MAX_LEVELS), ("g1_offset", C.c_int64 * MAX_LEVELS),
        ("g0_packed", C.c_int64 * MAX_LEVELS), ("g1_packed", C.c_int64 * MAX_LEVELS),
        ("mip_offset", C.c_int64 * MAX_MIPS),
        ("latent_count", C.c_int64), ("packed_bytes", C.c_int64), ("target_count", C.c_int64),
        ("mlp_params", C.c_int64),
    ]


class TrainStateC(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "latents", "latents_fwd", "lat_m", "lat_v", "lat_grad", "mlp", "mlp_m", "mlp_v", "mlp_packed",
        "loss", "loss_scale", "scale_state")]


class HParams(C.Structure):
    _fields_ = [
        ("lr_latent", C.c_float), ("lr_mlp", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
        ("eps", C.c_float), ("noise_seed", C.c_uint64), ("step", C.c_int32), ("precision", C.c_int32),
        ("noise", C.c_int32), ("freeze_latents", C.c_int32), ("scale_growth_interval", C.c_int32),
        ("step_dev", C.c_void_p), ("lr_dev", C.c_void_p),
    ]


class TrainTuning(C.Structure):
    _fields_ = [("chunk", C.c_int32), ("tile", C.c_int32), ("microseconds", C.c_double)]


_P = C.POINTER
_sig = {
    "ntc_status_string": (C.c_char_p, [C.c_int]),
    "ntc_last_error": (C.c_char_p, []),
    "ntc_material_init": (C.c_int, [_P(Material)]),
    "ntc_shape_supported": (C.c_int, [_P(Material), C.c_int]),
    "ntc_quantize_latents": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_void_p]),
    "ntc_dequantize_latents": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_void_p]),
    "ntc_mlp_packed_bytes": (C.c_size_t, [_P(Material), C.c_int]),
    "ntc_pack_mlp": (C.c_int, [_P(Material), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ntc_decode": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p,
                             C.c_int, C.c_void_p]),
    "ntc_train_packed_bytes": (C.c_size_t, [_P(Material), C.c_int]),
    "ntc_train_workspace_bytes": (C.c_size_t, [_P(Material), C.c_int64, C.c_int]),
    "ntc_train_prepare": (C.c_int, [_P(Material), _P(TrainStateC), _P(HParams), C.c_void_p]),
    "ntc_train_step": (C.c_int, [_P(Material), _P(TrainStateC), C.c_void_p, C.c_int64, C.c_void_p, _P(HParams),
                                 C.c_void_p, C.c_size_t, C.c_void_p]),
    "ntc_train_step_noalloc": (C.c_int, [_P(Material), _P(TrainStateC), C.c_void_p, C.c_int64, C.c_void_p,
                                         _P(HParams), C.c_void_p]),
    "ntc_train_gradients": (C.c_int, [_P(Material), _P(TrainStateC), C.c_void_p, C.c_int64, C.c_void_p,
                                      _P(HParams), C.c_void_p, C.c_size_t, C.c_void_p]),
    "ntc_train_update": (C.c_int, [_P(Material), _P(TrainStateC), C.c_int64, _P(HParams), C.c_void_p, C.c_size_t,
                                   C.c_void_p]),
    "ntc_pack_mlp_train": (C.c_int, [_P(Material), C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "ntc_forward": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                              C.c_void_p, C.c_void_p]),
    "ntc_backward_workspace_bytes": (C.c_size_t, [_P(Material), C.c_int64, C.c_int]),
    "ntc_backward": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                               C.c_void_p, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "ntc_decode_tile": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_int, C.c_int32, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_int32, C.c_void_p, C.c_int, C.c_void_p]),
    "ntc_train_autotune": (C.c_int, [_P(Material), _P(TrainStateC), C.c_void_p, C.c_int64, C.c_void_p, _P(HParams),
                                     C.c_void_p, C.c_size_t, C.c_void_p, _P(TrainTuning)]),
    "ntc_train_set_tuning": (C.c_int, [_P(Material), C.c_int, _P(TrainTuning)]),
    "ntc_train_get_tuning": (C.c_int, [_P(Material), C.c_int, _P(TrainTuning)]),
    "ntc_train_workspace_bytes_batched": (C.c_size_t, [_P(Material), C.c_int32, _P(C.c_int64), C.c_int]),
    "ntc_train_step_batched": (C.c_int, [_P(Material), C.c_int32, _P(TrainStateC), C.c_void_p, _P(C.c_int64),
                                         _P(C.c_void_p), _P(HParams), C.c_void_p, C.c_size_t, C.c_void_p]),
    "ntc_decode_batched": (C.c_int, [_P(Material), C.c_int32, _P(C.c_void_p), _P(C.c_void_p), C.c_int, C.c_void_p,
                                     _P(C.c_int64), C.c_void_p, C.c_int, C.c_void_p]),
    "ntc_crop_queries": (C.c_int, [_P(Material), C.c_uint64, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_void_p,
                                   C.c_void_p]),
    "ntc_decode_filtered": (C.c_int, [_P(Material), C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                                      C.c_int32, C.c_uint64, C.c_void_p, C.c_int, C.c_void_p]),
    "ntc_train_table_bytes": (C.c_size_t, [C.c_int32]),
    "ntc_train_table_init": (C.c_int, [_P(Material), C.c_int32, _P(TrainStateC), _P(C.c_int64), _P(C.c_void_p),
                                       C.c_int, C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t]),
    "ntc_train_step_grouped": (C.c_int, [_P(Material), C.c_int32, _P(TrainStateC), C.c_void_p, _P(C.c_int64),
                                         _P(C.c_void_p), _P(HParams), C.c_void_p, C.c_size_t, C.c_void_p,
                                         C.c_void_p]),
    "ntc_decode_table_bytes": (C.c_size_t, [C.c_int32]),
    "ntc_decode_mixed": (C.c_int, [_P(Material), C.c_int32, C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p,
                                   C.c_int, C.c_void_p]),
    "ntc_decode_table_init": (C.c_int, [_P(Material), C.c_int32, _P(C.c_void_p), _P(C.c_void_p), C.c_int,
                                        C.c_void_p, C.c_size_t]),
    "ntc_decode_grouped": (C.c_int, [_P(Material), C.c_int32, C.c_void_p, C.c_int, C.c_void_p, _P(C.c_int64),
                                     C.c_void_p, C.c_int, C.c_void_p]),
    "ntc_timing_begin": (C.c_int, [C.c_int32]),
    "ntc_timing_read": (C.c_int, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "ntc_timing_end": (C.c_int, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class NtcError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = _lib.ntc_last_error().decode()
        super().__init__(f"{where}: {_lib.ntc_status_string(status).decode()} ({msg})")


def _check(status, where):
    if status != OK:
        raise NtcError(status, where)


def exported_symbols():
    """Names of the C entry points this binding resolves from the library."""
    return sorted(_sig)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------ descriptor
def material_init(width, height, channels, c0, c1, b0, b1, hidden=64, num_mips=0, grid_shift=2,
                  activation=ACT_RELU, posenc=PE_SINCOS, lod_input=0) -> Material:
    m = Material()
    m.width, m.height, m.channels, m.num_mips = width, height, channels, num_mips
    m.c0, m.c1, m.b0, m.b1 = c0, c1, b0, b1
    m.grid_shift, m.hidden, m.activation, m.posenc = grid_shift, hidden, activation, posenc
    m.lod_input = lod_input
    _check(_lib.ntc_material_init(C.byref(m)), "ntc_material_init")
    return m


def shape_supported(m: Material, for_decode: bool) -> bool:
    return bool(_lib.ntc_shape_supported(C.byref(m), int(for_decode)))


def mlp_packed_bytes(m: Material, precision=F32) -> int:
    return int(_lib.ntc_mlp_packed_bytes(C.byref(m), precision))


def train_packed_bytes(m: Material, precision=F32) -> int:
    return int(_lib.ntc_train_packed_bytes(C.byref(m), precision))


def train_workspace_bytes(m: Material, n: int, precision=F32) -> int:
    return int(_lib.ntc_train_workspace_bytes(C.byref(m), n, precision))


# ------------------------------------------------------------------ entry points (device tensors)
def quantize_latents(m: Material, latents, packed, stream=None):
    _check(_lib.ntc_quantize_latents(C.byref(m), _ptr(latents), _ptr(packed), _stream(stream)), "ntc_quantize_latents")


def dequantize_latents(m: Material, packed, latents, stream=None):
    _check(_lib.ntc_dequantize_latents(C.byref(m), _ptr(packed), _ptr(latents), _stream(stream)),
           "ntc_dequantize_latents")


def pack_mlp(m: Material, mlp, precision, packed, stream=None):
    _check(_lib.ntc_pack_mlp(C.byref(m), _ptr(mlp), precision, _ptr(packed), _stream(stream)), "ntc_pack_mlp")


def decode(m: Material, packed_latents, mlp_packed, precision, queries, n, out, out_dtype, stream=None):
    _check(_lib.ntc_decode(C.byref(m), _ptr(packed_latents), _ptr(mlp_packed), precision, _ptr(queries), n,
                           _ptr(out), out_dtype, _stream(stream)), "ntc_decode")


def decode_tile(m: Material, packed_latents, mlp_packed, precision, lod, x0, y0, width, height, out, out_dtype,
                stream=None):
    _check(_lib.ntc_decode_tile(C.byref(m), _ptr(packed_latents), _ptr(mlp_packed), precision, lod, x0, y0, width,
                                height, _ptr(out), out_dtype, _stream(stream)), "ntc_decode_tile")


def train_prepare(m: Material, state: "TrainState", hp: HParams, stream=None):
    _check(_lib.ntc_train_prepare(C.byref(m), C.byref(state.c), C.byref(hp), _stream(stream)), "ntc_train_prepare")


def train_step(m: Material, state: "TrainState", queries, n, targets, hp: HParams, workspace, stream=None):
    _check(_lib.ntc_train_step(C.byref(m), C.byref(state.c), _ptr(queries), n, _ptr(targets), C.byref(hp),
                               _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)),
           "ntc_train_step")


NOALLOC_SCRATCH_BYTES = 128 << 20  # NTC_NOALLOC_SCRATCH_BYTES


def train_step_noalloc(m: Material, state: "TrainState", queries, n, targets, hp: HParams, stream=None):
    """ntc_train_step with the library's static scratch array as its workspace."""
    _check(_lib.ntc_train_step_noalloc(C.byref(m), C.byref(state.c), _ptr(queries), n, _ptr(targets), C.byref(hp),
                                       _stream(stream)), "ntc_train_step_noalloc")


def train_gradients(m: Material, state: "TrainState", queries, n, targets, hp: HParams, workspace, stream=None):
    _check(_lib.ntc_train_gradients(C.byref(m), C.byref(state.c), _ptr(queries), n, _ptr(targets), C.byref(hp),
                                    _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream)),
           "ntc_train_gradients")


def train_update(m: Material, state: "TrainState", n, hp: HParams, workspace, stream=None):
    _check(_lib.ntc_train_update(C.byref(m), C.byref(state.c), n, C.byref(hp), _ptr(workspace),
                                 workspace.numel() * workspace.element_size(), _stream(stream)), "ntc_train_update")


def pack_mlp_train(m: Material, mlp, precision, packed, stream=None):
    _check(_lib.ntc_pack_mlp_train(C.byref(m), _ptr(mlp), precision, _ptr(packed), _stream(stream)),
           "ntc_pack_mlp_train")


def forward(m: Material, latents, mlp, mlp_train_packed, precision, queries, n, out, stream=None):
    _check(_lib.ntc_forward(C.byref(m), _ptr(latents), _ptr(mlp), _ptr(mlp_train_packed), precision, _ptr(queries),
                            n, _ptr(out), _stream(stream)), "ntc_forward")


def backward_workspace_bytes(m: Material, n: int, precision=F32) -> int:
    return int(_lib.ntc_backward_workspace_bytes(C.byref(m), n, precision))


def backward(m: Material, latents, mlp, mlp_train_packed, precision, queries, n, dout, dout_scale, grad_latents,
             grad_mlp, workspace, stream=None):
    _check(_lib.ntc_backward(C.byref(m), _ptr(latents), _ptr(mlp), _ptr(mlp_train_packed), precision, _ptr(queries),
                             n, _ptr(dout), float(dout_scale), _ptr(grad_latents), _ptr(grad_mlp), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream)), "ntc_backward")


def hparams(lr_latent=0.01, lr_mlp=0.005, step=0, precision=F32, noise=True, freeze=False, seed=0,
            beta1=0.9, beta2=0.999, eps=1e-8, growth=2000, step_dev=None, lr_dev=None) -> HParams:
    """step_dev: int32 device tensor (1 element) holding the step index for graph
    replay; lr_dev: float32 device tensor (latent lr, MLP lr).  Both optional."""
    hp = HParams()
    hp.lr_latent, hp.lr_mlp, hp.beta1, hp.beta2, hp.eps = lr_latent, lr_mlp, beta1, beta2, eps
    hp.noise_seed, hp.step, hp.precision = seed, step, precision
    hp.noise, hp.freeze_latents, hp.scale_growth_interval = int(noise), int(freeze), growth
    hp.step_dev = _ptr(step_dev) if step_dev is not None else None
    hp.lr_dev = _ptr(lr_dev) if lr_dev is not None else None
    return hp


def crop_queries(m: Material, seed, step, out, crops=8, side=256, uniform_fraction=0.05, stream=None):
    """Fill `out` (uint8 device tensor of crops*side^2*12 bytes) with one training batch."""
    _check(_lib.ntc_crop_queries(C.byref(m), seed, step, crops, side, uniform_fraction, _ptr(out), _stream(stream)),
           "ntc_crop_queries")


def train_autotune(m: Material, state: "TrainState", queries, n, targets, hp: HParams, workspace, stream=None):
    """Pick the fastest (samples per work item, tile side) for this material's shape; returns
    (chunk, tile, microseconds per gradient pass)."""
    t = TrainTuning()
    _check(_lib.ntc_train_autotune(C.byref(m), C.byref(state.c), _ptr(queries), n, _ptr(targets), C.byref(hp),
                                   _ptr(workspace), workspace.numel() * workspace.element_size(), _stream(stream),
                                   C.byref(t)), "ntc_train_autotune")
    return t.chunk, t.tile, t.microseconds


def train_set_tuning(m: Material, precision, chunk, tile):
    """Set the tuning-table entry (samples per work item, tile side) of this material's shape."""
    t = TrainTuning(chunk, tile, 0.0)
    _check(_lib.ntc_train_set_tuning(C.byref(m), precision, C.byref(t)), "ntc_train_set_tuning")


def train_get_tuning(m: Material, precision):
    """(chunk, tile) a training plan of this material uses now."""
    t = TrainTuning()
    _check(_lib.ntc_train_get_tuning(C.byref(m), precision, C.byref(t)), "ntc_train_get_tuning")
    return t.chunk, t.tile


def _materials(mats):
    arr = (Material * len(mats))()
    for i, m in enumerate(mats):
        arr[i] = m
    return arr


def train_workspace_bytes_batched(mats, offsets, precision=F32) -> int:
    off = (C.c_int64 * len(offsets))(*[int(o) for o in offsets])
    return int(_lib.ntc_train_workspace_bytes_batched(_materials(mats), len(mats), off, precision))


def train_step_batched(mats, states, queries, offsets, targets, hp: HParams, workspace, stream=None):
    """One training step of every material; queries grouped per material by offsets
    (len(mats) + 1, host); targets: one device tensor per material."""
    n = len(mats)
    st = (TrainStateC * n)()
    for i, s in enumerate(states):
        st[i] = s.c
    off = (C.c_int64 * (n + 1))(*[int(o) for o in offsets])
    tg = (C.c_void_p * n)(*[_ptr(t) for t in targets])
    _check(_lib.ntc_train_step_batched(_materials(mats), n, st, _ptr(queries), off, tg, C.byref(hp), _ptr(workspace),
                                       workspace.numel() * workspace.element_size(), _stream(stream)),
           "ntc_train_step_batched")


class TrainTable:
    """A grouped training step's device table (ntc_train_table_init) with the host
    arrays the step passes again; the materials, states, targets and workspace stay
    referenced."""

    def __init__(self, mats, states, offsets, targets, precision, workspace, device="cuda"):
        import torch
        n = len(mats)
        self.nmat = n
        self.mats = _materials(mats)
        self.states = (TrainStateC * n)()
        for i, s in enumerate(states):
            self.states[i] = s.c
        self.offsets = (C.c_int64 * (n + 1))(*[int(o) for o in offsets])
        self.targets = (C.c_void_p * n)(*[_ptr(t) for t in targets])
        self.workspace = workspace
        self._keep = (list(states), list(targets))
        nbytes = int(_lib.ntc_train_table_bytes(n))
        self.table = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        _check(_lib.ntc_train_table_init(self.mats, n, self.states, self.offsets, self.targets, precision,
                                         _ptr(workspace), workspace.numel() * workspace.element_size(),
                                         _ptr(self.table), nbytes), "ntc_train_table_init")


def train_step_grouped(table: TrainTable, queries, hp: HParams, stream=None):
    """ntc_train_step_batched's step with one launch per stage for the whole group."""
    ws = table.workspace
    _check(_lib.ntc_train_step_grouped(table.mats, table.nmat, table.states, _ptr(queries), table.offsets,
                                       table.targets, C.byref(hp), _ptr(ws), ws.numel() * ws.element_size(),
                                       _ptr(table.table), _stream(stream)), "ntc_train_step_grouped")


def decode_batched(mats, packed, wpacks, precision, queries, offsets, out, out_dtype, stream=None):
    """Decode the query groups of every material into one output buffer: material i's
    n_i x C_i values follow those of materials < i."""
    n = len(mats)
    off = (C.c_int64 * (n + 1))(*[int(o) for o in offsets])
    pk = (C.c_void_p * n)(*[_ptr(p) for p in packed])
    wp = (C.c_void_p * n)(*[_ptr(w) for w in wpacks])
    _check(_lib.ntc_decode_batched(_materials(mats), n, pk, wp, precision, _ptr(queries), off, _ptr(out), out_dtype,
                                   _stream(stream)), "ntc_decode_batched")


def decode_filtered(m: Material, packed, wpack, precision, fqueries, n, filt, out, out_dtype, seed=0, stream=None):
    """Filtered decode of n filter queries (12-byte records u, v, lod as float32):
    bilinear, trilinear or stochastic (ntc_decode_filtered)."""
    _check(_lib.ntc_decode_filtered(C.byref(m), _ptr(packed), _ptr(wpack), precision, _ptr(fqueries), int(n),
                                    int(filt), int(seed) & (2 ** 64 - 1), _ptr(out), out_dtype, _stream(stream)),
           "ntc_decode_filtered")


class DecodeTable:
    """Device table of a grouped decode batch (ntc_decode_table_init): the materials,
    their packed latents and decode packs; the buffers are kept referenced."""

    def __init__(self, mats, packed, wpacks, precision, device="cuda"):
        import torch
        n = len(mats)
        self.mats = _materials(mats)
        self.nmat = n
        self.precision = precision
        self._keep = (list(packed), list(wpacks))
        nbytes = int(_lib.ntc_decode_table_bytes(n))
        self.table = torch.zeros(nbytes, dtype=torch.uint8, device=device)
        pk = (C.c_void_p * n)(*[_ptr(p) for p in packed])
        wp = (C.c_void_p * n)(*[_ptr(w) for w in wpacks])
        _check(_lib.ntc_decode_table_init(self.mats, n, pk, wp, precision, _ptr(self.table), nbytes),
               "ntc_decode_table_init")


def decode_mixed(table: DecodeTable, mqueries, n, out, out_dtype, stream=None):
    """Decode n queries that each name their material (16-byte records u, v, lod,
    material) in one launch (ntc_decode_mixed); out in query order."""
    _check(_lib.ntc_decode_mixed(table.mats, table.nmat, _ptr(table.table), table.precision, _ptr(mqueries), int(n),
                                 _ptr(out), out_dtype, _stream(stream)), "ntc_decode_mixed")


def decode_grouped(table: DecodeTable, queries, offsets, out, out_dtype, stream=None, precision=None):
    """ntc_decode_batched's result with one launch per kernel shape (see DecodeTable)."""
    n = table.nmat
    off = (C.c_int64 * (n + 1))(*[int(o) for o in offsets])
    prec = table.precision if precision is None else precision
    _check(_lib.ntc_decode_grouped(table.mats, n, _ptr(table.table), prec, _ptr(queries), off, _ptr(out),
                                   out_dtype, _stream(stream)), "ntc_decode_grouped")


class TrainState:
    """Device buffers of a training run, allocated through PyTorch."""

    def __init__(self, m: Material, latents, mlp, precision=F32, device="cuda", loss_scale=65536.0):
        import torch
        L, P = int(m.latent_count), int(m.mlp_params)
        f = dict(dtype=torch.float32, device=device)
        self.latents = torch.as_tensor(latents, **f).clone().contiguous()
        assert self.latents.numel() == L
        self.latents_fwd = torch.zeros(L, **f)
        self.lat_m = torch.zeros(L, **f)
        self.lat_v = torch.zeros(L, **f)
        self.lat_grad = torch.zeros(L, **f)
        self.mlp = torch.as_tensor(mlp, **f).clone().contiguous()
        assert self.mlp.numel() == P
        self.mlp_m = torch.zeros(P, **f)
        self.mlp_v = torch.zeros(P, **f)
        self.mlp_packed = torch.zeros(train_packed_bytes(m, precision), dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, **f)
        self.loss_scale = torch.full((2,), loss_scale, **f)
        self.scale_state = torch.zeros(2, dtype=torch.int32, device=device)
        self.c = TrainStateC(*[C.c_void_p(getattr(self, n).data_ptr()) for n, _ in TrainStateC._fields_])


def timing_begin(max_launches: int):
    """Record HIP events around the next max_launches launches of each timed kernel."""
    _check(_lib.ntc_timing_begin(max_launches), "ntc_timing_begin")


def timing_read(kernel: str):
    """(total ms, launches) recorded for kernel "train_fused" or "decode"."""
    ms, n = C.c_double(0.0), C.c_int32(0)
    _check(_lib.ntc_timing_read(kernel.encode(), C.byref(ms), C.byref(n)), "ntc_timing_read")
    return ms.value, n.value


def timing_end():
    _check(_lib.ntc_timing_end(), "ntc_timing_end")
