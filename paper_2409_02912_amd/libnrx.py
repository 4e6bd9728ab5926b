"""Thin ctypes binding of libnrx.so: same names as the C ABI, argument marshalling only.

Device buffers are torch tensors on the GPU (PyTorch supplies memory and the
stream); every computation happens in the HIP library.  Importing this module
fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnrx-gfx950.so")

NRX_OK, NRX_ERR_INVALID, NRX_ERR_SHAPE, NRX_ERR_UNSUPPORTED, NRX_ERR_WORKSPACE, NRX_ERR_HIP = range(6)
NRX_FP32, NRX_BF16, NRX_FP8 = 0, 1, 2
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "SHAPE", 3: "UNSUPPORTED", 4: "WORKSPACE", 5: "HIP"}


class NrxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libnrx {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ModelConfig(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("d", ctypes.c_int32), ("n_blocks", ctypes.c_int32),
                ("n_rounds", ctypes.c_int32), ("m_max", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SlotDesc(ctypes.Structure):
    _fields_ = [("n_prb", ctypes.c_int32), ("n_ant", ctypes.c_int32), ("n_ue", ctypes.c_int32),
                ("bits_per_sym", ctypes.c_int32 * 4), ("slot_number", ctypes.c_int32),
                ("n_id", ctypes.c_int32), ("n_scid", ctypes.c_int32), ("n0", ctypes.c_float),
                ("snr_offset_db", ctypes.c_float), ("dmrs_sym_mask", ctypes.c_uint32),
                ("y_offset", ctypes.c_int64), ("h_offset", ctypes.c_int64),
                ("llr_offset", ctypes.c_int64), ("bits_offset", ctypes.c_int64)]


class SimConfig(ctypes.Structure):
    _fields_ = [("n_taps", ctypes.c_int32), ("tap_spacing_ns", ctypes.c_int32), ("tap_decay_ns", ctypes.c_float),
                ("doppler_max_hz", ctypes.c_float), ("rho", ctypes.c_float), ("snr_db_lo", ctypes.c_float),
                ("snr_db_hi", ctypes.c_float), ("scs_khz", ctypes.c_int32)]


# torch must be loaded first: it ships its own HIP runtime (SONAME libamdhip64.so.7), and libnrx must bind
# to that same runtime so that device pointers and streams created by torch are valid in the library.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2409_02912_amd/build.py "
                      "(the receiver has no fallback path)")
_lib = ctypes.CDLL(LIB_PATH)

_vp, _sz, _i32, _i64, _u64, _u32, _f = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.c_uint64, ctypes.c_uint32, ctypes.c_float)
_DESC = ctypes.POINTER(SlotDesc)

_SIGS = {
    "nrx_model_create": (_i32, [ctypes.POINTER(ModelConfig), ctypes.POINTER(_vp)]),
    "nrx_model_destroy": (_i32, [_vp]),
    "nrx_weight_count": (_i64, [_vp]),
    "nrx_weight_tensor": (_i32, [_vp, _i32, ctypes.c_char_p, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_i32),
                                 ctypes.POINTER(_i32)]),
    "nrx_workspace_bytes": (_sz, [_vp, _DESC, _i32, _i32]),
    "nrx_forward": (_i32, [_vp, _vp, _DESC, _i32, _vp, _vp, _vp, _i32, _vp, _sz, _vp]),
    "nrx_backward": (_i32, [_vp, _vp, _DESC, _i32, _vp, _vp, _vp, _sz, _vp]),
    "nrx_num_iterations": (_i32, [_vp]),
    "nrx_set_iterations": (_i32, [_vp, _i32]),
    "nrx_forward_iters": (_i32, [_vp, _vp, _DESC, _i32, _vp, _vp, _vp, _i64, _i32, _vp, _sz, _vp]),
    "nrx_backward_iters": (_i32, [_vp, _vp, _DESC, _i32, _vp, _i64, _vp, _vp, _sz, _vp]),
    "nrx_forward_chest": (_i32, [_vp, _vp, _DESC, _i32, _vp, _vp, _vp, _i64, _vp, _i64, _i32, _vp, _sz, _vp]),
    "nrx_backward_chest": (_i32, [_vp, _vp, _DESC, _i32, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp]),
    "nrx_mse_workspace_bytes": (_sz, [_DESC, _i32]),
    "nrx_mse": (_i32, [_DESC, _i32, _vp, _vp, ctypes.c_float, _vp, _vp, _vp, _sz, _vp]),
    "nrx_bce_workspace_bytes": (_sz, [_DESC, _i32, _i32]),
    "nrx_bce": (_i32, [_DESC, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nrx_adam": (_i32, [_vp, _vp, _vp, _vp, _i64, _i64, _f, _f, _f, _f, _vp]),
    "nrx_ls_estimate": (_i32, [_DESC, _i32, _vp, _vp, _vp, _sz, _vp]),
    "lmmse_workspace_bytes": (_sz, [_DESC, _i32]),
    "lmmse_demap": (_i32, [_DESC, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "lmmse_noalloc_scratch_bytes": (_sz, [_DESC, _i32, _i32]),
    "lmmse_demap_noalloc": (_i32, [_DESC, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "slot_sim_workspace_bytes": (_sz, [ctypes.POINTER(SimConfig), _DESC, _i32]),
    "slot_sim": (_i32, [ctypes.POINTER(SimConfig), _u64, _u32, _DESC, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp,
                        _sz, _vp]),
    "nrx_profile_enable": (_i32, [_vp, _i32]),
    "nrx_profile_read": (_i32, [_vp, _i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64), _i32]),
    "nrx_autotune": (_i32, [_vp, _vp, _DESC, _i32, _vp, _vp, _vp, _sz, ctypes.c_char_p, _vp]),
    "nrx_conv_variant": (_i32, [_vp, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "nrx_fp8_layers": (_i32, [_vp, _i32, ctypes.POINTER(_i32)]),
    "nrx_slot_latency": (_i32, [_vp, _DESC, _i32, _vp, _vp, _vp]),
    "nrx_act_scale_count": (_i32, [_vp]),
    "nrx_act_scales": (_i32, [_vp, _vp, _vp, _i32]),
    "nrx_calibrate": (_i32, [_vp, _vp, _DESC, _i32, _vp, _vp, _vp, ctypes.c_size_t, ctypes.c_float, _vp]),
    "nrx_slot_flags": (_i32, [_vp, _DESC, _i32, _vp, _sz, _vp, _vp]),
    "nrx_fallback_lmmse": (_i32, [_DESC, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "nrx_persist_schedule": (_i64, [_vp, _DESC, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _i32]),
    "nrx_saved_token": (_i64, [_vp]),
    "nrx_check_token": (_i32, [_vp, _vp, _i64]),
    "nrx_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(status):
    if status != NRX_OK:
        raise NrxError(status, _lib.nrx_last_error().decode())


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _descs(slots):
    arr = (SlotDesc * len(slots))(*slots)
    return arr, len(slots)


# ------------------------------------------------------------ descriptors ---

def make_slots(shapes, m_max, model_b=None):
    """Builds packed descriptors. shapes: list of dicts with n_prb, n_ant, n_ue, bits (list), optional
    slot_number, n_id, n_scid, n0, snr_offset_db.  Returns (descs, sizes) with the element counts of y, h, llr, bits."""
    out = []
    yo = ho = lo = bo = 0
    for i, sh in enumerate(shapes):
        S = 12 * sh["n_prb"]
        B, U = sh["n_ant"], sh["n_ue"]
        d = SlotDesc()
        d.n_prb, d.n_ant, d.n_ue = sh["n_prb"], B, U
        bits = list(sh["bits"]) + [0] * (4 - len(sh["bits"]))
        for u in range(4):
            d.bits_per_sym[u] = bits[u]
        d.slot_number = sh.get("slot_number", i % 20)
        d.n_id = sh.get("n_id", 0)
        d.n_scid = sh.get("n_scid", 0)
        d.n0 = sh.get("n0", 0.0)
        d.snr_offset_db = sh.get("snr_offset_db", 0.0)
        d.dmrs_sym_mask = sh.get("dmrs_sym_mask", 0)
        d.y_offset, d.h_offset, d.llr_offset, d.bits_offset = yo, ho, lo, bo
        yo += S * 14 * B
        ho += S * 14 * U * B
        lo += U * 14 * S * m_max
        bo += U * 12 * S * m_max
        out.append(d)
    return out, dict(y=yo, h=ho, llr=lo, bits=bo)


# ------------------------------------------------------------------ model ---

def nrx_model_create(n_ant, d, n_blocks, n_rounds, m_max, precision=NRX_FP32, flags=0):
    cfg = ModelConfig(n_ant, d, n_blocks, n_rounds, m_max, precision, flags, 0)
    h = _vp()
    _check(_lib.nrx_model_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def nrx_model_destroy(model):
    _check(_lib.nrx_model_destroy(model))


def nrx_weight_count(model):
    return int(_lib.nrx_weight_count(model))


def nrx_weight_tensor(model, idx):
    name = ctypes.create_string_buffer(64)
    off, nd = _i64(), _i32()
    shape = (_i32 * 4)()
    _check(_lib.nrx_weight_tensor(model, idx, name, 64, ctypes.byref(off), ctypes.byref(nd), shape))
    return name.value.decode(), int(off.value), tuple(shape[i] for i in range(nd.value))


def weight_layout(model):
    out, i = [], 0
    while True:
        name = ctypes.create_string_buffer(64)
        off, nd = _i64(), _i32()
        shape = (_i32 * 4)()
        if _lib.nrx_weight_tensor(model, i, name, 64, ctypes.byref(off), ctypes.byref(nd), shape) != NRX_OK:
            return out
        out.append((name.value.decode(), int(off.value), tuple(shape[k] for k in range(nd.value))))
        i += 1


def nrx_workspace_bytes(model, slots, save_acts=False):
    arr, n = _descs(slots)
    return int(_lib.nrx_workspace_bytes(model, arr, n, int(save_acts)))


def nrx_forward(model, w, slots, y, llr, ws, h_ls=None, save_acts=False, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_forward(model, _ptr(w), arr, n, _ptr(y), _ptr(h_ls), _ptr(llr), int(save_acts), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream(stream)))


def nrx_backward(model, w, slots, dllr, dw, ws, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_backward(model, _ptr(w), arr, n, _ptr(dllr), _ptr(dw), _ptr(ws),
                             ws.numel() * ws.element_size(), _stream(stream)))


def nrx_num_iterations(model):
    return int(_lib.nrx_num_iterations(model))


def nrx_set_iterations(model, n_iter):
    _check(_lib.nrx_set_iterations(model, int(n_iter)))


def nrx_forward_iters(model, w, slots, y, llr, llr_stride, ws, h_ls=None, save_acts=False, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_forward_iters(model, _ptr(w), arr, n, _ptr(y), _ptr(h_ls), _ptr(llr), int(llr_stride),
                                  int(save_acts), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def nrx_backward_iters(model, w, slots, dllr, llr_stride, dw, ws, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_backward_iters(model, _ptr(w), arr, n, _ptr(dllr), int(llr_stride), _ptr(dw), _ptr(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)))


def nrx_forward_chest(model, w, slots, y, llr, h_est, ws, llr_stride=0, h_stride=0, h_ls=None, save_acts=False,
                      stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_forward_chest(model, _ptr(w), arr, n, _ptr(y), _ptr(h_ls), _ptr(llr), int(llr_stride),
                                  _ptr(h_est), int(h_stride), int(save_acts), _ptr(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)))


def nrx_backward_chest(model, w, slots, dllr, dh_est, dw, ws, llr_stride=0, h_stride=0, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_backward_chest(model, _ptr(w), arr, n, _ptr(dllr), int(llr_stride), _ptr(dh_est),
                                   int(h_stride), _ptr(dw), _ptr(ws), ws.numel() * ws.element_size(),
                                   _stream(stream)))


def nrx_mse_workspace_bytes(slots):
    arr, n = _descs(slots)
    return int(_lib.nrx_mse_workspace_bytes(arr, n))


def nrx_mse(slots, h_est, h_true, gamma, dh_est, loss, ws, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_mse(arr, n, _ptr(h_est), _ptr(h_true), float(gamma), _ptr(dh_est), _ptr(loss), _ptr(ws),
                        ws.numel() * ws.element_size(), _stream(stream)))


def nrx_bce_workspace_bytes(slots, m_max):
    arr, n = _descs(slots)
    return int(_lib.nrx_bce_workspace_bytes(arr, n, m_max))


def nrx_bce(slots, m_max, llr, bits, dllr, loss, nerr, ws, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_bce(arr, n, m_max, _ptr(llr), _ptr(bits), _ptr(dllr), _ptr(loss), _ptr(nerr), _ptr(ws),
                        ws.numel() * ws.element_size(), _stream(stream)))


def nrx_adam(w, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(_lib.nrx_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), w.numel(), step, lr, beta1, beta2, eps,
                         _stream(stream)))


# -------------------------------------------------------- classical judge ---

def lmmse_workspace_bytes(slots):
    arr, n = _descs(slots)
    return int(_lib.lmmse_workspace_bytes(arr, n))


def nrx_ls_estimate(slots, y, h, ws, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_ls_estimate(arr, n, _ptr(y), _ptr(h), _ptr(ws), ws.numel() * ws.element_size(),
                                _stream(stream)))


def lmmse_demap(slots, m_max, y, llr, ws, h=None, n0=None, stream=None):
    arr, n = _descs(slots)
    _check(_lib.lmmse_demap(arr, n, m_max, _ptr(y), _ptr(h), _ptr(n0), _ptr(llr), _ptr(ws),
                            ws.numel() * ws.element_size(), _stream(stream)))


NRX_NOALLOC_SCRATCH_BYTES = 64 << 20


def lmmse_noalloc_scratch_bytes(slots, internal_ls=True):
    arr, n = _descs(slots)
    return int(_lib.lmmse_noalloc_scratch_bytes(arr, n, 1 if internal_ls else 0))


def lmmse_demap_noalloc(slots, m_max, y, llr, h=None, n0=None, stream=None):
    arr, n = _descs(slots)
    _check(_lib.lmmse_demap_noalloc(arr, n, m_max, _ptr(y), _ptr(h), _ptr(n0), _ptr(llr), _stream(stream)))


def nrx_slot_flags(model, slots, ws, flags, stream=None):
    """flags: int32/uint32 device tensor of one word per slot (bit 0: an LLR is not finite, bit 1: a channel
    estimate is not finite) for the last forward on ws."""
    arr, n = _descs(slots)
    _check(_lib.nrx_slot_flags(model, arr, n, _ptr(ws), ws.numel() * ws.element_size(), _ptr(flags),
                               _stream(stream)))


def nrx_fallback_lmmse(slots, m_max, y, flags, llr, ws, h=None, n0=None, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_fallback_lmmse(arr, n, m_max, _ptr(y), _ptr(h), _ptr(n0), _ptr(flags), _ptr(llr), _ptr(ws),
                                   ws.numel() * ws.element_size(), _stream(stream)))


def nrx_persist_schedule(model, slots, cap=1 << 22):
    """Work order of the persistent forward: (stage, slot, first tile, tiles) arrays over the items, and the
    stage kinds."""
    arr, n = _descs(slots)
    st, sl, ti, nt = (np.zeros(cap, dtype=np.int32) for _ in range(4))
    kinds = np.zeros(64, dtype=np.int32)
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    k = int(_lib.nrx_persist_schedule(model, arr, n, c(st), c(sl), c(ti), c(nt), cap, c(kinds), 64))
    if k < 0:
        raise NrxError(NRX_ERR_INVALID, _lib.nrx_last_error().decode())
    ns = int(st[:k].max()) + 1 if k else 0
    return st[:k].copy(), sl[:k].copy(), ti[:k].copy(), nt[:k].copy(), kinds[:ns].copy()


def nrx_saved_token(model):
    return int(_lib.nrx_saved_token(model))


def nrx_check_token(model, ws, token):
    _check(_lib.nrx_check_token(model, _ptr(ws), int(token)))


# ------------------------------------------------------------- data model ---

def sim_config(n_taps=12, tap_spacing_ns=100, tap_decay_ns=487.42, doppler_max_hz=0.0, rho=0.0,
               snr_db_lo=10.0, snr_db_hi=10.0, scs_khz=30):
    return SimConfig(n_taps, tap_spacing_ns, tap_decay_ns, doppler_max_hz, rho, snr_db_lo, snr_db_hi, scs_khz)


def slot_sim_workspace_bytes(cfg, slots):
    arr, n = _descs(slots)
    return int(_lib.slot_sim_workspace_bytes(ctypes.byref(cfg), arr, n))


def slot_sim(cfg, seed, batch_index, slots, m_max, y, ws, h_true=None, bits=None, snr_db=None, n0=None,
             stream=None):
    arr, n = _descs(slots)
    _check(_lib.slot_sim(ctypes.byref(cfg), seed, batch_index, arr, n, m_max, _ptr(y), _ptr(h_true), _ptr(bits),
                         _ptr(snr_db), _ptr(n0), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def nrx_last_error():
    return _lib.nrx_last_error().decode()


# ------------------------------------------------------------ diagnostics ---

NRX_K_FRONTEND, NRX_K_CONV_IN, NRX_K_CONV_A, NRX_K_CONV_A_MP, NRX_K_CONV_B, NRX_K_MP, NRX_K_READOUT = range(7)
KERNEL_CLASSES = ("frontend", "conv_in", "conv_a", "conv_a_mp", "conv_b", "mp", "readout")


def nrx_profile_enable(model, enable=True):
    _check(_lib.nrx_profile_enable(model, int(enable)))


def nrx_profile_read(model, cls, reset=False):
    ms, n = ctypes.c_double(), _i64()
    _check(_lib.nrx_profile_read(model, cls, ctypes.byref(ms), ctypes.byref(n), int(reset)))
    return float(ms.value), int(n.value)


def nrx_autotune(model, w, slots, y, llr, ws, cache_path=None, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_autotune(model, _ptr(w), arr, n, _ptr(y), _ptr(llr), _ptr(ws), ws.numel() * ws.element_size(),
                             cache_path.encode() if cache_path else None, _stream(stream)))


def nrx_fp8_layers(model, mask=-1):
    """FP8 model: block convs in E4M3 (bit 0 conv_a, bit 1 conv_b); sets mask when >= 0, returns the current one."""
    cur = _i32()
    _check(_lib.nrx_fp8_layers(model, mask, ctypes.byref(cur)))
    return cur.value


def nrx_conv_variant(model, cls, variant=-1):
    cur, nv = _i32(), _i32()
    _check(_lib.nrx_conv_variant(model, cls, variant, ctypes.byref(cur), ctypes.byref(nv)))
    return int(cur.value), int(nv.value)


CONV_CLASSES = (NRX_K_CONV_IN, NRX_K_CONV_A, NRX_K_CONV_A_MP, NRX_K_CONV_B)


def set_all_conv_variants(model, variant):
    for c in CONV_CLASSES:
        nrx_conv_variant(model, c, variant)


def nrx_slot_latency(model, slots, ws, latency_us, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_slot_latency(model, arr, n, _ptr(ws), _ptr(latency_us), _stream(stream)))


def nrx_act_scales(model, scales=None):
    """Returns the FP8 activation scales (numpy float32); sets them first when given."""
    import numpy as np
    if scales is not None:
        src = np.ascontiguousarray(scales, dtype=np.float32).reshape(-1)
        _check(_lib.nrx_act_scales(model, src.ctypes.data, None, src.size))
    n = int(_lib.nrx_act_scale_count(model))
    out = np.zeros(n, dtype=np.float32)
    _check(_lib.nrx_act_scales(model, None, out.ctypes.data, n))
    return out


def nrx_calibrate(model, w, slots, y, llr, ws, headroom=1.25, stream=None):
    arr, n = _descs(slots)
    _check(_lib.nrx_calibrate(model, _ptr(w), arr, n, _ptr(y), _ptr(llr), _ptr(ws), ws.numel() * ws.element_size(),
                              float(headroom), _stream(stream)))
