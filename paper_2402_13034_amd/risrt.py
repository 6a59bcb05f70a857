"""Python binding of librisrt (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  Device buffers
and streams come from PyTorch (ROCm).

The library must have been built (``python -m paper_2402_13034_amd.build``);
there is no fallback: loading fails loudly without it.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librisrt.so")

RT_OK = 0
RT_EINVAL = -1
RT_ENOMEM = -2
RT_EDEVICE = -3
RT_EBUSY = -4
RT_ENOTFOUND = -5
RT_EUNSUPPORTED = -6

PAT_ISO = 0
PAT_COSPOW = 1
PAT_MONOPOLE = 2

FLAG_KEEP_HITS = 1
FLAG_KEEP_PATHS = 2
FLAG_BRUTE_FORCE = 4
FLAG_EXHAUSTIVE = 8
FLAG_COUNT_WORK = 16
FLAG_RIS_INCOMING = 32
FLAG_FRESNEL_TE = 64
FLAG_FRESNEL_TM = 128
FLAG_KEEP_CIR = 256
FLAG_STAGE_TIMES = 512

MAX_ORDER = 5   # largest reflection order rt_trace accepts (RT_MAX_ORDER)

PREC_VALU_F32 = 0
PREC_MFMA_BF16X2 = 1
PREC_MFMA_BF16X3 = 2
PREC_MFMA_F16X2 = 3

# every entry point declared in include/risrt.h
ENTRY_POINTS = (
    "rt_last_error", "rt_init", "rt_shutdown", "rt_mem_info", "rt_scene_create", "rt_ris_create",
    "rt_trace", "rt_channel_create", "rt_channel_info", "rt_channel_read", "rt_hits_read",
    "rt_paths_read", "rt_candidates_read", "rt_ris_sum", "rt_destroy", "rt_scene_set_materials", "rt_cir",
    "rt_ris_paths_read", "rt_ris_sum_noalloc", "rt_keys_sort", "rt_scene_info",
)


class RtTx(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_double * 3), ("axis", ctypes.c_double * 3), ("power_w", ctypes.c_double),
                ("gain", ctypes.c_double), ("pattern", ctypes.c_int32), ("param", ctypes.c_double)]


class RtRx(ctypes.Structure):
    _fields_ = [("axis", ctypes.c_double * 3), ("gain", ctypes.c_double), ("pattern", ctypes.c_int32),
                ("param", ctypes.c_double)]


class RtParams(ctypes.Structure):
    _fields_ = [("freq_hz", ctypes.c_double), ("max_order", ctypes.c_int32), ("n_rays", ctypes.c_int64),
                ("flags", ctypes.c_uint32)]


class RtStats(ctypes.Structure):
    _fields_ = [("segments", ctypes.c_int64), ("discovery_segments", ctypes.c_int64),
                ("leg_segments", ctypes.c_int64), ("n_cand_tx", ctypes.c_int64), ("n_cand_u", ctypes.c_int64),
                ("n_env_paths", ctypes.c_int64), ("n_u_paths", ctypes.c_int64), ("n_ris_slots", ctypes.c_int64),
                ("ms_stage", ctypes.c_float * 8), ("ris_work", ctypes.c_int64 * 5),
                ("leg_walk_fallbacks", ctypes.c_int64), ("n_in_seq", ctypes.c_int64),
                ("n_in_paths", ctypes.c_int64), ("discovery_work", ctypes.c_int64 * 6),
                ("ms_discovery", ctypes.c_float * 3)]

    def as_dict(self):
        arrays = ("ms_stage", "ris_work", "discovery_work", "ms_discovery")
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in arrays}
        for f in arrays:
            d[f] = list(getattr(self, f))
        return d


class RtEnvPath(ctypes.Structure):
    _fields_ = [("rx", ctypes.c_int32), ("order", ctypes.c_int32), ("seq", ctypes.c_int32 * MAX_ORDER),
                ("tri", ctypes.c_int32 * MAX_ORDER), ("length", ctypes.c_double), ("amp", ctypes.c_float * 2)]


ENV_DTYPE = np.dtype([("rx", "<i4"), ("order", "<i4"), ("seq", "<i4", MAX_ORDER), ("tri", "<i4", MAX_ORDER),
                      ("length", "<f8"), ("amp", "<f4", 2)])
assert ENV_DTYPE.itemsize == ctypes.sizeof(RtEnvPath)


class RtError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("risrt error %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librisrt.so is not built: run python -m paper_2402_13034_amd.build")
        # torch (which supplies device memory and streams) is imported before the
        # library starts the HIP runtime: imported afterwards, it finds no device
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        u64 = ctypes.c_uint64
        pu64 = ctypes.POINTER(ctypes.c_uint64)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "rt_last_error": (ctypes.c_char_p, []),
            "rt_init": (ctypes.c_int32, [ctypes.c_int, u64, ctypes.POINTER(P)]),
            "rt_shutdown": (ctypes.c_int32, [P]),
            "rt_mem_info": (ctypes.c_int32, [P, pu64, pu64]),
            "rt_scene_create": (ctypes.c_int32, [P, P, i64, P, i64, P, P, P, P, pu64]),
            "rt_ris_create": (ctypes.c_int32, [P, P, i64, P, P, ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_double, pu64]),
            "rt_trace": (ctypes.c_int32, [P, u64, u64, ctypes.POINTER(RtTx), P, i64, ctypes.POINTER(RtRx),
                                          ctypes.POINTER(RtParams), P, pu64, ctypes.POINTER(RtStats)]),
            "rt_channel_create": (ctypes.c_int32, [P, i64, i64, P, P, P, pu64]),
            "rt_channel_info": (ctypes.c_int32, [P, u64, pi64, pi64, pi64, pi64]),
            "rt_channel_read": (ctypes.c_int32, [P, u64, P, P, P]),
            "rt_hits_read": (ctypes.c_int32, [P, u64, ctypes.c_int32, P, i64, pi64]),
            "rt_paths_read": (ctypes.c_int32, [P, u64, P, i64, pi64, P, i64, pi64, P, i64, pi64]),
            "rt_candidates_read": (ctypes.c_int32, [P, u64, ctypes.c_int32, P, i64, pi64]),
            "rt_ris_paths_read": (ctypes.c_int32, [P, u64, P, P, i64, pi64]),
            "rt_ris_sum": (ctypes.c_int32, [P, u64, P, i64, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                            P, P, P]),
            "rt_ris_sum_noalloc": (ctypes.c_int32, [P, u64, P, i64, ctypes.c_float, ctypes.c_int32,
                                                    ctypes.c_int32, P, P, P]),
            "rt_keys_sort": (ctypes.c_int32, [P, P, i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, pi64, P]),
            "rt_scene_info": (ctypes.c_int32, [P, u64, pi64, pi64, ctypes.POINTER(ctypes.c_int32), pu64]),
            "rt_destroy": (ctypes.c_int32, [P, u64]),
            "rt_scene_set_materials": (ctypes.c_int32, [P, u64, P, P, P]),
            "rt_cir": (ctypes.c_int32, [P, u64, P, ctypes.c_double, i64, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != RT_OK:
        raise RtError(status, lib().rt_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _torch_stream(stream):
    """The torch stream a call's work goes to (raw hipStream_t handles are
    wrapped), so that outputs are allocated and temporaries kept in its order."""
    import torch
    if stream is None:
        return torch.cuda.current_stream()
    if isinstance(stream, int):
        return torch.cuda.ExternalStream(stream)
    return stream


class _OnStream:
    """Enqueue a library call on `stream` from torch's current stream: the
    stream first waits for the current one (inputs written there are ready),
    tensors allocated inside are ordered on `stream`, and tensors read by the
    call are kept alive for it (record_stream) when the two streams differ."""

    def __init__(self, stream):
        import torch
        self.s = _torch_stream(stream)
        self.cur = torch.cuda.current_stream()
        self.other = self.s.cuda_stream != self.cur.cuda_stream
        self._ctx = torch.cuda.stream(self.s)

    def __enter__(self):
        if self.other:
            self.s.wait_stream(self.cur)
        self._ctx.__enter__()
        return self

    def __exit__(self, *a):
        return self._ctx.__exit__(*a)

    def keep(self, *tensors):
        if self.other:
            for t in tensors:
                if t is not None:
                    t.record_stream(self.s)

    @property
    def handle(self):
        return ctypes.c_void_p(self.s.cuda_stream)


def _v3(x):
    return (ctypes.c_double * 3)(*[float(v) for v in x])


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0, mem_budget_bytes: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().rt_init(device, mem_budget_bytes, ctypes.byref(self._h)))
        self.device = device

    def close(self):
        if self._h:
            _check(lib().rt_shutdown(self._h))
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def mem_info(self):
        u, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().rt_mem_info(self._h, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    # ---- objects ----
    def scene_create(self, V, T, surf, refl_re, refl_im, stream=None) -> int:
        """Arrays may be NumPy (host) or torch device tensors."""
        keep = []

        def arg(x, dt):
            if hasattr(x, "data_ptr"):
                keep.append(x)
                return ctypes.c_void_p(x.data_ptr())
            a = np.ascontiguousarray(x, dt)
            keep.append(a)
            return _ptr(a)

        h = ctypes.c_uint64()
        _check(lib().rt_scene_create(self._h, arg(V, np.float32), int(V.shape[0]), arg(T, np.int32),
                                     int(T.shape[0]), arg(surf, np.int32), arg(refl_re, np.float32),
                                     arg(refl_im, np.float32), _stream_handle(stream), ctypes.byref(h)))
        return h.value

    def scene_info(self, scene: int) -> dict:
        nt, ns, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
        d = ctypes.c_int32()
        _check(lib().rt_scene_info(self._h, ctypes.c_uint64(scene), ctypes.byref(nt), ctypes.byref(ns),
                                   ctypes.byref(d), ctypes.byref(b)))
        return {"n_tri": nt.value, "n_surf": ns.value, "bvh_depth": d.value, "bytes": b.value}

    def scene_set_materials(self, scene: int, eps_r, sigma, stream=None) -> None:
        """Per-triangle relative permittivity and conductivity (S/m) for the
        Fresnel flags; NumPy (host) or torch device arrays."""
        keep = []

        def arg(x):
            if hasattr(x, "data_ptr"):
                keep.append(x)
                return ctypes.c_void_p(x.data_ptr())
            a = np.ascontiguousarray(x, np.float32)
            keep.append(a)
            return _ptr(a)

        _check(lib().rt_scene_set_materials(self._h, ctypes.c_uint64(scene), arg(eps_r), arg(sigma),
                                            _stream_handle(stream)))

    def ris_create(self, elems, centre, normal, dy, dz, gain, q) -> int:
        E = np.ascontiguousarray(elems, np.float64)
        c = np.ascontiguousarray(centre, np.float64)
        n = np.ascontiguousarray(normal, np.float64)
        h = ctypes.c_uint64()
        _check(lib().rt_ris_create(self._h, _ptr(E), E.shape[0], _ptr(c), _ptr(n), dy, dz, gain, q,
                                   ctypes.byref(h)))
        return h.value

    def channel_create(self, E_env, H, stream=None) -> int:
        E = np.ascontiguousarray(E_env, np.complex64)
        Hh = np.ascontiguousarray(H, np.complex64)
        h = ctypes.c_uint64()
        _check(lib().rt_channel_create(self._h, Hh.shape[0], Hh.shape[1], _ptr(E), _ptr(Hh),
                                       _stream_handle(stream), ctypes.byref(h)))
        return h.value

    def destroy(self, handle: int):
        _check(lib().rt_destroy(self._h, handle))

    # ---- tracing ----
    def trace(self, scene: int, ris: int, tx_pos, tx_axis, tx_power_w, tx_gain, tx_pattern, tx_param, rx_pos,
              rx_axis, rx_gain, rx_pattern, rx_param, freq_hz, max_order, n_rays, flags=0, stream=None,
              stats=True):
        tx = RtTx(_v3(tx_pos), _v3(tx_axis), float(tx_power_w), float(tx_gain), int(tx_pattern), float(tx_param))
        rx = RtRx(_v3(rx_axis), float(rx_gain), int(rx_pattern), float(rx_param))
        prm = RtParams(float(freq_hz), int(max_order), int(n_rays), int(flags))
        if hasattr(rx_pos, "data_ptr"):
            rp = ctypes.c_void_p(rx_pos.data_ptr())
            R = int(rx_pos.shape[0])
            keep = rx_pos
        else:
            keep = np.ascontiguousarray(rx_pos, np.float64)
            rp = _ptr(keep)
            R = keep.shape[0]
        st = RtStats()
        ch = ctypes.c_uint64()
        _check(lib().rt_trace(self._h, scene, ris, ctypes.byref(tx), rp, R, ctypes.byref(rx), ctypes.byref(prm),
                              _stream_handle(stream), ctypes.byref(ch), ctypes.byref(st) if stats else None))
        del keep
        return ch.value, (st.as_dict() if stats else None)

    def channel_info(self, ch: int):
        R, M, ne, ns = (ctypes.c_int64() for _ in range(4))
        _check(lib().rt_channel_info(self._h, ch, ctypes.byref(R), ctypes.byref(M), ctypes.byref(ne),
                                     ctypes.byref(ns)))
        return R.value, M.value, ne.value, ns.value

    def channel_read(self, ch: int, stream=None):
        R, M, _, _ = self.channel_info(ch)
        E = np.zeros(R, np.complex64)
        H = np.zeros((R, M), np.complex64)
        _check(lib().rt_channel_read(self._h, ch, _ptr(E), _ptr(H) if H.size else None, _stream_handle(stream)))
        return E, H

    def hits_read(self, ch: int, source: int, K: int):
        rows = ctypes.c_int64()
        _check(lib().rt_hits_read(self._h, ch, source, None, 0, ctypes.byref(rows)))
        out = np.zeros((rows.value, K), np.int32)
        _check(lib().rt_hits_read(self._h, ch, source, _ptr(out), out.size, ctypes.byref(rows)))
        return out

    def candidates_read(self, ch: int, source: int):
        n = ctypes.c_int64()
        _check(lib().rt_candidates_read(self._h, ch, source, None, 0, ctypes.byref(n)))
        out = np.zeros((n.value, MAX_ORDER), np.int32)
        _check(lib().rt_candidates_read(self._h, ch, source, _ptr(out), out.size, ctypes.byref(n)))
        return out

    def paths_read(self, ch: int):
        R, M, _, _ = self.channel_info(ch)
        ne, nu, ns = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().rt_paths_read(self._h, ch, None, 0, ctypes.byref(ne), None, 0, ctypes.byref(nu), None, 0,
                                   ctypes.byref(ns)))
        env = np.zeros(ne.value, ENV_DTYPE)
        useq = np.zeros((nu.value, 1 + MAX_ORDER), np.int32)
        valid = np.zeros((ns.value, M), np.uint8)
        _check(lib().rt_paths_read(self._h, ch, _ptr(env) if env.size else None, ne.value, ctypes.byref(ne),
                                   _ptr(useq) if useq.size else None, nu.value, ctypes.byref(nu),
                                   _ptr(valid) if valid.size else None, ns.value, ctypes.byref(ns)))
        return {"env": env, "useq": useq, "ris_valid": valid.astype(bool)}

    def keys_sort(self, keys, begin_bit: int = 0, end_bit: Optional[int] = None, unique: bool = False,
                  stream=None) -> int:
        """Sort a torch int64 device tensor of keys in place: shape [n] (one
        word) or [n, 2] (word 0 least significant); returns the number of
        keys left (all of them unless unique)."""
        words = 1 if keys.dim() == 1 else int(keys.shape[1])
        if not keys.is_contiguous():
            raise ValueError("keys must be contiguous")
        n_out = ctypes.c_int64()
        _check(lib().rt_keys_sort(self._h, ctypes.c_void_p(keys.data_ptr()), int(keys.shape[0]), words,
                                  int(begin_bit), int(64 * words if end_bit is None else end_bit), int(unique),
                                  ctypes.byref(n_out), _stream_handle(stream)))
        return n_out.value

    def ris_paths_read(self, ch: int):
        """Per (slot, element) amplitude (complex64, 0 where no path) and
        unfolded length of the element paths, [n_slots, M] each (the channel
        needs FLAG_KEEP_PATHS or FLAG_KEEP_CIR)."""
        R, M, _, ns = self.channel_info(ch)
        n = ctypes.c_int64()
        amp = np.zeros((ns, M), np.complex64)
        length = np.zeros((ns, M), np.float64)
        _check(lib().rt_ris_paths_read(self._h, ch, _ptr(amp) if amp.size else None,
                                       _ptr(length) if length.size else None, amp.size, ctypes.byref(n)))
        return amp, length

    # ---- RIS sum ----
    def cir(self, ch: int, gamma, bin_s: float, n_bins: int, stream=None):
        """Delay-binned impulse response of one configuration (gamma: torch
        complex64 device tensor [M]); returns a torch complex64 [R, n_bins]
        device tensor.  The channel needs FLAG_KEEP_CIR."""
        import torch
        R = int(self.channel_info(ch)[0])
        dev = gamma.device if hasattr(gamma, "device") else torch.device("cuda")
        with _OnStream(stream) as on:
            g = gamma.contiguous()
            out = torch.zeros((R, n_bins), dtype=torch.complex64, device=dev)   # cleared in the call's order
            _check(lib().rt_cir(self._h, ctypes.c_uint64(ch), ctypes.c_void_p(g.data_ptr()), float(bin_s),
                                int(n_bins), ctypes.c_void_p(out.data_ptr()), on.handle))
            on.keep(gamma)
        return out

    def ris_sum(self, ch: int, gamma, scale: float = 1.0, gamma_is_real: bool = False,
                precision: int = PREC_MFMA_BF16X2, want_E: bool = False, want_P: bool = True, stream=None,
                E_out=None, P_out=None):
        """gamma: torch complex64 device tensor [M, C].  Returns (E, P) device
        tensors (None where not requested)."""
        import torch
        R, M, _, _ = self.channel_info(ch)
        C = int(gamma.shape[1])
        given = (gamma, E_out, P_out)
        with _OnStream(stream) as on:
            g = gamma.contiguous()
            dev = g.device
            if want_E and E_out is None:
                E_out = torch.empty((R, C), dtype=torch.complex64, device=dev)
            if want_P and P_out is None:
                P_out = torch.empty((R, C), dtype=torch.float32, device=dev)
            _check(lib().rt_ris_sum(self._h, ch, ctypes.c_void_p(g.data_ptr()), C, float(scale),
                                    int(gamma_is_real), int(precision),
                                    ctypes.c_void_p(E_out.data_ptr()) if E_out is not None else None,
                                    ctypes.c_void_p(P_out.data_ptr()) if P_out is not None else None, on.handle))
            on.keep(*given)
        return E_out, P_out


def ris_sum_noalloc(ctx: Context, ch: int, gamma, E_out=None, P_out=None, scale: float = 1.0,
                    gamma_is_real: bool = False, precision: int = PREC_MFMA_BF16X2, stream=None):
    """rt_ris_sum_noalloc: the sum into caller-allocated outputs (torch device
    tensors: E_out complex64 [R, C] and/or P_out float32 [R, C]) with the
    library's static scratch; gamma must be a contiguous complex64 device
    tensor [M, C].  Nothing is allocated here either."""
    if E_out is None and P_out is None:
        raise ValueError("give E_out and/or P_out")
    if not gamma.is_contiguous():
        raise ValueError("gamma must be contiguous")
    _check(lib().rt_ris_sum_noalloc(ctx._h, ch, ctypes.c_void_p(gamma.data_ptr()), int(gamma.shape[1]),
                                    float(scale), int(gamma_is_real), int(precision),
                                    ctypes.c_void_p(E_out.data_ptr()) if E_out is not None else None,
                                    ctypes.c_void_p(P_out.data_ptr()) if P_out is not None else None,
                                    _stream_handle(stream)))


CHANNEL_FILE_VERSION = 1


def channel_save(ctx: Context, ch: int, path: str, **meta) -> str:
    """Write a channel to an ``.npz`` file: E_env complex64 [R], H complex64
    [R, M] (receiver-major, as rt_channel_read gives them) and a JSON string of
    the keyword arguments (deployment parameters, say).  Nothing in the file is
    pickled.  Returns the path written (numpy adds ``.npz`` if it is missing)."""
    E, H = ctx.channel_read(ch)
    doc = dict(meta, version=CHANNEL_FILE_VERSION, R=int(H.shape[0]), M=int(H.shape[1]))
    if not path.endswith(".npz"):
        path += ".npz"
    np.savez(path, E_env=E, H=H, meta=np.array(json.dumps(doc, sort_keys=True)))
    return path


def read_channel_file(path: str):
    """(E_env, H, meta) of a file written by channel_save, checked: complex64
    arrays, E_env [R] and H [R, M] with the R and M the metadata states, all
    finite.  Raises ValueError on anything else."""
    with np.load(path, allow_pickle=False) as f:
        for k in ("E_env", "H", "meta"):
            if k not in f.files:
                raise ValueError("%s: no %s array" % (path, k))
        E, H, raw = f["E_env"], f["H"], f["meta"]
    if raw.shape != () or raw.dtype.kind != "U":
        raise ValueError("%s: meta is not a string" % path)
    try:
        meta = json.loads(str(raw))
    except json.JSONDecodeError as e:
        raise ValueError("%s: meta is not JSON (%s)" % (path, e)) from None
    if not isinstance(meta, dict):
        raise ValueError("%s: meta is not a JSON object" % path)
    if meta.get("version") != CHANNEL_FILE_VERSION:
        raise ValueError("%s: channel file version %r" % (path, meta.get("version")))
    if E.dtype != np.complex64 or H.dtype != np.complex64:
        raise ValueError("%s: arrays must be complex64" % path)
    if E.ndim != 1 or H.ndim != 2 or H.shape[0] != E.shape[0] or (meta.get("R"), meta.get("M")) != H.shape:
        raise ValueError("%s: shapes E_env %s, H %s do not match R, M = %s, %s"
                         % (path, E.shape, H.shape, meta.get("R"), meta.get("M")))
    if not (np.isfinite(E.view(np.float32)).all() and np.isfinite(H.view(np.float32)).all()):
        raise ValueError("%s: non-finite values" % path)
    return E, H, meta


def channel_load(ctx: Context, path: str, stream=None):
    """Channel handle (rt_channel_create) and metadata of a file written by
    channel_save."""
    E, H, meta = read_channel_file(path)
    return ctx.channel_create(E, H, stream=stream), meta


def upload_problem(ctx: Context, prob, stream=None):
    """Create the scene and RIS objects of a synthetic problem.  Returns
    (scene handle, ris handle or 0)."""
    sc = prob.scene
    scene = ctx.scene_create(sc.V, sc.T, sc.surf, sc.refl_re, sc.refl_im, stream=stream)
    if getattr(prob, "mat_eps_r", None) is not None:
        ctx.scene_set_materials(scene, prob.mat_eps_r, prob.mat_sigma, stream=stream)
    ris = 0
    if prob.ris is not None:
        r = prob.ris
        ris = ctx.ris_create(r.elems, r.centre, r.normal, r.dy, r.dz, r.gain, r.q)
    return scene, ris


def trace_problem(ctx: Context, prob, scene: int, ris: int, flags: int = 0, n_rays: Optional[int] = None,
                  rx=None, stream=None):
    """Trace a synthetic problem (its Fresnel choice, if any, adds the flag)."""
    pol = getattr(prob, "fresnel", 0)
    flags |= FLAG_FRESNEL_TE if pol == 1 else FLAG_FRESNEL_TM if pol == 2 else 0
    return ctx.trace(scene, ris, prob.tx_pos, prob.tx_ant.axis, prob.tx_power_w, prob.tx_ant.gain,
                     prob.tx_ant.pattern, prob.tx_ant.param, prob.rx_pos if rx is None else rx,
                     prob.rx_ant.axis, prob.rx_ant.gain, prob.rx_ant.pattern, prob.rx_ant.param, prob.freq,
                     prob.order, prob.n_rays if n_rays is None else n_rays, flags=flags, stream=stream)
