"""Python binding of libunihenn (include/unihenn.h): argument marshalling only.

Every computation runs in the HIP library; torch provides device memory
(int64 tensors reinterpreted as uint64 residues) and streams.  The binding
refuses to run without the built library: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # imported first so the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libunihenn.so")

OK, EINVAL, ELEVEL, ESCALE, ENOKEY, ESLOTS, ENOMEM, EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
LAYER_CONV, LAYER_SQUARE, LAYER_AVGPOOL, LAYER_FLATTEN, LAYER_FC, LAYER_RELU_APPROX = 1, 2, 3, 4, 5, 6
EVAL_PLAIN, EVAL_HOISTED, EVAL_GRAPH = 0, 1, 2
PLAN_LAZY_MODDOWN, PLAN_FC_DOUBLING, PLAN_CHANNEL_CTS = 1, 2, 4
KERNEL_FAMILIES = ["ntt_fwd_col", "ntt_fwd_row", "ntt_inv_row", "ntt_inv_col", "modup", "ks_inner", "moddown",
                   "rescale", "mac", "automorphism", "tensor", "add", "encode", "other", "ks_rowfused"]


class UnihennError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"unihenn error {code}: {msg}")
        self.code = code


class CT(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n_limbs", C.c_uint32), ("batch", C.c_uint32), ("scale", C.c_double)]


class EVK(C.Structure):
    _fields_ = [("data", C.c_void_p), ("n_data", C.c_uint32)]


class LAYER(C.Structure):
    _fields_ = [("kind", C.c_int32), ("ch_in", C.c_uint32), ("ch_out", C.c_uint32), ("k", C.c_uint32),
                ("s", C.c_uint32), ("dims", C.c_uint32), ("weights", C.POINTER(C.c_double)),
                ("bias", C.POINTER(C.c_double)), ("pad", C.c_uint32)]


class TUNING(C.Structure):
    _fields_ = [("ntt_split", C.c_int32), ("ntt_tile_log", C.c_int32), ("mac_min_wg", C.c_int32),
                ("ks_min_wg", C.c_int32), ("ks_group", C.c_int32), ("ks_order", C.c_int32), ("ntt_ms", C.c_double),
                ("net_ms", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class INPUT(C.Structure):
    _fields_ = [("c", C.c_uint32), ("h", C.c_uint32), ("w", C.c_uint32), ("samples", C.c_uint32),
                ("stride", C.c_uint32), ("pitch", C.c_uint32), ("lead", C.c_uint32)]


# name -> (restype, argtypes); every symbol declared in include/unihenn.h
_vp, _u32, _i32, _u64, _d, _sz = C.c_void_p, C.c_uint32, C.c_int32, C.c_uint64, C.c_double, C.c_size_t
_P = C.POINTER
SIGNATURES = {
    "unihenn_last_error": (C.c_char_p, []),
    "unihenn_ctx_create": (C.c_int, [_u32, _P(_u32), _u32, _u32, _d, _P(_vp)]),
    "unihenn_ctx_destroy": (C.c_int, [_vp]),
    "unihenn_ctx_primes": (C.c_int, [_vp, _P(_u64)]),
    "unihenn_to_ntt": (C.c_int, [_vp, _vp, _u32, _u32, _vp]),
    "unihenn_from_ntt": (C.c_int, [_vp, _vp, _u32, _u32, _vp]),
    "unihenn_import_ct": (C.c_int, [_vp, _vp, _P(CT), _vp]),
    "unihenn_export_ct": (C.c_int, [_vp, _P(CT), _vp, _vp]),
    "unihenn_import_evk": (C.c_int, [_vp, _vp, _u32, _vp, _vp]),
    "unihenn_encode": (C.c_int, [_vp, _P(_d), _u32, _d, _u32, C.c_int, _vp, _vp]),
    "unihenn_import_pt": (C.c_int, [_vp, _vp, _u32, C.c_int, _vp, _vp]),
    "unihenn_export_pt": (C.c_int, [_vp, _vp, _u32, C.c_int, _vp, _vp]),
    "unihenn_ks_workspace_size": (_sz, [_vp, _u32, _u32]),
    "unihenn_rotate": (C.c_int, [_vp, _P(CT), _i32, _P(EVK), _P(CT), _vp, _sz, _vp]),
    "unihenn_rotate_hoisted": (C.c_int, [_vp, _P(CT), _P(_i32), _u32, _P(EVK), _P(CT), _vp, _sz, _vp]),
    "unihenn_rotate_noalloc": (C.c_int, [_vp, _P(CT), _i32, _P(EVK), _P(CT), _vp]),
    "unihenn_mul_plain_acc": (C.c_int, [_vp, _P(CT), _P(_vp), _u32, C.c_int, _P(CT), _vp]),
    "unihenn_rescale": (C.c_int, [_vp, _P(CT), _P(CT), _vp, _sz, _vp]),
    "unihenn_square_relin": (C.c_int, [_vp, _P(CT), _P(EVK), _P(CT), _vp, _sz, _vp]),
    "unihenn_drop_level_workspace_size": (C.c_size_t, [_vp, _u32, _u32]),
    "unihenn_drop_level": (C.c_int, [_vp, _P(CT), _P(CT), _u32, _P(EVK), _P(CT), _vp, C.c_size_t, _vp]),
    "unihenn_mul_relin": (C.c_int, [_vp, _P(CT), _P(CT), _P(EVK), _P(CT), _vp, _sz, _vp]),
    "unihenn_add": (C.c_int, [_vp, _P(CT), _P(CT), _P(CT), _vp]),
    "unihenn_add_plain": (C.c_int, [_vp, _P(CT), _vp, _P(CT), _vp]),
    "unihenn_mod_drop": (C.c_int, [_vp, _P(CT), _u32, _P(CT), _vp]),
    "unihenn_net_create": (C.c_int, [_vp, _P(INPUT), _P(LAYER), _u32, _u32, _P(_vp)]),
    "unihenn_net_create_ex": (C.c_int, [_vp, _P(INPUT), _P(LAYER), _u32, _u32, _u32, _P(_vp)]),
    "unihenn_net_inputs": (C.c_int, [_vp, _P(_u32)]),
    "unihenn_net_destroy": (C.c_int, [_vp]),
    "unihenn_net_info": (C.c_int, [_vp, _P(_u32), _P(_u32), _P(_u32), _P(_u32)]),
    "unihenn_net_rotations": (C.c_int, [_vp, _P(_i32)]),
    "unihenn_net_bind_keys": (C.c_int, [_vp, _P(_i32), _P(EVK), _u32, _P(EVK)]),
    "unihenn_net_set_mode": (C.c_int, [_vp, C.c_int]),
    "unihenn_conv": (C.c_int, [_vp, _vp, _u32, _P(CT), _u32, _P(CT), _P(_u32), _vp]),
    "unihenn_eval_network": (C.c_int, [_vp, _vp, _P(CT), _P(CT), _vp]),
    "unihenn_net_output_slots": (C.c_int, [_vp, _P(_u64), _P(_u32)]),
    "unihenn_net_stages": (C.c_int, [_vp, _P(_u32)]),
    "unihenn_eval_stage": (C.c_int, [_vp, _vp, _u32, _u32, _u32, _P(CT), _P(CT), _vp]),
    "unihenn_net_memory": (C.c_int, [_vp, _P(_sz), _P(_sz)]),
    "unihenn_workspace_size": (C.c_int, [_vp, _vp, _u32, _P(_sz)]),
    "unihenn_autotune": (C.c_int, [_vp, _vp, _u32, C.c_char_p, _P(TUNING), _vp]),
    "unihenn_tuning_get": (C.c_int, [_vp, _vp, _P(TUNING)]),
    "unihenn_tuning_set": (C.c_int, [_vp, _vp, _P(TUNING)]),
    "unihenn_keygen_secret": (C.c_int, [_vp, _u64, _vp, _vp]),
    "unihenn_gen_switch_key": (C.c_int, [_vp, _vp, _u64, _i32, C.c_int, _vp, _vp]),
    "unihenn_encrypt_sk": (C.c_int, [_vp, _vp, _vp, _u64, _P(CT), _vp]),
    "unihenn_decrypt_slots": (C.c_int, [_vp, _vp, _P(CT), _P(_u32), _u32, _P(_d), _vp]),
    "unihenn_stats_enable": (C.c_int, [C.c_int]),
    "unihenn_stats_reset": (C.c_int, []),
    "unihenn_stats_get": (C.c_int, [C.c_int, _P(_u64), _P(_d), _P(_d), _P(_d)]),
    "unihenn_kernel_family_name": (C.c_char_p, [C.c_int]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2402_03060_amd/build.py "
                               "(there is no fallback path)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue  # reported by missing_symbols()
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def missing_symbols() -> list[str]:
    L = lib()
    return [n for n in SIGNATURES if getattr(L, n, None) is None]


def _check(rc: int):
    if rc != OK:
        raise UnihennError(rc, lib().unihenn_last_error().decode())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def device_u64(a: np.ndarray, device="cuda") -> torch.Tensor:
    """uint64 numpy array -> int64 device tensor with the same bits."""
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).to(device)


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


class Ciphertext:
    """A batch of device ciphertexts [batch][2][n_limbs][N] (NTT form)."""

    def __init__(self, data: torch.Tensor, scale: float):
        assert data.dtype == torch.int64 and data.is_cuda and data.is_contiguous() and data.dim() == 4
        self.data = data
        self.scale = float(scale)

    @property
    def batch(self):
        return self.data.shape[0]

    @property
    def n_limbs(self):
        return self.data.shape[2]

    def desc(self) -> CT:
        return CT(self.data.data_ptr(), self.n_limbs, self.batch, self.scale)


class Context:
    def __init__(self, log_n: int, prime_bits, special_bits: int, scale: float):
        self.log_n = log_n
        self.n = 1 << log_n
        self.slots = self.n // 2
        self.n_data = len(prime_bits)
        self.scale = float(scale)
        bits = (C.c_uint32 * len(prime_bits))(*prime_bits)
        h = C.c_void_p()
        _check(lib().unihenn_ctx_create(log_n, bits, len(prime_bits), special_bits, float(scale), C.byref(h)))
        self.h = h
        out = (C.c_uint64 * (self.n_data + 1))()
        _check(lib().unihenn_ctx_primes(self.h, out))
        self.primes = [int(x) for x in out[: self.n_data]]
        self.special = int(out[self.n_data])

    def close(self):
        if self.h:
            lib().unihenn_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- launch parameters ----
    def tuning(self) -> dict:
        t = TUNING()
        _check(lib().unihenn_tuning_get(self.h, None, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = TUNING(**{k: int(v) for k, v in kw.items()})
        _check(lib().unihenn_tuning_set(self.h, None, C.byref(t)))

    def autotune(self, batch: int = 1, cache_path: str | None = None) -> dict:
        """Tune the NTT split and tile for transforms of about `batch` ciphertexts."""
        t = TUNING()
        _check(lib().unihenn_autotune(self.h, None, batch, cache_path.encode() if cache_path else None,
                                      C.byref(t), _stream()))
        return t.as_dict()

    # ---- allocation helpers (torch) ----
    def empty_ct(self, batch: int, n_limbs: int, scale: float = 0.0) -> Ciphertext:
        return Ciphertext(torch.empty((batch, 2, n_limbs, self.n), dtype=torch.int64, device="cuda"), scale)

    def workspace(self, n_limbs: int, batch: int) -> torch.Tensor:
        nbytes = lib().unihenn_ks_workspace_size(self.h, n_limbs, batch)
        return torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device="cuda")

    # ---- conversions ----
    def to_ntt(self, t: torch.Tensor, n_limbs: int, n_polys: int, stream=None):
        _check(lib().unihenn_to_ntt(self.h, t.data_ptr(), n_limbs, n_polys, _stream(stream)))

    def from_ntt(self, t: torch.Tensor, n_limbs: int, n_polys: int, stream=None):
        _check(lib().unihenn_from_ntt(self.h, t.data_ptr(), n_limbs, n_polys, _stream(stream)))

    def import_ct(self, coeff: np.ndarray, scale: float) -> Ciphertext:
        """unihenn_import_ct from host memory; coeff: uint64 [batch][2][n_limbs][N]
        or [2][n_limbs][N] (coefficient form)."""
        if coeff.ndim == 3:
            coeff = coeff[None]
        coeff = np.ascontiguousarray(coeff, dtype=np.uint64)
        ct = Ciphertext(torch.empty(coeff.shape, dtype=torch.int64, device="cuda"), scale)
        d = ct.desc()
        _check(lib().unihenn_import_ct(self.h, coeff.ctypes.data, C.byref(d), _stream()))
        torch.cuda.current_stream().synchronize()  # the host buffer is read by the copy
        return ct

    def export_ct(self, ct: Ciphertext) -> np.ndarray:
        """unihenn_export_ct into a device buffer, returned as uint64 host array."""
        out = torch.empty_like(ct.data)
        d = ct.desc()
        _check(lib().unihenn_export_ct(self.h, C.byref(d), out.data_ptr(), _stream()))
        torch.cuda.synchronize()
        return host_u64(out)

    def import_evk(self, coeff: np.ndarray) -> torch.Tensor:
        t = device_u64(coeff)
        _check(lib().unihenn_import_evk(self.h, t.data_ptr(), coeff.shape[0], t.data_ptr(), _stream()))
        return t

    def evk(self, t: torch.Tensor) -> EVK:
        return EVK(t.data_ptr(), self.n_data)

    def encode(self, z, scale: float, n_limbs: int, mont: bool = True) -> torch.Tensor:
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        out = torch.empty((n_limbs, self.n), dtype=torch.int64, device="cuda")
        _check(lib().unihenn_encode(self.h, z.ctypes.data_as(C.POINTER(C.c_double)), len(z), float(scale), n_limbs,
                                    int(mont), out.data_ptr(), _stream()))
        return out

    def import_pt(self, coeff: np.ndarray, mont: bool = True) -> torch.Tensor:
        t = device_u64(coeff)
        _check(lib().unihenn_import_pt(self.h, t.data_ptr(), coeff.shape[0], int(mont), t.data_ptr(), _stream()))
        return t

    def export_pt(self, pt: torch.Tensor, mont: bool = True) -> np.ndarray:
        out = torch.empty_like(pt)
        _check(lib().unihenn_export_pt(self.h, pt.data_ptr(), pt.shape[0], int(mont), out.data_ptr(), _stream()))
        torch.cuda.synchronize()
        return host_u64(out)

    # ---- primitives ----
    def rotate(self, ct: Ciphertext, steps: int, key: torch.Tensor | None, ws: torch.Tensor) -> Ciphertext:
        out = self.empty_ct(ct.batch, ct.n_limbs)
        o = out.desc()
        k = self.evk(key) if key is not None else None
        _check(lib().unihenn_rotate(self.h, C.byref(ct.desc()), int(steps), C.byref(k) if k else None, C.byref(o),
                                    ws.data_ptr(), ws.numel() * 8, _stream()))
        out.scale = o.scale
        return out

    def rotate_noalloc(self, ct: Ciphertext, steps: int, key: torch.Tensor | None, out: Ciphertext,
                       stream=None) -> Ciphertext:
        """unihenn_rotate_noalloc into a caller-made output (the library's
        fixed scratch array replaces the workspace)."""
        o = out.desc()
        k = self.evk(key) if key is not None else None
        _check(lib().unihenn_rotate_noalloc(self.h, C.byref(ct.desc()), int(steps), C.byref(k) if k else None,
                                            C.byref(o), _stream(stream)))
        out.scale = o.scale
        return out

    def rotate_hoisted(self, ct: Ciphertext, steps, keys, ws: torch.Tensor) -> list[Ciphertext]:
        steps = list(steps)
        outs = [self.empty_ct(ct.batch, ct.n_limbs) for _ in steps]
        od = (CT * len(steps))(*[o.desc() for o in outs])
        kd = (EVK * len(steps))(*[self.evk(k) if k is not None else EVK(None, self.n_data) for k in keys])
        sa = (C.c_int32 * len(steps))(*steps)
        _check(lib().unihenn_rotate_hoisted(self.h, C.byref(ct.desc()), sa, len(steps), kd, od, ws.data_ptr(),
                                            ws.numel() * 8, _stream()))
        for o, d in zip(outs, od):
            o.scale = d.scale
        return outs

    def mul_plain_acc(self, cts: list[Ciphertext], pts: list[torch.Tensor], acc: Ciphertext | None = None,
                      overwrite: bool = True) -> Ciphertext:
        if acc is None:
            acc = self.empty_ct(cts[0].batch, cts[0].n_limbs)
        cd = (CT * len(cts))(*[c.desc() for c in cts])
        pd = (C.c_void_p * len(pts))(*[p.data_ptr() for p in pts])
        a = acc.desc()
        _check(lib().unihenn_mul_plain_acc(self.h, cd, pd, len(cts), int(overwrite), C.byref(a), _stream()))
        acc.scale = a.scale
        return acc

    def rescale(self, ct: Ciphertext, ws: torch.Tensor) -> Ciphertext:
        out = self.empty_ct(ct.batch, ct.n_limbs - 1)
        o = out.desc()
        _check(lib().unihenn_rescale(self.h, C.byref(ct.desc()), C.byref(o), ws.data_ptr(), ws.numel() * 8,
                                     _stream()))
        out.scale = o.scale
        return out

    def square_relin(self, ct: Ciphertext, rlk: torch.Tensor, ws: torch.Tensor) -> Ciphertext:
        out = self.empty_ct(ct.batch, ct.n_limbs)
        o = out.desc()
        _check(lib().unihenn_square_relin(self.h, C.byref(ct.desc()), C.byref(self.evk(rlk)), C.byref(o),
                                          ws.data_ptr(), ws.numel() * 8, _stream()))
        out.scale = o.scale
        return out

    def mul_relin(self, a: Ciphertext, b: Ciphertext, rlk: torch.Tensor, ws: torch.Tensor) -> Ciphertext:
        out = self.empty_ct(a.batch, a.n_limbs)
        d = out.desc()
        k = self.evk(rlk)
        _check(lib().unihenn_mul_relin(self.h, C.byref(a.desc()), C.byref(b.desc()), C.byref(k), C.byref(d),
                                       ws.data_ptr(), ws.numel() * 8, _stream()))
        out.scale = d.scale
        return out

    def add(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        out = self.empty_ct(a.batch, a.n_limbs)
        o = out.desc()
        _check(lib().unihenn_add(self.h, C.byref(a.desc()), C.byref(b.desc()), C.byref(o), _stream()))
        out.scale = o.scale
        return out

    def add_plain(self, a: Ciphertext, pt: torch.Tensor) -> Ciphertext:
        out = self.empty_ct(a.batch, a.n_limbs)
        o = out.desc()
        _check(lib().unihenn_add_plain(self.h, C.byref(a.desc()), pt.data_ptr(), C.byref(o), _stream()))
        out.scale = o.scale
        return out

    def drop_level(self, a: Ciphertext, ones: list[Ciphertext], rlk: torch.Tensor) -> Ciphertext:
        """Drop-Level of Section IV-A as written: len(ones) products with
        encryptions of all-ones vectors, each relinearised and rescaled."""
        out = self.empty_ct(a.batch, a.n_limbs - len(ones))
        o = out.desc()
        oa = (CT * len(ones))(*[x.desc() for x in ones])
        nbytes = lib().unihenn_drop_level_workspace_size(self.h, a.n_limbs, a.batch)
        ws = torch.empty(max(nbytes // 8, 1), dtype=torch.int64, device="cuda")
        _check(lib().unihenn_drop_level(self.h, C.byref(a.desc()), oa, len(ones), C.byref(self.evk(rlk)),
                                        C.byref(o), ws.data_ptr(), nbytes, _stream()))
        out.scale = o.scale
        self._last_drop_ws = ws  # kept until the next call: the launches are asynchronous
        return out

    def mod_drop(self, a: Ciphertext, n_limbs: int) -> Ciphertext:
        out = self.empty_ct(a.batch, n_limbs)
        o = out.desc()
        _check(lib().unihenn_mod_drop(self.h, C.byref(a.desc()), n_limbs, C.byref(o), _stream()))
        out.scale = o.scale
        return out


def stats_enable(on: bool = True):
    _check(lib().unihenn_stats_enable(int(on)))


def stats_reset():
    _check(lib().unihenn_stats_reset())


def stats() -> dict:
    """{family: (launches, total_ms, algorithmic_bytes, algorithmic_ops)}"""
    out = {}
    for i, name in enumerate(KERNEL_FAMILIES):
        n = C.c_uint64()
        ms = C.c_double()
        by = C.c_double()
        op = C.c_double()
        _check(lib().unihenn_stats_get(i, C.byref(n), C.byref(ms), C.byref(by), C.byref(op)))
        out[name] = (int(n.value), float(ms.value), float(by.value), float(op.value))
    return out


# ---------------------------------------------------------------- client
def keygen_secret(ctx: Context, seed: int) -> torch.Tensor:
    sk = torch.empty((ctx.n_data + 1, ctx.n), dtype=torch.int64, device="cuda")
    _check(lib().unihenn_keygen_secret(ctx.h, seed, sk.data_ptr(), _stream()))
    return sk


def gen_switch_key(ctx: Context, sk: torch.Tensor, seed: int, steps: int = 0, relin: bool = False) -> torch.Tensor:
    nd = ctx.n_data
    out = torch.empty((nd, 2, nd + 1, ctx.n), dtype=torch.int64, device="cuda")
    _check(lib().unihenn_gen_switch_key(ctx.h, sk.data_ptr(), seed, int(steps), int(relin), out.data_ptr(), _stream()))
    return out


def encrypt_sk(ctx: Context, sk: torch.Tensor, pts: torch.Tensor, seed: int, scale: float) -> Ciphertext:
    """pts: [batch][n_limbs][N] plain-form plaintexts (encode with mont=False)."""
    B, nl = pts.shape[0], pts.shape[1]
    ct = ctx.empty_ct(B, nl, scale)
    d = ct.desc()
    _check(lib().unihenn_encrypt_sk(ctx.h, sk.data_ptr(), pts.data_ptr(), seed, C.byref(d), _stream()))
    return ct


def decrypt_slots(ctx: Context, sk: torch.Tensor, ct: Ciphertext, slots) -> np.ndarray:
    slots = np.ascontiguousarray(np.asarray(slots, dtype=np.uint32))
    out = np.zeros((ct.batch, len(slots)), dtype=np.float64)
    _check(lib().unihenn_decrypt_slots(ctx.h, sk.data_ptr(), C.byref(ct.desc()),
                                       slots.ctypes.data_as(C.POINTER(C.c_uint32)), len(slots),
                                       out.ctypes.data_as(C.POINTER(C.c_double)), _stream()))
    return out


# ---------------------------------------------------------------- network
_KIND = {"conv": LAYER_CONV, "square": LAYER_SQUARE, "avgpool": LAYER_AVGPOOL, "flatten": LAYER_FLATTEN,
         "fc": LAYER_FC, "relu_approx": LAYER_RELU_APPROX}


class Net:
    """A planned network with its plaintexts encoded on the device."""

    def __init__(self, ctx: Context, inp: dict, layers, params, samples: int = 1, stride: int = 0,
                 max_batch: int = 1, lazy: bool = False, fc_doubling: bool = False, channel_cts: bool = False):
        """lazy: plan with deferred ModDown (PLAN_LAZY_MODDOWN); fc_doubling:
        the FC's closing sum by doubling (PLAN_FC_DOUBLING); channel_cts: one
        input ciphertext per channel (PLAN_CHANNEL_CTS; eval takes a list)."""
        self.ctx = ctx
        self.lazy = lazy
        self.fc_doubling = fc_doubling
        self.channel_cts = channel_cts
        self._keep = []
        arr = (LAYER * len(layers))()
        for i, (L, p) in enumerate(zip(layers, params)):
            d = arr[i]
            d.kind = _KIND[L["kind"]]
            if L["kind"] == "conv":
                d.ch_in, d.ch_out, d.k, d.s, d.dims = L["ch_in"], L["ch_out"], L["k"], L["s"], L.get("dims", 2)
                d.pad = L.get("pad", 0)
            elif L["kind"] == "avgpool":
                d.k = L["c"]
            elif L["kind"] == "fc":
                d.ch_in, d.ch_out = L["din"], L["dout"]
            elif L["kind"] == "relu_approx" and "coeffs" in L:
                cf = np.ascontiguousarray(L["coeffs"], dtype=np.float64)
                self._keep.append(cf)
                d.weights = cf.ctypes.data_as(C.POINTER(C.c_double))
            if p is not None:
                w = np.ascontiguousarray(p[0], dtype=np.float64)
                b = np.ascontiguousarray(p[1], dtype=np.float64)
                self._keep += [w, b]
                d.weights = w.ctypes.data_as(C.POINTER(C.c_double))
                d.bias = b.ctypes.data_as(C.POINTER(C.c_double))
        ind = INPUT(inp["c"], inp["h"], inp["w"], samples, stride, inp.get("pitch", 0), inp.get("lead", 0))
        h = C.c_void_p()
        _check(lib().unihenn_net_create_ex(ctx.h, C.byref(ind), arr, len(layers), max_batch,
                                           (PLAN_LAZY_MODDOWN if lazy else 0) |
                                           (PLAN_FC_DOUBLING if fc_doubling else 0) |
                                           (PLAN_CHANNEL_CTS if channel_cts else 0), C.byref(h)))
        self.h = h
        self.samples = samples
        self.max_batch = max_batch
        dep, nrot, nout, inl = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check(lib().unihenn_net_info(h, C.byref(dep), C.byref(nrot), C.byref(nout), C.byref(inl)))
        self.depth, self.n_rot, self.n_out, self.in_limbs = dep.value, nrot.value, nout.value, inl.value
        nin = C.c_uint32()
        _check(lib().unihenn_net_inputs(h, C.byref(nin)))
        self.n_inputs = nin.value
        self._bound = None

    def close(self):
        if self.h:
            lib().unihenn_net_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rotations(self) -> list[int]:
        a = (C.c_int32 * max(self.n_rot, 1))()
        _check(lib().unihenn_net_rotations(self.h, a))
        return [int(x) for x in a[: self.n_rot]]

    def bind_keys(self, keys: dict, rlk: torch.Tensor | None):
        steps = sorted(keys)
        sa = (C.c_int32 * max(len(steps), 1))(*steps)
        ka = (EVK * max(len(steps), 1))(*[self.ctx.evk(keys[s]) for s in steps])
        r = self.ctx.evk(rlk) if rlk is not None else None
        _check(lib().unihenn_net_bind_keys(self.h, sa, ka, len(steps), C.byref(r) if r is not None else None))
        self._bound = (keys, rlk)  # the library keeps raw pointers

    def set_mode(self, mode: int):
        _check(lib().unihenn_net_set_mode(self.h, mode))

    def tuning(self) -> dict:
        t = TUNING()
        _check(lib().unihenn_tuning_get(self.ctx.h, self.h, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = TUNING(**{k: int(v) for k, v in kw.items()})
        _check(lib().unihenn_tuning_set(self.ctx.h, self.h, C.byref(t)))

    def autotune(self, batch: int | None = None, cache_path: str | None = None) -> dict:
        """Tune the context's NTT launches and this net's key-switch group size
        and workgroup targets on whole evaluations of `batch` ciphertexts
        (default max_batch); with cache_path, reuse or record the result."""
        t = TUNING()
        b = self.max_batch if batch is None else batch
        _check(lib().unihenn_autotune(self.ctx.h, self.h, b, cache_path.encode() if cache_path else None,
                                      C.byref(t), _stream()))
        return t.as_dict()

    def output_slots(self) -> np.ndarray:
        nv = C.c_uint32()
        _check(lib().unihenn_net_output_slots(self.h, None, C.byref(nv)))
        pos = np.zeros(self.samples * nv.value, dtype=np.uint64)
        _check(lib().unihenn_net_output_slots(self.h, pos.ctypes.data_as(C.POINTER(C.c_uint64)), None))
        return pos.reshape(self.samples, nv.value)

    def alloc_outputs(self, batch: int) -> list[Ciphertext]:
        return [self.ctx.empty_ct(batch, 1) for _ in range(self.n_out)]

    def eval(self, ct, outs: list[Ciphertext] | None = None, stream=None) -> list[Ciphertext]:
        """ct: the input Ciphertext, or a list of n_inputs of them (one per
        channel with channel_cts)."""
        cts = list(ct) if isinstance(ct, (list, tuple)) else [ct]
        if len(cts) != self.n_inputs:
            raise ValueError(f"the net takes {self.n_inputs} input ciphertexts, got {len(cts)}")
        outs = self.alloc_outputs(cts[0].batch) if outs is None else outs
        od = (CT * self.n_out)(*[o.desc() for o in outs])
        ia = (CT * len(cts))(*[c.desc() for c in cts])
        _check(lib().unihenn_eval_network(self.ctx.h, self.h, ia, od, _stream(stream)))
        for o, d in zip(outs, od):
            o.scale = d.scale
        return outs

    def stages(self) -> int:
        n = C.c_uint32()
        _check(lib().unihenn_net_stages(self.h, C.byref(n)))
        return n.value

    def memory(self) -> tuple[int, int]:
        """(fixed bytes, bytes per batch slot) of the net's device memory."""
        f, p = C.c_size_t(), C.c_size_t()
        _check(lib().unihenn_net_memory(self.h, C.byref(f), C.byref(p)))
        return f.value, p.value

    def workspace_size(self, batch: int | None = None) -> int:
        """unihenn_workspace_size: bytes of the workspace the net evaluates in."""
        b = C.c_size_t()
        _check(lib().unihenn_workspace_size(self.ctx.h, self.h, self.max_batch if batch is None else batch,
                                            C.byref(b)))
        return b.value

    def eval_stage(self, stage: int, slot: int, batch: int, ct=None, outs: list[Ciphertext] | None = None,
                   stream=None):
        """unihenn_eval_stage: stage `stage` on batch slots [slot, slot + batch);
        ct (stage 0): the input Ciphertext or a list of n_inputs of them; outs
        (last stage): n_out Ciphertexts of `batch` entries."""
        ia = None
        if ct is not None:
            cts = list(ct) if isinstance(ct, (list, tuple)) else [ct]
            ia = (CT * len(cts))(*[c.desc() for c in cts])
        od = (CT * self.n_out)(*[o.desc() for o in outs]) if outs is not None else None
        _check(lib().unihenn_eval_stage(self.ctx.h, self.h, stage, slot, batch, ia, od, _stream(stream)))
        if outs is not None:
            for o, d in zip(outs, od):
                o.scale = d.scale
        return outs

    def conv(self, layer: int, ins: list[Ciphertext], n_out: int, out_limbs: int):
        outs = [self.ctx.empty_ct(ins[0].batch, out_limbs) for _ in range(n_out)]
        ia = (CT * len(ins))(*[c.desc() for c in ins])
        od = (CT * n_out)(*[o.desc() for o in outs])
        interval = C.c_uint32()
        _check(lib().unihenn_conv(self.ctx.h, self.h, layer, ia, len(ins), od, C.byref(interval), _stream()))
        for o, d in zip(outs, od):
            o.scale = d.scale
        return outs, interval.value
