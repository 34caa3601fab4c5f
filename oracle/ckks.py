"""Python face of the CPU oracle: client (keys, encryption, decryption, decoding)
and a slow evaluator of the CKKS primitives of UniHENN Section II-B.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the benchmark's
CPU-baseline leg.  The product library never imports this package.

All ciphertexts here are in coefficient form, residues in [0, q_i), laid out
[2][limbs][N] (numpy uint64).  Heavy arithmetic runs in ckks_oracle.c; the CRT
reconstruction and the decoding run here on Python integers and numpy FFTs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ckks_oracle.c")
_LIB = os.path.join(_HERE, "libckks_oracle.so")

_u64p = C.POINTER(C.c_uint64)
_i64p = C.POINTER(C.c_int64)
_vp = C.c_void_p


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no GPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", _SRC, "-lquadmath", "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        L.or_gen_primes.argtypes = [C.c_int, C.POINTER(C.c_int), C.c_int, _u64p]
        L.or_is_prime.argtypes = [C.c_uint64]
        L.or_prng_new.argtypes = [C.c_uint64]
        L.or_prng_new.restype = _vp
        L.or_prng_free.argtypes = [_vp]
        L.or_sample.argtypes = [_vp, C.c_int, C.c_uint64, C.c_int, _i64p]
        L.or_gauss_candidate.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int)]
        L.or_ctx_new.argtypes = [C.c_int, _u64p, C.c_int]
        L.or_ctx_new.restype = _vp
        L.or_ctx_free.argtypes = [_vp]
        L.or_ctx_psi.argtypes = [_vp, C.c_int]
        L.or_ctx_psi.restype = C.c_uint64
        L.or_poly_mul.argtypes = [_vp, C.c_int, _u64p, _u64p, _u64p]
        L.or_encode.argtypes = [_vp, C.POINTER(C.c_double), C.c_int, C.c_double, C.c_int, _u64p]
        L.or_encode_scaled.argtypes = [_vp, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double), C.c_int,
                                       C.c_double, C.c_int, _u64p]
        L.or_real_transform.argtypes = [_vp, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.or_galois_elt.argtypes = [_vp, C.c_int64]
        L.or_galois_elt.restype = C.c_uint64
        L.or_automorphism.argtypes = [_vp, _u64p, C.c_int, C.c_uint64, _u64p]
        L.or_gen_secret.argtypes = [_vp, _vp, C.POINTER(C.c_int8)]
        L.or_gen_pk.argtypes = [_vp, _vp, C.POINTER(C.c_int8), C.c_int, _u64p]
        L.or_gen_rotation_key.argtypes = [_vp, _vp, C.POINTER(C.c_int8), C.c_int, C.c_int64, _u64p]
        L.or_gen_relin_key.argtypes = [_vp, _vp, C.POINTER(C.c_int8), C.c_int, _u64p]
        L.or_gen_rotation_key_rows.argtypes = [_vp, _vp, C.POINTER(C.c_int8), C.c_int, C.c_int64, C.c_int, _u64p]
        L.or_gen_relin_key_rows.argtypes = [_vp, _vp, C.POINTER(C.c_int8), C.c_int, C.c_int, _u64p]
        L.or_encrypt_pk.argtypes = [_vp, _vp, _u64p, _u64p, C.c_int, _u64p]
        L.or_decrypt.argtypes = [_vp, C.POINTER(C.c_int8), _u64p, C.c_int, _u64p]
        L.or_key_load.argtypes = [_vp, _u64p, C.c_int]
        L.or_key_load.restype = _vp
        L.or_key_free.argtypes = [_vp]
        L.or_keyswitch.argtypes = [_vp, _u64p, C.c_int, _vp, _u64p]
        L.or_rotate.argtypes = [_vp, _u64p, C.c_int, C.c_int64, _vp, _u64p]
        L.or_rotate_hoisted.argtypes = [_vp, _u64p, C.c_int, _i64p, C.c_int, C.POINTER(_vp), _u64p]
        L.or_mac_matrix.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(_u64p), C.c_int, C.POINTER(_u64p),
                                    C.POINTER(_u64p)]
        L.or_add.argtypes = [_vp, _u64p, _u64p, C.c_int, C.c_int, _u64p]
        L.or_square_relin.argtypes = [_vp, _u64p, C.c_int, _vp, _u64p]
        L.or_mul_relin.argtypes = [_vp, _u64p, _u64p, C.c_int, _vp, _u64p]
        L.or_rescale.argtypes = [_vp, _u64p, C.c_int, C.c_int, _u64p]
        L.or_encode_scaled_ext.argtypes = [_vp, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double), C.c_int,
                                           C.c_double, C.c_int, _u64p]
        L.or_rotate_ext.argtypes = [_vp, _u64p, C.c_int, C.c_int64, _vp, _u64p]
        L.or_to_ext.argtypes = [_vp, _u64p, C.c_int, C.c_int, _u64p]
        L.or_moddown.argtypes = [_vp, _u64p, C.c_int, C.c_int, _u64p]
        L.or_add_ext.argtypes = [_vp, _u64p, _u64p, C.c_int, C.c_int, _u64p]
        L.or_mac_matrix_ext.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(_u64p), C.c_int, C.POINTER(_u64p),
                                        C.POINTER(_u64p)]
        _lib = L
    return _lib


def _p64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def _pd(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def gen_primes(log_n: int, bits) -> list[int]:
    """Prime chain (reading of the unspecified parameter choice): for each bit
    size in order, the largest unused prime p < 2^b, p = 1 mod 2N."""
    bits = list(bits)
    out = np.zeros(len(bits), dtype=np.uint64)
    arr = (C.c_int * len(bits))(*bits)
    if lib().or_gen_primes(log_n, arr, len(bits), _p64(out)) != 0:
        raise ValueError("no prime found")
    return [int(x) for x in out]


@dataclass
class Ciphertext:
    data: np.ndarray  # uint64 [2][nl][N], coefficient form
    scale: float

    @property
    def nl(self) -> int:
        return self.data.shape[1]


@dataclass
class ExtCiphertext:
    """Ciphertext over the extended basis {q_0..q_{nl-1}, P}: it stands for
    ModDown of itself (see the deferred-ModDown section of ckks_oracle.c)."""
    data: np.ndarray  # uint64 [2][nl+1][N], coefficient form
    scale: float

    @property
    def nl(self) -> int:
        return self.data.shape[1] - 1


class Secret:
    def __init__(self, s: np.ndarray):
        self.s = s  # int8 [N]


class OracleCKKS:
    """CKKS context over R = Z[X]/(X^N+1) with data primes q_0..q_L and a
    special prime P (key switching only)."""

    def __init__(self, log_n: int, prime_bits, special_bits: int, log_scale: int = 40):
        self.log_n = log_n
        self.n = 1 << log_n
        self.slots = self.n // 2
        allp = gen_primes(log_n, list(prime_bits) + [special_bits])
        self.primes = allp[:-1]
        self.special = allp[-1]
        self.n_data = len(self.primes)
        self.delta = float(2 ** log_scale)
        mods = np.array(allp, dtype=np.uint64)
        self.ctx = lib().or_ctx_new(log_n, _p64(mods), len(allp))
        self._keys: list = []

    def __del__(self):
        try:
            L = lib()
            for k in self._keys:
                L.or_key_free(k)
            L.or_ctx_free(self.ctx)
        except Exception:
            pass

    # -- slots / encoding ------------------------------------------------
    def galois_elt(self, r: int) -> int:
        return int(lib().or_galois_elt(self.ctx, int(r)))

    def encode(self, z, scale: float, nl: int) -> np.ndarray:
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        out = np.zeros((nl, self.n), dtype=np.uint64)
        if lib().or_encode(self.ctx, _pd(z), len(z), float(scale), nl, _p64(out)) != 0:
            raise ValueError("encode overflow")
        return out

    def encode_scaled(self, z, ws, scale: float, nl: int) -> np.ndarray:
        """Encode(w * z) for every w in ws: [len(ws)][nl][N]."""
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        ws = np.ascontiguousarray(np.asarray(ws, dtype=np.float64).ravel())
        out = np.zeros((len(ws), nl, self.n), dtype=np.uint64)
        rc = lib().or_encode_scaled(self.ctx, _pd(z), len(z), _pd(ws), len(ws), float(scale), nl, _p64(out))
        if rc != 0:
            raise ValueError("encode overflow")
        return out

    def encode_scaled_ext(self, z, ws, scale: float, nl: int) -> np.ndarray:
        """encode_scaled with the residue mod P as limb nl: [len(ws)][nl+1][N]."""
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        ws = np.ascontiguousarray(np.asarray(ws, dtype=np.float64).ravel())
        out = np.zeros((len(ws), nl + 1, self.n), dtype=np.uint64)
        rc = lib().or_encode_scaled_ext(self.ctx, _pd(z), len(z), _pd(ws), len(ws), float(scale), nl, _p64(out))
        if rc != 0:
            raise ValueError("encode overflow")
        return out

    def real_transform(self, z) -> tuple[np.ndarray, np.ndarray]:
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float64))
        hi = np.zeros(self.n)
        lo = np.zeros(self.n)
        lib().or_real_transform(self.ctx, _pd(z), len(z), _pd(hi), _pd(lo))
        return hi, lo

    def crt_centered(self, res: np.ndarray) -> list[int]:
        """Centered CRT reconstruction of residues [nl][N] to Python ints."""
        nl = res.shape[0]
        qs = self.primes[:nl]
        Q = 1
        for q in qs:
            Q *= q
        coef = [0] * self.n
        for i, q in enumerate(qs):
            Qi = Q // q
            f = Qi * pow(Qi, -1, q)
            col = res[i].tolist()
            for j in range(self.n):
                coef[j] += col[j] * f
        half = Q // 2
        out = []
        for v in coef:
            v %= Q
            out.append(v - Q if v > half else v)
        return out

    def decode_coeffs(self, coeffs, scale: float) -> np.ndarray:
        """Slots z_k = m(zeta_k) / scale, zeta_k = exp(i pi 5^k / N), via a
        length-2N FFT evaluation at every odd power of exp(i pi / N)."""
        m = np.array([float(c) for c in coeffs]) / scale
        pad = np.zeros(2 * self.n)
        pad[: self.n] = m
        ev = np.fft.ifft(pad) * (2 * self.n)  # sum_j m_j exp(+2 pi i t j / 2N)
        e = np.array([pow(5, k, 2 * self.n) for k in range(self.slots)])
        return ev[e].real

    def decode(self, res: np.ndarray, scale: float) -> np.ndarray:
        return self.decode_coeffs(self.crt_centered(res), scale)

    # -- client ------------------------------------------------------------
    def keygen(self, seed: int) -> Secret:
        self._prng = lib().or_prng_new(seed)
        s = np.zeros(self.n, dtype=np.int8)
        lib().or_gen_secret(self.ctx, self._prng, s.ctypes.data_as(C.POINTER(C.c_int8)))
        self.sk = Secret(s)
        self.pk = np.zeros((2, self.n_data, self.n), dtype=np.uint64)
        lib().or_gen_pk(self.ctx, self._prng, s.ctypes.data_as(C.POINTER(C.c_int8)), self.n_data, _p64(self.pk))
        return self.sk

    def rotation_key(self, r: int) -> np.ndarray:
        """Coefficient-form switching key [L+1][2][L+2][N] for Rot(., r)."""
        k = np.zeros((self.n_data, 2, self.n_data + 1, self.n), dtype=np.uint64)
        lib().or_gen_rotation_key(self.ctx, self._prng, self.sk.s.ctypes.data_as(C.POINTER(C.c_int8)),
                                  self.n_data, int(r), _p64(k))
        return k

    def relin_key(self) -> np.ndarray:
        k = np.zeros((self.n_data, 2, self.n_data + 1, self.n), dtype=np.uint64)
        lib().or_gen_relin_key(self.ctx, self._prng, self.sk.s.ctypes.data_as(C.POINTER(C.c_int8)),
                               self.n_data, _p64(k))
        return k

    def seeded_key(self, seed: int, r: int | None = None, levels: int | None = None) -> np.ndarray:
        """A switching key from a generator of its own (seeded by `seed`, not
        the session's stream), so that keys can be made in any order or in
        parallel: Rot(., r), or relinearisation when r is None.  With
        `levels`, only the rows a ciphertext of that many limbs reads are
        formed (digits and limbs below `levels`, and P); the others are zero
        and the formed rows equal the whole key's."""
        lv = self.n_data if levels is None else int(levels)
        assert 1 <= lv <= self.n_data
        k = np.zeros((self.n_data, 2, self.n_data + 1, self.n), dtype=np.uint64)
        p = lib().or_prng_new(seed)
        s = self.sk.s.ctypes.data_as(C.POINTER(C.c_int8))
        if r is None:
            lib().or_gen_relin_key_rows(self.ctx, p, s, self.n_data, lv, _p64(k))
        else:
            lib().or_gen_rotation_key_rows(self.ctx, p, s, self.n_data, int(r), lv, _p64(k))
        lib().or_prng_free(p)
        return k

    def load_key(self, key: np.ndarray):
        h = lib().or_key_load(self.ctx, _p64(np.ascontiguousarray(key)), key.shape[0])
        self._keys.append(h)
        return h

    def encrypt(self, z, seed: int, scale: float | None = None) -> Ciphertext:
        scale = self.delta if scale is None else scale
        pt = self.encode(z, scale, self.n_data)
        return self.encrypt_pt(pt, seed, scale)

    def encrypt_pt(self, pt: np.ndarray, seed: int, scale: float) -> Ciphertext:
        p = lib().or_prng_new(seed)
        ct = np.zeros((2, self.n_data, self.n), dtype=np.uint64)
        lib().or_encrypt_pk(self.ctx, p, _p64(self.pk), _p64(np.ascontiguousarray(pt)), self.n_data, _p64(ct))
        lib().or_prng_free(p)
        return Ciphertext(ct, scale)

    def decrypt_residues(self, ct: Ciphertext) -> np.ndarray:
        m = np.zeros((ct.nl, self.n), dtype=np.uint64)
        lib().or_decrypt(self.ctx, self.sk.s.ctypes.data_as(C.POINTER(C.c_int8)),
                         _p64(np.ascontiguousarray(ct.data)), ct.nl, _p64(m))
        return m

    def decrypt(self, ct: Ciphertext) -> np.ndarray:
        return self.decode(self.decrypt_residues(ct), ct.scale)

    # -- evaluator -----------------------------------------------------------
    def limb_drop(self, ct: Ciphertext, nl: int) -> Ciphertext:
        """Drop-Level read as discarding the top limbs (Section IV-A)."""
        return Ciphertext(np.ascontiguousarray(ct.data[:, :nl, :]), ct.scale)

    def automorphism(self, poly: np.ndarray, g: int) -> np.ndarray:
        poly = np.ascontiguousarray(poly)
        out = np.zeros_like(poly)
        lib().or_automorphism(self.ctx, _p64(poly), poly.shape[0], int(g), _p64(out))
        return out

    def keyswitch(self, d: np.ndarray, key) -> np.ndarray:
        d = np.ascontiguousarray(d)
        out = np.zeros((2,) + d.shape, dtype=np.uint64)
        if lib().or_keyswitch(self.ctx, _p64(d), d.shape[0], key, _p64(out)) != 0:
            raise ValueError("key level")
        return out

    def rotate(self, ct: Ciphertext, r: int, key) -> Ciphertext:
        out = np.zeros_like(ct.data)
        if lib().or_rotate(self.ctx, _p64(np.ascontiguousarray(ct.data)), ct.nl, int(r), key, _p64(out)) != 0:
            raise ValueError("key level")
        return Ciphertext(out, ct.scale)

    def rotate_hoisted(self, ct: Ciphertext, rs, keys) -> list[Ciphertext]:
        rs = list(rs)
        outs = np.zeros((len(rs),) + ct.data.shape, dtype=np.uint64)
        ra = np.array(rs, dtype=np.int64)
        ka = (_vp * len(rs))(*keys)
        rc = lib().or_rotate_hoisted(self.ctx, _p64(np.ascontiguousarray(ct.data)), ct.nl,
                                     ra.ctypes.data_as(_i64p), len(rs), ka, _p64(outs))
        if rc != 0:
            raise ValueError("key level")
        return [Ciphertext(outs[i], ct.scale) for i in range(len(rs))]

    def mac_matrix(self, cts: list[Ciphertext], pts) -> list[np.ndarray]:
        """acc[o] = sum_t pts[o][t] * cts[t] (pts[o][t] may be None)."""
        nl = cts[0].nl
        n_ct, n_out = len(cts), len(pts)
        keep = [np.ascontiguousarray(c.data) for c in cts]
        ca = (_u64p * n_ct)(*[_p64(c) for c in keep])
        flat = []
        for o in range(n_out):
            for t in range(n_ct):
                p = pts[o][t]
                flat.append(None if p is None else np.ascontiguousarray(p))
        pa = (_u64p * len(flat))(*[(_p64(p) if p is not None else _u64p()) for p in flat])
        outs = [np.zeros((2, nl, self.n), dtype=np.uint64) for _ in range(n_out)]
        oa = (_u64p * n_out)(*[_p64(o) for o in outs])
        lib().or_mac_matrix(self.ctx, nl, n_ct, ca, n_out, pa, oa)
        return outs

    # -- deferred ModDown ----------------------------------------------------
    def rotate_ext(self, ct: Ciphertext, r: int, key) -> ExtCiphertext:
        """Rot(ct, r) before its ModDown: (P tau(c0) + U_0, U_1)."""
        out = np.zeros((2, ct.nl + 1, self.n), dtype=np.uint64)
        if lib().or_rotate_ext(self.ctx, _p64(np.ascontiguousarray(ct.data)), ct.nl, int(r), key, _p64(out)) != 0:
            raise ValueError("key level")
        return ExtCiphertext(out, ct.scale)

    def to_ext(self, ct: Ciphertext) -> ExtCiphertext:
        out = np.zeros((2, ct.nl + 1, self.n), dtype=np.uint64)
        lib().or_to_ext(self.ctx, _p64(np.ascontiguousarray(ct.data)), ct.nl, 2, _p64(out))
        return ExtCiphertext(out, ct.scale)

    def moddown(self, e: ExtCiphertext) -> Ciphertext:
        out = np.zeros((2, e.nl, self.n), dtype=np.uint64)
        lib().or_moddown(self.ctx, _p64(np.ascontiguousarray(e.data)), e.nl, 2, _p64(out))
        return Ciphertext(out, e.scale)

    def add_ext(self, a: ExtCiphertext, b: ExtCiphertext) -> ExtCiphertext:
        if a.nl != b.nl:
            raise ValueError("operands at different levels")
        out = np.zeros_like(a.data)
        lib().or_add_ext(self.ctx, _p64(np.ascontiguousarray(a.data)), _p64(np.ascontiguousarray(b.data)),
                         a.nl, 2, _p64(out))
        return ExtCiphertext(out, a.scale)

    def mac_matrix_ext(self, cts: list[ExtCiphertext], pts) -> list[np.ndarray]:
        """acc[o] = sum_t pts[o][t] * cts[t] over the extended basis
        (pts[o][t]: [nl+1][N] or None); acc[o]: [2][nl+1][N]."""
        nl = cts[0].nl
        n_ct, n_out = len(cts), len(pts)
        keep = [np.ascontiguousarray(c.data) for c in cts]
        ca = (_u64p * n_ct)(*[_p64(c) for c in keep])
        flat = []
        for o in range(n_out):
            for t in range(n_ct):
                p = pts[o][t]
                flat.append(None if p is None else np.ascontiguousarray(p))
        pa = (_u64p * len(flat))(*[(_p64(p) if p is not None else _u64p()) for p in flat])
        outs = [np.zeros((2, nl + 1, self.n), dtype=np.uint64) for _ in range(n_out)]
        oa = (_u64p * n_out)(*[_p64(o) for o in outs])
        lib().or_mac_matrix_ext(self.ctx, nl, n_ct, ca, n_out, pa, oa)
        return outs

    def add(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        assert a.nl == b.nl
        out = np.zeros_like(a.data)
        lib().or_add(self.ctx, _p64(np.ascontiguousarray(a.data)), _p64(np.ascontiguousarray(b.data)),
                     a.nl, 2, _p64(out))
        return Ciphertext(out, a.scale)

    def add_plain(self, a: Ciphertext, pt: np.ndarray) -> Ciphertext:
        out = a.data.copy()
        c0 = np.zeros_like(pt)
        lib().or_add(self.ctx, _p64(np.ascontiguousarray(a.data[0])), _p64(np.ascontiguousarray(pt)),
                     a.nl, 1, _p64(c0))
        out[0] = c0
        return Ciphertext(out, a.scale)

    def square_relin(self, ct: Ciphertext, rlk) -> Ciphertext:
        out = np.zeros_like(ct.data)
        if lib().or_square_relin(self.ctx, _p64(np.ascontiguousarray(ct.data)), ct.nl, rlk, _p64(out)) != 0:
            raise ValueError("key level")
        return Ciphertext(out, ct.scale * ct.scale)

    def mul_relin(self, a: Ciphertext, b: Ciphertext, rlk) -> Ciphertext:
        """Mul(C) + relinearisation of two ciphertexts at the same level."""
        if a.nl != b.nl:
            raise ValueError("operands at different levels")
        out = np.zeros_like(a.data)
        if lib().or_mul_relin(self.ctx, _p64(np.ascontiguousarray(a.data)), _p64(np.ascontiguousarray(b.data)),
                              a.nl, rlk, _p64(out)) != 0:
            raise ValueError("key level")
        return Ciphertext(out, a.scale * b.scale)

    def drop_level(self, ct: Ciphertext, ones: list, rlk) -> Ciphertext:
        """Drop-Level of Section IV-A as written: multiply by encryptions of
        all-ones vectors, one per level to drop, each product relinearised
        and rescaled (the all-ones ciphertext dropped to its product's level)."""
        x = ct
        for o in ones:
            x = self.rescale(self.mul_relin(x, self.limb_drop(o, x.nl), rlk))
        return x

    def rescale(self, ct: Ciphertext) -> Ciphertext:
        nl = ct.nl
        if nl < 2:
            raise ValueError("level exhausted")
        out = np.zeros((2, nl - 1, self.n), dtype=np.uint64)
        lib().or_rescale(self.ctx, _p64(np.ascontiguousarray(ct.data)), nl, 2, _p64(out))
        return Ciphertext(out, ct.scale / float(self.primes[nl - 1]))
