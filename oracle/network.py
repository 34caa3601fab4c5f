"""Oracle UniHENN network: the layer algorithms of Sections IV and VI written
out step by step, over two interchangeable evaluators:

  SlotEval -- plaintext slot vectors in FP64 (Rot = cyclic left shift,
              Mul(P) = elementwise product).  Pins the layout and planning
              against a direct FP64 CNN without any encryption.
  CkksEval -- the CPU CKKS oracle (oracle.ckks).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU-baseline leg).

Every multiplicative stage has one normal form,
    out = Rescale( sum_t Rot(X_t, r_t) * Encode(w_t * mask_t) )  [+ bias],
where a "multiply by a mask, then rotate" in the paper is computed as
"rotate, then multiply by the mask moved to the destination slots" (same
message, same rotation count).  Rotations by 0 are the identity.

Layout of a feature map (Section IV-B, VI-A): the value (c, y, x) of packed
sample b sits at slot  b*stride + ch_off[c] + I*(x + W_img*y),  with I the
interval (product of conv strides and pooling kernels so far) and W_img the
width of the original input, which every layer keeps as its row pitch.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# layout and planning
# --------------------------------------------------------------------------
@dataclass
class Layout:
    kind: str                 # "map" (C,H,W feature map) or "vec" (flat vector)
    C: int = 1
    H: int = 1
    W: int = 1
    I: int = 1                # interval
    W_img: int = 1            # row pitch
    ch_ct: list = field(default_factory=list)   # ciphertext index of channel c
    ch_off: list = field(default_factory=list)  # slot offset of channel c
    prev: str = "input"       # last non-square layer: input / conv / avgpool
    pending: float = 1.0      # deferred average-pooling factor (Section IV-C)
    length: int = 0           # vector length for kind == "vec"
    clean: bool = True        # zero on every grid slot outside the valid map (padded reads need it)
    lead: int = 0             # leading zero slots of each sample (the reserved padding space)


class PlanError(ValueError):
    pass


# degree-2 approximation of ReLU (Section V-A): f(x) = a + b x + c x^2
RELU_APPROX = (0.375373, 0.5, 0.117071)


def relu_coeffs(lay) -> tuple:
    return tuple(lay.get("coeffs", RELU_APPROX))


def kernel_hw(lay) -> tuple[int, int, int, int]:
    """(K_h, K_w, S_h, S_w): a 1D convolution has a 1 x K kernel."""
    if lay.get("dims") == 1:
        return 1, lay["k"], 1, lay["s"]
    return lay["k"], lay["k"], lay["s"], lay["s"]


def pad_hw(lay) -> tuple[int, int]:
    """(P_h, P_w) zero padding of a convolution (a 1D one pads its width)."""
    p = lay.get("pad", 0)
    return (0, p) if lay.get("dims") == 1 else (p, p)


def conv_out(H: int, W: int, lay) -> tuple[int, int]:
    Kh, K, Sh, S = kernel_hw(lay)
    Ph, Pw = pad_hw(lay)
    return (H + 2 * Ph - Kh) // Sh + 1, (W + 2 * Pw - K) // S + 1


def input_layout(inp: dict, channel_cts: bool = False) -> Layout:
    """Sample layout: `lead` zero slots (the space Section VI reserves for
    padding), then the rows at pitch W_img = inp["pitch"] (default W; the
    extra columns are zero); channels row-major at offset c*H*W_img
    (Section III-A), or one ciphertext per channel at offset lead."""
    C, H, W = inp["c"], inp["h"], inp["w"]
    Wp, lead = inp.get("pitch", W), inp.get("lead", 0)
    if Wp < W or lead < 0:
        raise PlanError("row pitch below the width or negative lead")
    if channel_cts:
        return Layout("map", C, H, W, 1, Wp, list(range(C)), [lead] * C, "input", 1.0, lead=lead)
    return Layout("map", C, H, W, 1, Wp, [0] * C, [lead + c * H * Wp for c in range(C)], "input", 1.0, lead=lead)


def check_padded_read(L: Layout, lay) -> None:
    """A padded convolution reads up to P_h rows above, P_w columns beside and
    P_h rows below the map.  Those slots must hold zeros: the map is clean,
    every channel has its own ciphertext (or there is one channel), the row
    pitch leaves P_w zero columns (a read left of column 0 lands in the
    previous row's right margin), and the sample's lead holds the rows above
    (I (P_h W_img + P_w) slots)."""
    Ph, Pw = pad_hw(lay)
    if not Ph and not Pw:
        return
    if not L.clean:
        raise PlanError("padded convolution of a pooled map (partial sums lie where the padding reads)")
    if L.C > 1 and len(set(L.ch_ct)) != L.C:
        raise PlanError("padded convolution needs one ciphertext per input channel")
    if L.W_img - L.W < Pw:
        raise PlanError("row pitch leaves fewer zero columns than the padding")
    if L.lead < L.I * (Ph * L.W_img + Pw):
        raise PlanError("leading space below the padding's rows")


def footprint(inp: dict, layers, channel_cts: bool = False) -> int:
    """Slots each packed sample needs (Section VI): the largest extent, over
    all layers, of the slots that hold the sample's valid values or that a
    valid output reads; the flatten output C*H*W; the FC width
    DAT_out * ceil(DAT_in / DAT_out).  With channel_cts each input channel
    sits in its own ciphertext (H*W slots)."""
    L = input_layout(inp, channel_cts)
    need = L.lead + (1 if channel_cts else inp["c"]) * inp["h"] * L.W_img
    for lay in layers:
        k = lay["kind"]
        if k == "conv":
            Kh, K, Sh, S = kernel_hw(lay)
            Ph, Pw = pad_hw(lay)
            if not K >= S >= 1:
                raise PlanError("Theorem 1 needs K >= S >= 1")
            Ho, Wo = conv_out(L.H, L.W, lay)
            # last slot read by a valid output
            read = max(L.ch_off) + L.I * ((S * (Wo - 1) + K - 1 - Pw) + L.W_img * (Sh * (Ho - 1) + Kh - 1 - Ph)) + 1
            need = max(need, read)
            I = L.I * S
            L = Layout("map", lay["ch_out"], Ho, Wo, I, L.W_img, list(range(lay["ch_out"])),
                       [L.lead] * lay["ch_out"], "conv", 1.0, lead=L.lead)
            need = max(need, L.lead + I * ((Wo - 1) + L.W_img * (Ho - 1)) + 1)
        elif k == "avgpool":
            c = lay["c"]
            read = max(L.ch_off) + L.I * ((c * (L.W // c) - 1) + L.W_img * (c * (L.H // c) - 1)) + 1
            need = max(need, read)
            L = Layout("map", L.C, L.H // c, L.W // c, L.I * c, L.W_img, L.ch_ct, L.ch_off, "avgpool", 1.0,
                       lead=L.lead)
        elif k == "flatten":
            need = max(need, L.C * L.H * L.W)
            L = Layout("vec", length=L.C * L.H * L.W)
        elif k == "fc":
            D = lay["dout"]
            need = max(need, D * math.ceil(lay["din"] / D))
            L = Layout("vec", length=D)
    return need


def check_packing(inp: dict, layers, n_slots: int, samples: int, stride: int, channel_cts: bool = False) -> int:
    fp = footprint(inp, layers, channel_cts)
    if samples == 1:
        if fp > n_slots:
            raise PlanError("model does not fit the slots")
        return n_slots
    if stride < fp or samples * stride > n_slots:
        raise PlanError(f"stride {stride} < footprint {fp} or {samples} samples exceed {n_slots} slots")
    return stride


def shapes(inp: dict, layers):
    """(C,H,W) or (len,) after each layer."""
    C, H, W = inp["c"], inp["h"], inp["w"]
    out = []
    flat = None
    for lay in layers:
        k = lay["kind"]
        if k == "conv":
            C = lay["ch_out"]
            H, W = conv_out(H, W, lay)
        elif k == "avgpool":
            H, W = H // lay["c"], W // lay["c"]
        elif k == "flatten":
            flat = C * H * W
        elif k == "fc":
            flat = lay["dout"]
        out.append((C, H, W) if flat is None else (flat,))
    return out


def network_depth(inp: dict, layers) -> int:
    d = 0
    prev, I, pending = "input", 1, 1.0
    H, W = inp["h"], inp["w"]
    for lay in layers:
        k = lay["kind"]
        if k == "conv":
            d += 1
            Kh, K, Sh, S = kernel_hw(lay)
            prev, I, pending = "conv", I * S, 1.0
            H, W = conv_out(H, W, lay)
        elif k == "square":
            d += 1
            pending *= pending
        elif k == "relu_approx":
            d += 2
            prev, pending = "relu", 1.0
        elif k == "avgpool":
            prev, I = "avgpool", I * lay["c"]
            pending /= lay["c"] ** 2
            H, W = H // lay["c"], W // lay["c"]
        elif k == "flatten":
            d += int(prev == "avgpool" or (I > 1 and W > 1) or pending != 1.0)
            d += int(H > 1)
        elif k == "fc":
            d += 1
    return d


# --------------------------------------------------------------------------
# FP64 reference CNN (valid convolutions, no padding)
# --------------------------------------------------------------------------
def cnn_fp64(x: np.ndarray, layers, params) -> np.ndarray:
    """Direct FP64 forward pass of one input x of shape (C, H, W)."""
    a = np.asarray(x, dtype=np.float64)
    for lay, p in zip(layers, params):
        k = lay["kind"]
        if k == "conv":
            w, b = p
            Kh, K, Sh, S = kernel_hw(lay)
            Ph, Pw = pad_hw(lay)
            a = np.pad(a, ((0, 0), (Ph, Ph), (Pw, Pw)))
            C, H, W = a.shape
            Ho, Wo = (H - Kh) // Sh + 1, (W - K) // S + 1
            out = np.zeros((w.shape[0], Ho, Wo))
            for o in range(w.shape[0]):
                for y in range(Ho):
                    for xx in range(Wo):
                        out[o, y, xx] = np.sum(w[o] * a[:, Sh * y:Sh * y + Kh, S * xx:S * xx + K]) + b[o]
            a = out
        elif k == "square":
            a = a * a
        elif k == "relu_approx":
            ca, cb, cc = relu_coeffs(lay)
            a = ca + cb * a + cc * a * a
        elif k == "avgpool":
            c = lay["c"]
            C, H, W = a.shape
            Ho, Wo = H // c, W // c
            a = a[:, :Ho * c, :Wo * c].reshape(C, Ho, c, Wo, c).mean(axis=(2, 4))
        elif k == "flatten":
            a = a.reshape(-1)
        elif k == "fc":
            w, b = p
            a = w @ a.reshape(-1) + b
    return a


# --------------------------------------------------------------------------
# evaluators
# --------------------------------------------------------------------------
class OpCount:
    def __init__(self):
        self.rot = 0
        self.mac = 0
        self.rescale = 0
        self.relin = 0

    def as_dict(self):
        return {"rot": self.rot, "mac": self.mac, "rescale": self.rescale, "relin": self.relin}


class SlotEval:
    """FP64 slot vectors; masks and weights applied exactly, no rescale."""

    def __init__(self, n_slots: int):
        self.n_slots = n_slots
        self.count = OpCount()

    def rot(self, x, r):
        if r % self.n_slots == 0:
            return x
        self.count.rot += 1
        return np.roll(x, -r)

    def mac_rescale(self, srcs, terms_per_out):
        """terms_per_out[o] = list of (src_index, weight, mask_vector)."""
        outs = []
        for terms in terms_per_out:
            acc = np.zeros(self.n_slots)
            for t, w, m in terms:
                acc = acc + srcs[t] * (w * m)
                self.count.mac += 1
            self.count.rescale += 1
            outs.append(acc)
        return outs

    def add_plain(self, x, vec):
        return x + vec

    def add(self, a, b):
        return a + b

    def square(self, x):
        self.count.relin += 1
        self.count.rescale += 1
        return x * x

    def mul(self, a, b):
        self.count.relin += 1
        self.count.rescale += 1
        return a * b

    def drop_to(self, x, like):
        return x

    def finish(self, x):
        return x


class CkksEval:
    """The CPU CKKS oracle.  keys: {r mod N/2: loaded key}, rlk: loaded key."""

    def __init__(self, ck, keys: dict, rlk):
        self.ck = ck
        self.n_slots = ck.slots
        self.keys = keys
        self.rlk = rlk
        self.count = OpCount()

    def rot(self, x, r):
        r = r % self.n_slots
        if r == 0:
            return x
        if r not in self.keys:
            raise KeyError(f"no rotation key for {r}")
        self.count.rot += 1
        return self.ck.rotate(x, r, self.keys[r])

    def mac_rescale(self, srcs, terms_per_out):
        return self._mac_rescale(srcs, terms_per_out, ext=False)

    def _mac_rescale(self, srcs, terms_per_out, ext: bool):
        """Rescale(sum_t Encode(w_t m_t) * srcs[t]) per output; with ext the
        sources are extended ciphertexts, the plaintexts carry their residue
        mod P, and each sum is brought down by one ModDown before the rescale."""
        from oracle.ckks import Ciphertext, ExtCiphertext
        ck = self.ck
        nl = srcs[0].nl
        scale = srcs[0].scale
        for s in srcs:
            if s.nl != nl or s.scale != scale:
                raise ValueError("MAC terms must share level and scale")
        encode = ck.encode_scaled_ext if ext else ck.encode_scaled
        outs = []
        chunk = 4
        for o0 in range(0, len(terms_per_out), chunk):
            block = terms_per_out[o0:o0 + chunk]
            pts = []
            for terms in block:
                row = [None] * len(srcs)
                # group this output's terms by mask so each mask is transformed once
                bymask = {}
                for t, w, m in terms:
                    bymask.setdefault(id(m), (m, []))[1].append((t, w))
                for _, (m, tw) in bymask.items():
                    enc = encode(m, [w for _, w in tw], ck.delta, nl)
                    for (t, _), p in zip(tw, enc):
                        if row[t] is not None:
                            raise ValueError("duplicate term")
                        row[t] = p
                self.count.mac += len(terms)
                pts.append(row)
            if ext:
                accs = [ck.moddown(ExtCiphertext(a, scale * ck.delta)).data for a in ck.mac_matrix_ext(srcs, pts)]
            else:
                accs = ck.mac_matrix(srcs, pts)
            for a in accs:
                self.count.rescale += 1
                outs.append(ck.rescale(Ciphertext(a, scale * ck.delta)))
        return outs

    def add_plain(self, x, vec):
        pt = self.ck.encode(vec, x.scale, x.nl)
        return self.ck.add_plain(x, pt)

    def add(self, a, b):
        return self.ck.add(a, b)

    def square(self, x):
        self.count.relin += 1
        self.count.rescale += 1
        return self.ck.rescale(self.ck.square_relin(x, self.rlk))

    def mul(self, a, b):
        self.count.relin += 1
        self.count.rescale += 1
        return self.ck.rescale(self.ck.mul_relin(a, b, self.rlk))

    def drop_to(self, x, like):
        """x with its top limbs discarded down to like's level (scale kept)."""
        return self.ck.limb_drop(x, like.nl)

    def finish(self, x):
        return x


class LazyCkksEval(CkksEval):
    """CkksEval with the ModDown of rotations deferred (an evaluator variant
    of this implementation; the paper's evaluator is the one above).

    A rotation by r != 0 yields its extended form (P tau(c0) + U_0, U_1) over
    {q_0..q_{nl-1}, P} (oracle.ckks.ExtCiphertext); a rotation by 0 returns
    its input unchanged.  Additions and plaintext sums with an extended
    operand stay extended (a plain ciphertext x enters as P x), and a sum of
    products is brought down by a single ModDown before its rescale.  Any
    other use of an extended value (a rotation source, a plaintext addition,
    a product, the network output) first takes its ModDown, once per value.
    Every sum is exact modulo each prime, so the result depends only on which
    sums are brought down, not on the order of their terms."""

    def _norm(self, x):
        from oracle.ckks import ExtCiphertext
        if not isinstance(x, ExtCiphertext):
            return x
        md = getattr(x, "_md", None)
        if md is None:
            md = self.ck.moddown(x)
            x._md = md
        return md

    def _ext(self, x):
        from oracle.ckks import ExtCiphertext
        return x if isinstance(x, ExtCiphertext) else self.ck.to_ext(x)

    @staticmethod
    def _is_ext(x) -> bool:
        from oracle.ckks import ExtCiphertext
        return isinstance(x, ExtCiphertext)

    def rot(self, x, r):
        r = r % self.n_slots
        if r == 0:
            return x
        if r not in self.keys:
            raise KeyError(f"no rotation key for {r}")
        self.count.rot += 1
        return self.ck.rotate_ext(self._norm(x), r, self.keys[r])

    def add(self, a, b):
        if self._is_ext(a) or self._is_ext(b):
            return self.ck.add_ext(self._ext(a), self._ext(b))
        return self.ck.add(a, b)

    def mac_rescale(self, srcs, terms_per_out):
        if any(self._is_ext(s) for s in srcs):
            return self._mac_rescale([self._ext(s) for s in srcs], terms_per_out, ext=True)
        return self._mac_rescale(srcs, terms_per_out, ext=False)

    def add_plain(self, x, vec):
        return super().add_plain(self._norm(x), vec)

    def square(self, x):
        return super().square(self._norm(x))

    def mul(self, a, b):
        return super().mul(self._norm(a), self._norm(b))

    def drop_to(self, x, like):
        return super().drop_to(self._norm(x), like)

    def finish(self, x):
        return self._norm(x)


# --------------------------------------------------------------------------
# the layers
# --------------------------------------------------------------------------
class Net:
    """Plan + evaluation of a UniHENN network on one ciphertext of packed
    samples (or one FP64 slot vector)."""

    def __init__(self, inp: dict, layers, params, n_slots: int, samples: int = 1, stride: int = 0,
                 fc_doubling: bool = False, channel_cts: bool = False):
        """fc_doubling: Algorithm 2's closing sum of ceil(DAT_in / DAT_out)
        rotated copies by doubling (a variant of this implementation, see
        _rotate_sum) instead of one rotation per copy.  channel_cts: the input
        arrives as one ciphertext per channel (for inputs whose C*H*W
        exceeds a sample's slots); run() then takes C input ciphertexts."""
        self.inp = inp
        self.layers = layers
        self.params = params
        self.fc_doubling = fc_doubling
        self.channel_cts = channel_cts
        self.n_slots = n_slots
        self.samples = samples
        self.stride = check_packing(inp, layers, n_slots, samples, stride if samples > 1 else n_slots, channel_cts)
        self.depth = network_depth(inp, layers)

    # slot vector helper: ones at the given in-sample positions of every sample
    def _mask(self, positions) -> np.ndarray:
        m = np.zeros(self.n_slots)
        pos = np.asarray(sorted(set(int(p) for p in positions)), dtype=np.int64)
        for b in range(self.samples):
            m[b * self.stride + pos] = 1.0
        return m

    def _vec(self, values_at: dict) -> np.ndarray:
        v = np.zeros(self.n_slots)
        for b in range(self.samples):
            for p, val in values_at.items():
                v[b * self.stride + p] = val
        return v

    def input_vector(self, xs: np.ndarray) -> np.ndarray:
        """Client-side packing (Section III-B): sample b's (C,H,W) data at
        slot b*stride + lead, channel c's rows at pitch W_img from
        lead + c*H*W_img (row-major when there is no lead or extra pitch)."""
        L = input_layout(self.inp)
        v = np.zeros(self.n_slots)
        for b, x in enumerate(xs):
            a = np.asarray(x, dtype=np.float64)
            for c in range(a.shape[0]):
                for y in range(a.shape[1]):
                    base = b * self.stride + L.ch_off[c] + y * L.W_img
                    v[base: base + a.shape[2]] = a[c, y]
        return v

    def input_vectors(self, xs: np.ndarray) -> list:
        """The network's input slot vectors: [input_vector(xs)], or with
        channel_cts one vector per channel c holding sample b's (H,W) plane
        of channel c at slot b*stride."""
        if not self.channel_cts:
            return [self.input_vector(xs)]
        L = input_layout(self.inp, True)
        vs = []
        for c in range(self.inp["c"]):
            v = np.zeros(self.n_slots)
            for b, x in enumerate(xs):
                a = np.asarray(x, dtype=np.float64)[c]
                for y in range(a.shape[0]):
                    base = b * self.stride + L.lead + y * L.W_img
                    v[base: base + a.shape[1]] = a[y]
            vs.append(v)
        return vs

    def rotation_set(self) -> list[int]:
        """Distinct non-zero rotation amounts (mod N/2) the evaluation uses."""
        rec = _RotRecorder(self.n_slots)
        self.run(rec, [np.zeros(self.n_slots)] * (self.inp["c"] if self.channel_cts else 1))
        return sorted(rec.seen)

    def run(self, ev, cts):
        L = input_layout(self.inp, self.channel_cts)
        xs = list(cts)
        for lay, p in zip(self.layers, self.params):
            k = lay["kind"]
            if k == "conv":
                xs, L = self._conv(ev, xs, L, lay, p)
            elif k == "square":
                xs = [ev.square(x) for x in xs]
                L.pending = L.pending * L.pending
            elif k == "relu_approx":
                xs, L = self._relu(ev, xs, L, lay)
            elif k == "avgpool":
                xs, L = self._avgpool(ev, xs, L, lay)
            elif k == "flatten":
                xs, L = self._flatten(ev, xs, L)
            elif k == "fc":
                xs, L = self._fc(ev, xs, L, lay, p)
            else:
                raise PlanError(k)
        self.out_layout = L
        return [ev.finish(x) for x in xs]

    # Algorithm 1 ----------------------------------------------------------
    def _conv(self, ev, xs, L, lay, p):
        """Output (y, x) sits at lead + I_out (x + W_img y); its term (i, j, k)
        reads input (S_h y + j - P_h, S x + k - P_w) of channel i, whose slot
        is ch_off[i] + I (...), so the rotation amount is
        ch_off[i] - lead + I ((k - P_w) + W_img (j - P_h)).  Unpadded and
        with lead 0 this is Algorithm 1's I (k + W_img j) plus the channel
        offset."""
        w, b = p
        Kh, K, Sh, S = kernel_hw(lay)
        Ph, Pw = pad_hw(lay)
        ci, co = lay["ch_in"], lay["ch_out"]
        if ci != L.C:
            raise PlanError("channel mismatch")
        if not K >= S >= 1:
            raise PlanError("Theorem 1 needs K >= S >= 1")
        check_padded_read(L, lay)
        Ho, Wo = conv_out(L.H, L.W, lay)
        I_out = L.I * S
        # first loop: C_rot(i,j,k) = Rot(C_in(i), I_in (k + W_img j)) (+ channel offset)
        rots, src_index = [], {}
        amount = lambda i, j, kk: L.ch_off[i] - L.lead + L.I * ((kk - Pw) + L.W_img * (j - Ph))
        for i in range(ci):
            for j in range(Kh):
                for kk in range(K):
                    key = (L.ch_ct[i], amount(i, j, kk))
                    if key not in src_index:
                        src_index[key] = len(rots)
                        rots.append(ev.rot(xs[key[0]], key[1]))
        # structured kernel vector: the weight on the valid output slots
        m_out = self._mask([L.lead + I_out * (x + L.W_img * y) for y in range(Ho) for x in range(Wo)])
        wp = w * L.pending
        terms = []
        for o in range(co):
            t = []
            for i in range(ci):
                for j in range(Kh):
                    for kk in range(K):
                        key = (L.ch_ct[i], amount(i, j, kk))
                        t.append((src_index[key], float(wp[o, i, j, kk]), m_out))
            terms.append(t)
        outs = ev.mac_rescale(rots, terms)
        outs = [ev.add_plain(outs[o], float(b[o]) * m_out) for o in range(co)]
        L2 = Layout("map", co, Ho, Wo, I_out, L.W_img, list(range(co)), [L.lead] * co, "conv", 1.0, lead=L.lead)
        return outs, L2

    def _valid_positions(self, L, ct: int) -> list:
        """In-sample slots of the valid values that ciphertext `ct` holds."""
        if L.kind == "vec":
            return list(range(L.length))
        pos = []
        for c in range(L.C):
            if L.ch_ct[c] == ct:
                pos.extend(L.ch_off[c] + L.I * (x + L.W_img * y) for y in range(L.H) for x in range(L.W))
        return pos

    # Section V-A: f(x) = a + b x + c x^2, as x (c x + b) + a ----------------
    def _relu(self, ev, xs, L, lay):
        """Two levels: Y = Rescale(X * Encode(c' M)) + b' M, then
        Z = Rescale(Relin(Y * X)) + a M, X dropped to Y's level, with M the
        valid slots.  A pending pooling factor p folds into the coefficients
        (c' = c p^2, b' = b p: f applied to the average, Section IV-C).  Zero
        outside M."""
        ca, cb, cc = relu_coeffs(lay)
        p = L.pending
        outs = []
        for i, X in enumerate(xs):
            M = self._mask(self._valid_positions(L, i))
            Y = ev.mac_rescale([X], [[(0, cc * p * p, M)]])[0]
            Y = ev.add_plain(Y, (cb * p) * M)
            Z = ev.mul(Y, ev.drop_to(X, Y))
            outs.append(ev.add_plain(Z, ca * M))
        L2 = Layout(L.kind, L.C, L.H, L.W, L.I, L.W_img, L.ch_ct, L.ch_off, "relu", 1.0, L.length, lead=L.lead)
        return outs, L2

    # Section IV-C -----------------------------------------------------------
    def _avgpool(self, ev, xs, L, lay):
        c = lay["c"]
        amounts = [L.I * (dx + L.W_img * dy) for dy in range(c) for dx in range(c)]
        outs = []
        for x in xs:
            acc = None
            for r in amounts:
                t = ev.rot(x, r)
                acc = t if acc is None else ev.add(acc, t)
            outs.append(acc)
        # the sums leave partial sums on slots around the pooled grid (and on
        # grid slots past its width, which alias other rows): not clean
        L2 = Layout("map", L.C, L.H // c, L.W // c, L.I * c, L.W_img, L.ch_ct, L.ch_off, "avgpool",
                    L.pending / (c * c), clean=False, lead=L.lead)
        return outs, L2

    # Section IV-E -----------------------------------------------------------
    def _flatten(self, ev, xs, L):
        """The channels sit at the sample's lead; the first stage that rotates
        (A, B or the packing) also moves them down by lead, so every mask is
        the one of a map at offset 0."""
        if len(set(L.ch_ct)) != L.C or any(off != L.lead for off in L.ch_off):
            raise PlanError("flatten expects one ciphertext per channel")
        S, Wi, Hi, Wimg = L.I, L.W, L.H, L.W_img
        ys = list(xs)
        sh = L.lead
        # step A: remove the row interval / invalid data
        if L.prev == "avgpool":
            # term x: Rot(X, x(S-1)) * (pending at slot S W_img y + x)
            rots_all = [[ev.rot(X, sh + x * (S - 1)) for x in range(Wi)] for X in ys]
            sh = 0
            masks = [self._mask([S * Wimg * y + x for y in range(Hi)]) for x in range(Wi)]
            ys = []
            for R in rots_all:
                ys.extend(ev.mac_rescale(R, [[(x, L.pending, masks[x]) for x in range(Wi)]]))
        elif S > 1 and Wi > 1:
            G = math.ceil(Wi / S)
            masks = [self._mask([S * Wimg * y + g * S + m for y in range(Hi) for m in range(S) if g * S + m < Wi])
                     for g in range(G)]
            out = []
            for X in ys:
                T = None
                for m in range(S):
                    t = ev.rot(X, sh + m * (S - 1))
                    T = t if T is None else ev.add(T, t)
                R = [ev.rot(T, g * S * (S - 1)) for g in range(G)]
                out.extend(ev.mac_rescale(R, [[(g, L.pending, masks[g]) for g in range(G)]]))
            ys = out
            sh = 0
        elif L.pending != 1.0:
            m = self._mask([Wimg * y + x for y in range(Hi) for x in range(Wi)])
            ys = [ev.mac_rescale([ev.rot(X, sh)], [[(0, L.pending, m)]])[0] for X in ys]
            sh = 0
        # now (y, x) sits at S W_img y + x
        # step B: remove the column interval
        if Hi > 1:
            masks = [self._mask([y * Wi + x for x in range(Wi)]) for y in range(Hi)]
            out = []
            for X in ys:
                R = [ev.rot(X, sh + y * (Wimg * S - Wi)) for y in range(Hi)]
                out.extend(ev.mac_rescale(R, [[(y, 1.0, masks[y]) for y in range(Hi)]]))
            ys = out
            sh = 0
        # step C: pack channel o at o * H * W (right rotation)
        acc = None
        for o, X in enumerate(ys):
            t = ev.rot(X, sh - o * Wi * Hi)
            acc = t if acc is None else ev.add(acc, t)
        return [acc], Layout("vec", length=L.C * Hi * Wi)

    # Algorithm 2 -------------------------------------------------------------
    def _fc(self, ev, xs, L, lay, p):
        w, b = p
        din, D = lay["din"], lay["dout"]
        if L.kind != "vec" or L.length != din:
            raise PlanError("FC input size mismatch")
        wp = w * L.pending
        Wvec = D * math.ceil(din / D)
        X = xs[0]
        srcs, terms = [], []
        for o in range(D):
            mrot = np.zeros(Wvec)
            for q in range(Wvec):
                col = (q + o) % Wvec
                mrot[q] = wp[q % D, col] if col < din else 0.0
            v1 = self._vec({q: mrot[q] for q in range(Wvec - o)})
            srcs.append(ev.rot(X, o))
            terms.append((len(srcs) - 1, 1.0, v1))
            if o >= 1:
                v2 = self._vec({q: mrot[q] for q in range(Wvec - o, Wvec)})
                srcs.append(ev.rot(X, o - Wvec))
                terms.append((len(srcs) - 1, 1.0, v2))
        csum = ev.mac_rescale(srcs, [terms])[0]
        reps = math.ceil(din / D)
        if self.fc_doubling:
            acc = self._rotate_sum(ev, csum, reps, D)
        else:
            acc = None
            for i in range(reps):
                t = ev.rot(csum, i * D)
                acc = t if acc is None else ev.add(acc, t)
        acc = ev.add_plain(acc, self._vec({q: float(b[q]) for q in range(D)}))
        return [acc], Layout("vec", length=D)

    @staticmethod
    def _rotate_sum(ev, x, reps: int, step: int):
        """sum_{i < reps} Rot(x, i step) by doubling: S_1 = x and
        S_2m = S_m + Rot(S_m, m step) give S_m = sum_{i < m} Rot(x, i step)
        for powers of two m <= reps; the result adds, for each set bit 2^b
        of reps from the highest down, Rot(S_(2^b), o step), o the sum of the
        bits above it.  floor(log2 reps) + popcount(reps) - 1 rotations
        instead of reps - 1; equal slot by slot (rotations are linear), not
        bit for bit, since each rotation rounds its own key switch."""
        S = {1: x}
        m = 1
        while 2 * m <= reps:
            S[2 * m] = ev.add(S[m], ev.rot(S[m], m * step))
            m *= 2
        acc, off = None, 0
        for bit in reversed(range(reps.bit_length())):
            if reps >> bit & 1:
                t = ev.rot(S[1 << bit], off * step)
                acc = t if acc is None else ev.add(acc, t)
                off += 1 << bit
        return acc

    # read-out -----------------------------------------------------------------
    def output_positions(self) -> list[list[int]]:
        """Per sample, the slots of the network output in FP64-CNN order."""
        L = self.out_layout
        res = []
        for b in range(self.samples):
            base = b * self.stride
            if L.kind == "vec":
                res.append([base + q for q in range(L.length)])
            else:
                pos = []
                for c in range(L.C):
                    for y in range(L.H):
                        for x in range(L.W):
                            pos.append((c, base + L.ch_off[c] + L.I * (x + L.W_img * y)))
                res.append(pos)
        return res


class _RotRecorder(SlotEval):
    def __init__(self, n_slots):
        super().__init__(n_slots)
        self.seen = set()

    def rot(self, x, r):
        r = r % self.n_slots
        if r:
            self.seen.add(r)
        return super().rot(x, r)


def read_outputs(net: Net, values_per_ct: list) -> np.ndarray:
    """Gather network outputs from decoded slot vectors (one per output
    ciphertext) into [samples][...] FP64-CNN order."""
    L = net.out_layout
    pos = net.output_positions()
    out = []
    for b in range(net.samples):
        if L.kind == "vec":
            out.append(np.array([values_per_ct[0][p] for p in pos[b]]))
        else:
            out.append(np.array([values_per_ct[L.ch_ct[c]][p] for c, p in pos[b]]))
    return np.array(out)
