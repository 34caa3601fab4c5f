// UniHENN network: planning on the host, then a straight-line program of
// rotations, multiply-accumulates, rescales, additions and squares executed
// on one stream.
//
// Layout of a feature map (Sections III-A, IV-B, VI-A): the value (c, y, x)
// of packed sample b sits at slot  b*stride + ch_off[c] + I*(x + W_img*y),
// with I the product of the conv strides and pooling kernels so far and W_img
// the width of the input, kept as the row pitch by every layer.
//
// Every multiplicative stage is  Rescale( sum_t Rot(X_t, r_t) * pt_t ), where
// pt_t = Encode(w_t * mask_t) puts the scalar on the destination slots.  The
// paper's "multiply by a mask, then rotate" steps of the flatten layer are
// computed as "rotate, then multiply by the mask moved to the destination":
// the message and the rotation count are the same, and all rotations of one
// source become consecutive, so they can share one digit decomposition.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "kernels.h"

int encode_scaled_batch(const unihenn_ctx* c, const double* z, int n_slots, const double* w, int n_w, double scale,
                        int nl, int mont, u64* out, hipStream_t s, int ext);

namespace {

enum StepKind {
    ST_DROP, ST_ROT, ST_MAC, ST_MACM, ST_RESCALE, ST_ADD, ST_ADD_PLAIN, ST_SQUARE, ST_MUL, ST_EXT, ST_MODDOWN, ST_SUM
};

// A register holds a batch of ciphertexts at level nl; an extended register
// (deferred ModDown) holds them over {q_0..q_{nl-1}, P}, one limb more, and
// stands for their ModDown.
struct VReg {
    int nl;
    double scale;
    int phys = -1;
    bool ext = false;
    int limbs() const { return nl + (ext ? 1 : 0); }
};

struct Term {
    int src;
    size_t pt;  // word offset of the plaintext in the arena
};

struct Step {
    StepKind kind;
    int dst = -1, a = -1, b = -1;
    int rot = 0;
    bool acc = false;
    std::vector<Term> terms;
    size_t pt = 0;
    // ST_MACM: outs[o] (+)= sum_t pt(o, t) (*) srcs[t], pt(o, t) at pt + (o * pt_ostride + pt_toff + t) * nl * N
    std::vector<int> outs, srcs;
    int pt_ostride = 0, pt_toff = 0;
    int in_idx = 0;  // ST_DROP: which network input
};

struct PtRequest {
    std::vector<double> z;
    std::vector<double> w;
    double scale;
    int nl;
    int mont;
    size_t offset;
    int ext;  // residue mod P as limb nl (plaintexts of extended products)
};

struct LayerRecord {
    int kind;
    size_t step_begin, step_end;
    std::vector<int> in_regs, out_regs;
    int interval_out = 0;
};

struct Layout {
    bool vec = false;
    int C = 1, H = 1, W = 1, I = 1, W_img = 1;
    std::vector<int> ch_reg, ch_off;  // register and slot offset of channel c
    int prev = 0;                      // 0 input, 1 conv, 2 avgpool, 3 approximate ReLU (last non-square layer)
    double pending = 1.0;              // deferred pooling factor (Section IV-C)
    int length = 0;
    bool clean = true;                 // zero on every slot off the valid map (padded reads need it)
    int lead = 0;                      // leading zero slots of each sample (the reserved padding space)
};

struct KernelGeom {
    int kh, kw, sh, sw, ph, pw;  // kernel, stride and zero padding (height, width)
};

// Largest total size of the rotated batches of one convolution kept live at
// once so that every output is one sum over all its terms.
constexpr size_t kOneSumBytes = (size_t)24 << 30;

KernelGeom geom(const unihenn_layer& L)
{
    if (L.dims == 1) return {1, (int)L.k, 1, (int)L.s, 0, (int)L.pad};
    return {(int)L.k, (int)L.k, (int)L.s, (int)L.s, (int)L.pad, (int)L.pad};
}

}  // namespace

struct unihenn_net {
    const unihenn_ctx* ctx = nullptr;
    int n_slots = 0, samples = 1, stride = 0, depth = 0, in_limbs = 0, max_batch = 1;
    std::vector<VReg> regs;
    std::vector<Step> steps;
    std::vector<LayerRecord> layers;
    std::vector<int> rotations;
    std::vector<int> out_regs;
    std::vector<uint64_t> out_slots;
    int n_values = 0;
    int input_reg = -1;
    int n_inputs = 1;  // input ciphertexts per evaluation (C with UNIHENN_PLAN_CHANNEL_CTS)
    std::vector<PtRequest> requests;
    size_t pt_words = 0;
    // device
    u64* pt_arena = nullptr;
    u64* reg_arena = nullptr;
    std::vector<size_t> phys_off;
    u64* ws = nullptr;
    int ws_nl = 0;
    int group_max = 1;       // rotations per grouped key-switch launch set (in use)
    int group_alloc = 1;     // group size the workspace layout holds
    size_t ws_words = 0;
    std::map<int, const u64*> keys;
    const u64* rlk = nullptr;
    int mode = UNIHENN_EVAL_PLAIN;
    bool lazy = false;  // planned with deferred ModDown (UNIHENN_PLAN_LAZY_MODDOWN)
    // captured evaluations (UNIHENN_EVAL_GRAPH), one per batch size and buffer set
    hipStream_t gstream = nullptr;  // capture only
    struct GraphEntry {
        int batch = 0, in_limbs = 0, mode = -1;
        int stage = -1, slot = 0;  // layer stages (unihenn_eval_stage); -1: whole evaluation
        std::vector<const u64*> in;
        std::vector<u64*> outs;
        size_t key_version = 0;
        hipGraphExec_t exec = nullptr;
        unsigned long long last_use = 0;
    };
    std::vector<GraphEntry> graphs;
    std::vector<GraphEntry> stage_graphs;
    unsigned long long graph_clock = 0;
    size_t key_version = 0;
};

namespace {

// ---------------------------------------------------------------- planning
struct Planner {
    unihenn_net* net;
    const unihenn_ctx* c;
    double delta;
    std::map<int, int> rotset;
    std::string err;
    int err_code = 0;
    // deferred ModDown: rotations by r != 0 give extended registers; sums
    // and plaintext products of extended registers stay extended and are
    // brought down once, before their rescale; every other use of an
    // extended register takes its ModDown first (once per register)
    bool lazy = false;
    bool fc_doubling = false;  // Algorithm 2's closing sum by doubling (UNIHENN_PLAN_FC_DOUBLING)
    std::map<int, int> md_of, ext_of;
    std::map<size_t, int> pt_ext;  // plaintext offset -> has the P limb

    int fail(int code, const std::string& m)
    {
        if (!err_code) { err_code = code; err = m; }
        return -1;
    }

    int newreg(int nl, double scale, bool ext = false)
    {
        VReg r;
        r.nl = nl;
        r.scale = scale;
        r.ext = ext;
        net->regs.push_back(r);
        return (int)net->regs.size() - 1;
    }

    bool is_ext(int r) const { return r >= 0 && net->regs[r].ext; }

    // the register in normal form: an extended one is brought down (once)
    int norm(int r)
    {
        if (!is_ext(r)) return r;
        auto it = md_of.find(r);
        if (it != md_of.end()) return it->second;
        const VReg v = net->regs[r];
        int d = newreg(v.nl, v.scale);
        Step s;
        s.kind = ST_MODDOWN;
        s.dst = d;
        s.a = r;
        net->steps.push_back(s);
        md_of[r] = d;
        return d;
    }

    // the register in extended form: a normal one enters as P x (once)
    int to_ext(int r)
    {
        if (is_ext(r)) return r;
        auto it = ext_of.find(r);
        if (it != ext_of.end()) return it->second;
        const VReg v = net->regs[r];
        int d = newreg(v.nl, v.scale, true);
        Step s;
        s.kind = ST_EXT;
        s.dst = d;
        s.a = r;
        net->steps.push_back(s);
        ext_of[r] = d;
        return d;
    }

    int norm_rot(long r) const
    {
        long h = net->n_slots;
        return (int)(((r % h) + h) % h);
    }

    int rot(int src, long r)
    {
        int rr = norm_rot(r);
        if (rr == 0) return src;
        src = norm(src);
        int d = newreg(net->regs[src].nl, net->regs[src].scale, lazy);
        Step s;
        s.kind = ST_ROT;
        s.dst = d;
        s.a = src;
        s.rot = rr;
        net->steps.push_back(s);
        rotset[rr] = 1;
        return d;
    }

    int add(int a, int b)
    {
        if (is_ext(a) || is_ext(b)) {
            a = to_ext(a);
            b = to_ext(b);
        }
        if (net->regs[a].nl != net->regs[b].nl || net->regs[a].scale != net->regs[b].scale)
            return fail(UNIHENN_ESCALE, "addition of ciphertexts at different levels or scales");
        int d = newreg(net->regs[a].nl, net->regs[a].scale, is_ext(a));
        Step s;
        s.kind = ST_ADD;
        s.dst = d;
        s.a = a;
        s.b = b;
        net->steps.push_back(s);
        return d;
    }

    // sum of ciphertexts: one n-ary step (an addition for two terms); the
    // same residues as a chain of additions, since the sum is exact mod q
    int sum(std::vector<int> xs)
    {
        if (xs.empty()) return fail(UNIHENN_EINVAL, "empty sum");
        if (xs.size() == 1) return xs[0];
        if (xs.size() == 2) return add(xs[0], xs[1]);
        if (any_ext(xs))
            for (int& x : xs) x = to_ext(x);
        const VReg r0 = net->regs[xs[0]];
        for (int x : xs)
            if (net->regs[x].nl != r0.nl || net->regs[x].scale != r0.scale)
                return fail(UNIHENN_ESCALE, "addition of ciphertexts at different levels or scales");
        int d = newreg(r0.nl, r0.scale, r0.ext);
        Step s;
        s.kind = ST_SUM;
        s.dst = d;
        s.srcs = xs;
        net->steps.push_back(s);
        return d;
    }

    // request plaintexts Encode(w_t * z) at `scale` and nl limbs (nl + 1
    // with ext: the residue mod P follows); returns the offset of the first
    // (the others follow, (nl + ext) * N words apart)
    size_t request(const std::vector<double>& z, const std::vector<double>& w, double scale, int nl, int mont,
                   bool ext = false)
    {
        PtRequest r{z, w, scale, nl, mont, net->pt_words, ext ? 1 : 0};
        for (size_t t = 0; t < w.size(); ++t) pt_ext[net->pt_words + t * (size_t)(nl + r.ext) * c->n] = r.ext;
        net->pt_words += w.size() * (size_t)(nl + r.ext) * c->n;
        net->requests.push_back(std::move(r));
        return net->requests.back().offset;
    }

    // whether a sum over these sources runs in extended form
    bool any_ext(const std::vector<int>& srcs) const
    {
        for (int r : srcs)
            if (is_ext(r)) return true;
        return false;
    }

    std::vector<double> mask(const std::vector<long>& pos, double value = 1.0) const
    {
        std::vector<double> z(net->n_slots, 0.0);
        for (int b = 0; b < net->samples; ++b)
            for (long p : pos) z[(size_t)b * net->stride + p] = value;
        return z;
    }

    // out = Rescale(sum_t pts[t] (*) srcs[t]); one MAC step then one rescale
    // (extended sources: the sum is extended and brought down before the
    // rescale; its plaintexts must carry the P limb)
    int mac_rescale(std::vector<Term> terms)
    {
        if (terms.empty()) return fail(UNIHENN_EINVAL, "empty sum");
        bool ext = false;
        for (const Term& t : terms) ext |= is_ext(t.src);
        for (Term& t : terms) {
            if (ext) t.src = to_ext(t.src);
            if (pt_ext.at(t.pt) != (int)ext) return fail(UNIHENN_EINVAL, "plaintext form does not match its sum");
        }
        const VReg r0 = net->regs[terms[0].src];
        for (const Term& t : terms)
            if (net->regs[t.src].nl != r0.nl || net->regs[t.src].scale != r0.scale)
                return fail(UNIHENN_ESCALE, "multiply-accumulate terms at different levels or scales");
        if (r0.nl < 2) return fail(UNIHENN_ELEVEL, "level exhausted");
        int acc = newreg(r0.nl, r0.scale * delta, ext);
        Step s;
        s.kind = ST_MAC;
        s.dst = acc;
        s.terms = terms;
        net->steps.push_back(s);
        return rescale(norm(acc));
    }

    int rescale(int a)
    {
        a = norm(a);
        const VReg r = net->regs[a];
        if (r.nl < 2) return fail(UNIHENN_ELEVEL, "level exhausted");
        int d = newreg(r.nl - 1, r.scale / (double)c->primes[r.nl - 1]);
        Step s;
        s.kind = ST_RESCALE;
        s.dst = d;
        s.a = a;
        net->steps.push_back(s);
        return d;
    }

    int add_plain_vec(int a, const std::vector<double>& z)
    {
        a = norm(a);
        const VReg r = net->regs[a];
        double one = 1.0;
        size_t off = request(z, std::vector<double>(1, one), r.scale, r.nl, 0);
        int d = newreg(r.nl, r.scale);
        Step s;
        s.kind = ST_ADD_PLAIN;
        s.dst = d;
        s.a = a;
        s.pt = off;
        net->steps.push_back(s);
        return d;
    }

    int square(int a)
    {
        a = norm(a);
        const VReg r = net->regs[a];
        if (r.nl < 2) return fail(UNIHENN_ELEVEL, "level exhausted");
        const double s2 = r.scale * r.scale;
        int d = newreg(r.nl - 1, s2 / (double)c->primes[r.nl - 1]);
        Step s;
        s.kind = ST_SQUARE;
        s.dst = d;
        s.a = a;
        net->steps.push_back(s);
        return d;
    }

    // Mul(C) + relinearisation + rescale of a by b (b dropped to a's level)
    int mul(int a, int b)
    {
        a = norm(a);
        b = norm(b);
        const VReg ra = net->regs[a], rb = net->regs[b];
        if (ra.nl < 2) return fail(UNIHENN_ELEVEL, "level exhausted");
        if (rb.nl < ra.nl) return fail(UNIHENN_ELEVEL, "product operand below the other's level");
        int d = newreg(ra.nl - 1, ra.scale * rb.scale / (double)c->primes[ra.nl - 1]);
        Step s;
        s.kind = ST_MUL;
        s.dst = d;
        s.a = a;
        s.b = b;
        net->steps.push_back(s);
        return d;
    }

    // in-sample slots of the valid values register `reg` holds
    std::vector<long> valid_positions(const Layout& L, int reg) const
    {
        std::vector<long> pos;
        if (L.vec) {
            for (int v = 0; v < L.length; ++v) pos.push_back(v);
            return pos;
        }
        for (int ch = 0; ch < L.C; ++ch)
            if (L.ch_reg[ch] == reg)
                for (int y = 0; y < L.H; ++y)
                    for (int x = 0; x < L.W; ++x) pos.push_back((long)L.ch_off[ch] + (long)L.I * (x + (long)L.W_img * y));
        return pos;
    }

    // Section V-A: f(x) = a + b x + c x^2 evaluated as x (c' x + b') + a in
    // two levels, with a pending pooling factor p folded into the
    // coefficients (c' = c p^2, b' = b p; Section IV-C); zero outside the
    // valid slots
    int relu_layer(Layout& L, const unihenn_layer& ly)
    {
        const double ca = ly.weights ? ly.weights[0] : 0.375373;
        const double cb = ly.weights ? ly.weights[1] : 0.5;
        const double cc = ly.weights ? ly.weights[2] : 0.117071;
        const double p = L.pending;
        std::map<int, int> mapped;
        for (int& reg : L.ch_reg) {
            if (!mapped.count(reg)) {
                const std::vector<long> pos = valid_positions(L, reg);
                const VReg r = net->regs[reg];
                size_t off = request(mask(pos), std::vector<double>(1, cc * p * p), delta, r.nl, 1, is_ext(reg));
                int y = mac_rescale({Term{reg, off}});
                if (y < 0) return -1;
                y = add_plain_vec(y, mask(pos, cb * p));
                int z = mul(y, reg);
                if (z < 0) return -1;
                mapped[reg] = add_plain_vec(z, mask(pos, ca));
            }
            reg = mapped[reg];
        }
        L.prev = 3;
        L.pending = 1.0;
        L.clean = true;  // masked to the valid slots
        return 0;
    }

    // Algorithm 1 -----------------------------------------------------------
    int conv(Layout& L, const unihenn_layer& ly)
    {
        const KernelGeom g = geom(ly);
        const int ci = (int)ly.ch_in, co = (int)ly.ch_out;
        if (L.vec || ci != L.C) return fail(UNIHENN_EINVAL, "conv input channels do not match");
        if (!(g.kw >= g.sw && g.sw >= 1 && g.kh >= g.sh && g.sh >= 1))
            return fail(UNIHENN_EINVAL, "conv needs kernel >= stride >= 1 (Theorem 1)");
        if (L.H + 2 * g.ph < g.kh || L.W + 2 * g.pw < g.kw) return fail(UNIHENN_EINVAL, "conv kernel larger than its input");
        if (!ly.weights || !ly.bias) return fail(UNIHENN_EINVAL, "conv without weights or bias");
        // Section VI's padding space: a padded read above the map lands in the
        // sample's lead, one left of column 0 in the previous row's zero
        // margin, one below the map past its last row; all of them must be
        // zero slots
        if (g.ph || g.pw) {
            if (!L.clean)
                return fail(UNIHENN_EINVAL, "padded convolution of a pooled map (partial sums lie where the padding reads)");
            bool own = true;
            for (int i = 0; i < ci; ++i)
                for (int i2 = i + 1; i2 < ci; ++i2) own &= L.ch_reg[i] != L.ch_reg[i2];
            if (!own) return fail(UNIHENN_EINVAL, "padded convolution needs one ciphertext per input channel");
            if (L.W_img - L.W < g.pw) return fail(UNIHENN_EINVAL, "row pitch leaves fewer zero columns than the padding");
            if ((long)L.lead < (long)L.I * ((long)g.ph * L.W_img + g.pw))
                return fail(UNIHENN_EINVAL, "leading space below the padding's rows");
        }
        const int Ho = (L.H + 2 * g.ph - g.kh) / g.sh + 1, Wo = (L.W + 2 * g.pw - g.kw) / g.sw + 1;
        const int I_out = L.I * g.sw;
        std::vector<long> pos;
        for (int y = 0; y < Ho; ++y)
            for (int x = 0; x < Wo; ++x) pos.push_back((long)L.lead + (long)I_out * (x + (long)L.W_img * y));
        const std::vector<double> m_out = mask(pos);
        const int nl = net->regs[L.ch_reg[0]].nl;
        const double s_in = net->regs[L.ch_reg[0]].scale;
        auto weight = [&](int o, int i, int j, int k) {
            return ly.weights[(((size_t)o * ci + i) * g.kh + j) * g.kw + k] * L.pending;
        };
        // output (y, x) sits at lead + I_out (x + W_img y) and its term (i, j, k)
        // reads input (S_h y + j - P_h, S x + k - P_w) of channel i
        auto amount = [&](int i, int j, int k) {
            return (long)L.ch_off[i] - L.lead + (long)L.I * ((k - g.pw) + (long)L.W_img * (j - g.ph));
        };
        bool one_ct = true;
        for (int i = 1; i < ci; ++i) one_ct &= L.ch_reg[i] == L.ch_reg[0];
        one_ct &= ci > 1;
        // deferred ModDown: the sums are extended when any term is (a
        // rotation by r != 0, or an extended input)
        bool ext = false;
        if (lazy)
            for (int i = 0; i < ci; ++i)
                for (int j = 0; j < g.kh; ++j)
                    for (int k = 0; k < g.kw; ++k) ext |= norm_rot(amount(i, j, k)) != 0 || is_ext(L.ch_reg[i]);

        std::vector<int> acc(co, -1);
        // plaintexts: per output, every (i, j, k) weight on the valid output slots
        std::vector<std::vector<size_t>> pt(co);
        for (int o = 0; o < co; ++o) {
            std::vector<double> w;
            for (int i = 0; i < ci; ++i)
                for (int j = 0; j < g.kh; ++j)
                    for (int k = 0; k < g.kw; ++k) w.push_back(weight(o, i, j, k));
            size_t off = request(m_out, w, delta, nl, 1, ext);
            for (size_t t = 0; t < w.size(); ++t) pt[o].push_back(off + t * (size_t)(nl + ext) * c->n);
        }
        const int kk = g.kh * g.kw;
        // one step per input channel: every output accumulates that channel's K^2 products
        for (int o = 0; o < co; ++o) acc[o] = newreg(nl, s_in * delta, ext);
        auto emit_macs = [&](int i_begin, int i_end, const std::vector<int>& rot_regs, bool accumulate) {
            Step s;
            s.kind = ST_MACM;
            s.outs = acc;
            s.srcs = rot_regs;
            s.pt = pt[0][0];
            s.pt_ostride = ci * kk;
            s.pt_toff = i_begin * kk;
            s.acc = accumulate;
            s.dst = acc[0];
            (void)i_end;
            net->steps.push_back(s);
        };
        for (int i = 0; i < ci; ++i)
            if (net->regs[L.ch_reg[i]].nl != nl || net->regs[L.ch_reg[i]].scale != s_in)
                return fail(UNIHENN_ESCALE, "conv inputs at different levels or scales");
        if (nl < 2) return fail(UNIHENN_ELEVEL, "level exhausted");
        if (one_ct) {
            // all channels in one ciphertext: every rotation first, then the sums
            std::map<long, int> seen;
            std::vector<int> rr;
            for (int i = 0; i < ci; ++i)
                for (int j = 0; j < g.kh; ++j)
                    for (int k = 0; k < g.kw; ++k) {
                        long r = norm_rot(amount(i, j, k));
                        auto it = seen.find(r);
                        int reg = it != seen.end() ? it->second : rot(L.ch_reg[0], r);
                        if (ext) reg = to_ext(reg);
                        seen[r] = reg;
                        rr.push_back(reg);
                    }
            emit_macs(0, ci, rr, false);
        } else {
            // every channel's K^2 rotations, then one sum per output over all
            // CH_in K^2 terms (each output written once); when the rotated
            // batches would not fit kOneSumBytes, one channel at a time, every
            // output accumulating that channel's K^2 products
            const size_t reg_bytes = (size_t)net->max_batch * 2 * (size_t)(nl + ext) * c->n * sizeof(u64);
            const bool one_sum = (size_t)ci * kk * reg_bytes <= kOneSumBytes;
            std::vector<int> all;
            for (int i = 0; i < ci; ++i) {
                std::map<long, int> seen;
                std::vector<int> rr;
                for (int j = 0; j < g.kh; ++j)
                    for (int k = 0; k < g.kw; ++k) {
                        long r = norm_rot(amount(i, j, k));
                        auto it = seen.find(r);
                        int reg = it != seen.end() ? it->second : rot(L.ch_reg[i], r);
                        if (ext) reg = to_ext(reg);
                        seen[r] = reg;
                        rr.push_back(reg);
                    }
                if (one_sum) all.insert(all.end(), rr.begin(), rr.end());
                else emit_macs(i, i + 1, rr, i > 0);
            }
            if (one_sum) emit_macs(0, ci, all, false);
        }
        Layout out;
        out.C = co;
        out.H = Ho;
        out.W = Wo;
        out.I = I_out;
        out.W_img = L.W_img;
        out.prev = 1;
        out.pending = 1.0;
        out.lead = L.lead;
        for (int o = 0; o < co; ++o) {
            int r = rescale(acc[o]);
            if (r < 0) return -1;
            std::vector<double> bz = mask(pos, ly.bias[o]);
            int d = add_plain_vec(r, bz);
            out.ch_reg.push_back(d);
            out.ch_off.push_back(L.lead);
        }
        L = out;
        return 0;
    }

    // Section IV-C ----------------------------------------------------------
    int avgpool(Layout& L, const unihenn_layer& ly)
    {
        const int cc = (int)ly.k;
        if (L.vec || cc < 1 || L.H < cc || L.W < cc) return fail(UNIHENN_EINVAL, "bad pooling shape");
        std::map<int, int> mapped;
        for (int reg : L.ch_reg) {
            if (mapped.count(reg)) continue;
            std::vector<int> terms;
            for (int dy = 0; dy < cc; ++dy)
                for (int dx = 0; dx < cc; ++dx) terms.push_back(rot(reg, (long)L.I * (dx + (long)L.W_img * dy)));
            int acc = sum(terms);
            if (acc < 0) return -1;
            mapped[reg] = acc;
        }
        for (int& reg : L.ch_reg) reg = mapped[reg];
        L.H /= cc;
        L.W /= cc;
        L.I *= cc;
        L.prev = 2;
        L.pending /= (double)(cc * cc);
        L.clean = false;  // partial sums around the pooled grid (and past its width)
        return 0;
    }

    int square_layer(Layout& L)
    {
        std::map<int, int> mapped;
        if (L.vec) {
            int d = square(L.ch_reg[0]);
            if (d < 0) return -1;
            L.ch_reg[0] = d;
        } else {
            for (int& reg : L.ch_reg) {
                if (!mapped.count(reg)) {
                    int d = square(reg);
                    if (d < 0) return -1;
                    mapped[reg] = d;
                }
                reg = mapped[reg];
            }
        }
        L.pending *= L.pending;
        return 0;
    }

    // Section IV-E ----------------------------------------------------------
    int flatten(Layout& L)
    {
        if (L.vec) return fail(UNIHENN_EINVAL, "flatten of a vector");
        for (int c0 = 0; c0 < L.C; ++c0)
            for (int c1 = c0 + 1; c1 < L.C; ++c1)
                if (L.ch_reg[c0] == L.ch_reg[c1]) return fail(UNIHENN_EINVAL, "flatten needs one ciphertext per channel");
        for (int off : L.ch_off)
            if (off != L.lead) return fail(UNIHENN_EINVAL, "flatten needs every channel at the sample's lead");
        const int S = L.I, Wi = L.W, Hi = L.H, Wimg = L.W_img;
        // the first stage that rotates also moves the maps from the lead to 0
        long sh = L.lead;
        std::vector<int> ys = L.ch_reg;
        const int nl = net->regs[ys[0]].nl;
        // a sum is extended when any of its terms is; its plaintexts follow (pts[ext])
        if (L.prev == 2) {
            // invalid values between the pooled ones: one mask per column x
            std::vector<size_t> pts[2];
            for (int& X : ys) {
                std::vector<int> srcs;
                for (int x = 0; x < Wi; ++x) srcs.push_back(rot(X, sh + (long)x * (S - 1)));
                const bool ext = any_ext(srcs);
                if (pts[ext].empty())
                    for (int x = 0; x < Wi; ++x) {
                        std::vector<long> pos;
                        for (int y = 0; y < Hi; ++y) pos.push_back((long)S * Wimg * y + x);
                        pts[ext].push_back(request(mask(pos), std::vector<double>(1, L.pending), delta, nl, 1, ext));
                    }
                std::vector<Term> terms;
                for (int x = 0; x < Wi; ++x) terms.push_back({srcs[x], pts[ext][x]});
                X = mac_rescale(terms);
                if (X < 0) return -1;
            }
            sh = 0;
        } else if (S > 1 && Wi > 1) {
            // zeros between the values: S shifted copies summed, then one mask per group of S columns
            const int G = (Wi + S - 1) / S;
            std::vector<size_t> pts[2];
            for (int& X : ys) {
                std::vector<int> shifted;
                for (int m = 0; m < S; ++m) shifted.push_back(rot(X, sh + (long)m * (S - 1)));
                int T = sum(shifted);
                if (T < 0) return -1;
                std::vector<int> srcs;
                for (int gq = 0; gq < G; ++gq) srcs.push_back(rot(T, (long)gq * S * (S - 1)));
                const bool ext = any_ext(srcs);
                if (pts[ext].empty())
                    for (int gq = 0; gq < G; ++gq) {
                        std::vector<long> pos;
                        for (int y = 0; y < Hi; ++y)
                            for (int m = 0; m < S; ++m)
                                if (gq * S + m < Wi) pos.push_back((long)S * Wimg * y + (long)gq * S + m);
                        pts[ext].push_back(request(mask(pos), std::vector<double>(1, L.pending), delta, nl, 1, ext));
                    }
                std::vector<Term> terms;
                for (int gq = 0; gq < G; ++gq) terms.push_back({srcs[gq], pts[ext][gq]});
                X = mac_rescale(terms);
                if (X < 0) return -1;
            }
            sh = 0;
        } else if (L.pending != 1.0) {
            std::vector<long> pos;
            for (int y = 0; y < Hi; ++y)
                for (int x = 0; x < Wi; ++x) pos.push_back((long)Wimg * y + x);
            size_t pts[2] = {0, 0};
            bool have[2] = {false, false};
            for (int& X : ys) {
                const int src = rot(X, sh);
                const bool ext = is_ext(src);
                if (!have[ext]) {
                    pts[ext] = request(mask(pos), std::vector<double>(1, L.pending), delta, nl, 1, ext);
                    have[ext] = true;
                }
                X = mac_rescale({{src, pts[ext]}});
                if (X < 0) return -1;
            }
            sh = 0;
        }
        // (y, x) now sits at S W_img y + x; remove the column interval
        if (Hi > 1) {
            const int nl2 = net->regs[ys[0]].nl;
            std::vector<size_t> pts[2];
            for (int& X : ys) {
                std::vector<int> srcs;
                for (int y = 0; y < Hi; ++y) srcs.push_back(rot(X, sh + (long)y * ((long)Wimg * S - Wi)));
                const bool ext = any_ext(srcs);
                if (pts[ext].empty())
                    for (int y = 0; y < Hi; ++y) {
                        std::vector<long> pos;
                        for (int x = 0; x < Wi; ++x) pos.push_back((long)y * Wi + x);
                        pts[ext].push_back(request(mask(pos), std::vector<double>(1, 1.0), delta, nl2, 1, ext));
                    }
                std::vector<Term> terms;
                for (int y = 0; y < Hi; ++y) terms.push_back({srcs[y], pts[ext][y]});
                X = mac_rescale(terms);
                if (X < 0) return -1;
            }
            sh = 0;
        }
        // pack: channel o shifted right by o H W
        std::vector<int> placed;
        for (int o = 0; o < (int)ys.size(); ++o) placed.push_back(rot(ys[o], sh - (long)o * Wi * Hi));
        int acc = sum(placed);
        if (acc < 0) return -1;
        Layout out;
        out.vec = true;
        out.length = L.C * Hi * Wi;
        out.ch_reg = {acc};
        out.ch_off = {0};
        L = out;
        return 0;
    }

    // sum_{i < reps} Rot(x, i step) by doubling: S_1 = x, S_2m = S_m +
    // Rot(S_m, m step); then, for each set bit 2^b of reps from the highest
    // down, Rot(S_(2^b), o step) with o the sum of the bits above it.
    // floor(log2 reps) + popcount(reps) - 1 rotations instead of reps - 1;
    // the same slots, different rounding (each rotation rounds its own key
    // switch)
    int rotate_sum(int x, int reps, int step)
    {
        std::map<int, int> S;
        S[1] = x;
        int m = 1;
        while (2 * m <= reps) {
            S[2 * m] = add(S[m], rot(S[m], (long)m * step));
            if (S[2 * m] < 0) return -1;
            m *= 2;
        }
        int acc = -1;
        long off = 0;
        for (int bit = 30; bit >= 0; --bit) {
            if (!((reps >> bit) & 1)) continue;
            int t = rot(S[1 << bit], off * step);
            acc = acc < 0 ? t : add(acc, t);
            if (acc < 0) return -1;
            off += 1L << bit;
        }
        return acc;
    }

    // Algorithm 2 -----------------------------------------------------------
    int fc(Layout& L, const unihenn_layer& ly)
    {
        const int din = (int)ly.ch_in, D = (int)ly.ch_out;
        if (!L.vec || L.length != din) return fail(UNIHENN_EINVAL, "FC input size does not match");
        if (!ly.weights || !ly.bias || D < 1) return fail(UNIHENN_EINVAL, "FC without weights or bias");
        const int reps = (din + D - 1) / D;
        const int Wvec = D * reps;
        const int X = L.ch_reg[0];
        const int nl = net->regs[X].nl;
        std::vector<int> srcs;
        std::vector<std::vector<double>> vs;
        for (int o = 0; o < D; ++o) {
            std::vector<double> mrot(Wvec);
            for (int p = 0; p < Wvec; ++p) {
                int col = (p + o) % Wvec;
                mrot[p] = col < din ? ly.weights[(size_t)(p % D) * din + col] * L.pending : 0.0;
            }
            std::vector<double> v1(net->n_slots, 0.0), v2(net->n_slots, 0.0);
            for (int b = 0; b < net->samples; ++b)
                for (int p = 0; p < Wvec; ++p) (p < Wvec - o ? v1 : v2)[(size_t)b * net->stride + p] = mrot[p];
            srcs.push_back(rot(X, o));
            vs.push_back(std::move(v1));
            if (o >= 1) {
                srcs.push_back(rot(X, (long)o - Wvec));
                vs.push_back(std::move(v2));
            }
        }
        const bool ext = any_ext(srcs);
        std::vector<Term> terms;
        for (size_t t = 0; t < srcs.size(); ++t)
            terms.push_back({srcs[t], request(vs[t], std::vector<double>(1, 1.0), delta, nl, 1, ext)});
        int csum = mac_rescale(terms);
        if (csum < 0) return -1;
        int acc;
        if (fc_doubling) {
            acc = rotate_sum(csum, reps, D);
        } else {
            std::vector<int> parts;
            for (int i = 0; i < reps; ++i) parts.push_back(rot(csum, (long)i * D));
            acc = sum(parts);
        }
        if (acc < 0) return -1;
        std::vector<long> pos;
        for (int p = 0; p < D; ++p) pos.push_back(p);
        std::vector<double> bz(net->n_slots, 0.0);
        for (int b = 0; b < net->samples; ++b)
            for (int p = 0; p < D; ++p) bz[(size_t)b * net->stride + p] = ly.bias[p];
        int out = add_plain_vec(acc, bz);
        Layout o;
        o.vec = true;
        o.length = D;
        o.ch_reg = {out};
        o.ch_off = {0};
        L = o;
        return 0;
    }
};

// Slots one packed sample needs (Section VI): the largest extent of the
// slots holding its valid values or read by a valid output, the flatten
// output C H W, and the FC width DAT_out ceil(DAT_in / DAT_out); with
// channel_cts the input holds one H x W plane per ciphertext.
int footprint(const unihenn_input& in, const unihenn_layer* ls, int n, long* out, bool channel_cts)
{
    // the sample's lead, then the rows at pitch W_img; one ciphertext per
    // channel: each holds one H x W_img plane after the lead
    const int Wimg = in.pitch ? (int)in.pitch : (int)in.w;
    const long lead = (long)in.lead;
    long need = lead + (long)(channel_cts ? 1 : in.c) * in.h * Wimg;
    int C = (int)in.c, H = (int)in.h, W = (int)in.w, I = 1;
    long max_off = lead + (channel_cts ? 0 : (long)(in.c - 1) * in.h * Wimg);
    bool vec = false;
    for (int l = 0; l < n; ++l) {
        const unihenn_layer& L = ls[l];
        if (L.kind == UNIHENN_LAYER_CONV) {
            KernelGeom g = geom(L);
            if (vec || H + 2 * g.ph < g.kh || W + 2 * g.pw < g.kw || g.sw < 1 || g.sh < 1) return UNIHENN_EINVAL;
            int Ho = (H + 2 * g.ph - g.kh) / g.sh + 1, Wo = (W + 2 * g.pw - g.kw) / g.sw + 1;
            need = std::max(need, max_off + (long)I * ((g.sw * (Wo - 1) + g.kw - 1 - g.pw) +
                                                       (long)Wimg * (g.sh * (Ho - 1) + g.kh - 1 - g.ph)) + 1);
            I *= g.sw;
            C = (int)L.ch_out;
            H = Ho;
            W = Wo;
            max_off = lead;
            need = std::max(need, lead + (long)I * ((Wo - 1) + (long)Wimg * (Ho - 1)) + 1);
        } else if (L.kind == UNIHENN_LAYER_AVGPOOL) {
            int cc = (int)L.k;
            if (vec || cc < 1 || H < cc || W < cc) return UNIHENN_EINVAL;
            need = std::max(need, max_off + (long)I * ((cc * (W / cc) - 1) + (long)Wimg * (cc * (H / cc) - 1)) + 1);
            H /= cc;
            W /= cc;
            I *= cc;
        } else if (L.kind == UNIHENN_LAYER_FLATTEN) {
            need = std::max(need, (long)C * H * W);
            vec = true;
        } else if (L.kind == UNIHENN_LAYER_FC) {
            long D = L.ch_out;
            if (D < 1) return UNIHENN_EINVAL;
            need = std::max(need, D * ((L.ch_in + D - 1) / D));
        }
    }
    *out = need;
    return UNIHENN_OK;
}

// multiplicative depth: conv 1, square 1, FC 1, flatten
// [after pooling, or interval > 1, or a pending factor] + [H > 1]
int count_depth(const unihenn_input& in, const unihenn_layer* ls, int n)
{
    int d = 0, prev = 0, I = 1, H = (int)in.h, W = (int)in.w;
    double pending = 1.0;
    for (int l = 0; l < n; ++l) {
        const unihenn_layer& L = ls[l];
        switch (L.kind) {
        case UNIHENN_LAYER_CONV: {
            KernelGeom g = geom(L);
            d += 1;
            prev = 1;
            I *= g.sw;
            pending = 1.0;
            H = (H + 2 * g.ph - g.kh) / g.sh + 1;
            W = (W + 2 * g.pw - g.kw) / g.sw + 1;
            break;
        }
        case UNIHENN_LAYER_SQUARE: d += 1; pending *= pending; break;
        case UNIHENN_LAYER_RELU_APPROX: d += 2; prev = 3; pending = 1.0; break;
        case UNIHENN_LAYER_AVGPOOL:
            prev = 2;
            I *= (int)L.k;
            pending /= (double)(L.k * L.k);
            H /= (int)L.k;
            W /= (int)L.k;
            break;
        case UNIHENN_LAYER_FLATTEN: d += (prev == 2 || (I > 1 && W > 1) || pending != 1.0) + (H > 1); break;
        case UNIHENN_LAYER_FC: d += 1; break;
        default: return -1;
        }
    }
    return d;
}

// register allocation: buffers by limb count (extended registers hold one
// more), reused after a value's last use
void allocate(unihenn_net* net, std::vector<int>& phys_nl)
{
    const int nr = (int)net->regs.size();
    std::vector<int> last(nr, -1), def(nr, -1);
    auto use = [&](int r, int s) { if (r >= 0) last[r] = std::max(last[r], s); };
    for (int s = 0; s < (int)net->steps.size(); ++s) {
        const Step& st = net->steps[s];
        use(st.a, s);
        use(st.b, s);
        for (const Term& t : st.terms) use(t.src, s);
        for (int r : st.srcs) use(r, s);
        if (st.acc) use(st.dst, s);
        if (st.dst >= 0 && def[st.dst] < 0) def[st.dst] = s;
        use(st.dst, s);
        for (int r : st.outs) {
            if (def[r] < 0) def[r] = s;
            use(r, s);
        }
    }
    for (int r : net->out_regs) last[r] = (int)net->steps.size();
    std::map<int, std::vector<int>> free_by_nl;
    // The executor issues runs of consecutive steps of one kind as a single
    // launch set, where every element reads and writes concurrently; a buffer
    // read anywhere in such a run is therefore released only after the run.
    const int ns = (int)net->steps.size();
    std::vector<int> run_end(ns);
    for (int s = ns - 1; s >= 0; --s)
        run_end[s] = (s + 1 < ns && net->steps[s + 1].kind == net->steps[s].kind) ? run_end[s + 1] : s;
    std::vector<std::vector<int>> dying(net->steps.size() + 1);
    for (int r = 0; r < nr; ++r)
        if (last[r] >= 0 && last[r] < (int)net->steps.size()) dying[run_end[last[r]]].push_back(r);
    for (int s = 0; s < (int)net->steps.size(); ++s) {
        std::vector<int> defs = net->steps[s].outs;
        if (net->steps[s].dst >= 0) defs.push_back(net->steps[s].dst);
        for (int d : defs) {
            if (def[d] != s || net->regs[d].phys >= 0) continue;
            auto& fl = free_by_nl[net->regs[d].limbs()];
            if (!fl.empty()) {
                net->regs[d].phys = fl.back();
                fl.pop_back();
            } else {
                net->regs[d].phys = (int)phys_nl.size();
                phys_nl.push_back(net->regs[d].limbs());
            }
        }
        for (int r : dying[s])
            if (net->regs[r].phys >= 0) free_by_nl[net->regs[r].limbs()].push_back(net->regs[r].phys);
    }
}

// Within each layer, order the steps by dependency level (independent steps
// become neighbours) and, inside a level, by kind and source, so that the
// executor can issue runs of independent steps of one kind together.
void schedule_layers(unihenn_net* net)
{
    auto kind_order = [](StepKind k) {
        switch (k) {
        case ST_ROT: return 0;
        case ST_EXT: return 1;       // after the rotations: their runs stay unbroken
        case ST_MACM: return 2;
        case ST_MAC: return 3;
        case ST_MODDOWN: return 4;
        case ST_RESCALE: return 4;
        case ST_SQUARE: return 5;
        case ST_MUL: return 5;
        case ST_ADD_PLAIN: return 6;
        case ST_ADD: return 7;
        case ST_SUM: return 7;
        default: return 8;
        }
    };
    for (LayerRecord& L : net->layers) {
        const size_t b = L.step_begin, e = L.step_end;
        if (e - b < 2) continue;
        std::map<int, size_t> producer;  // register -> step index (in range)
        std::vector<int> level(e - b, 0);
        for (size_t i = b; i < e; ++i) {
            const Step& st = net->steps[i];
            int lv = 0;
            auto dep = [&](int r) {
                auto it = producer.find(r);
                if (r >= 0 && it != producer.end()) lv = std::max(lv, level[it->second - b] + 1);
            };
            dep(st.a);
            dep(st.b);
            for (const Term& t : st.terms) dep(t.src);
            for (int r : st.srcs) dep(r);
            if (st.acc) {
                dep(st.dst);
                for (int r : st.outs) dep(r);
            }
            level[i - b] = lv;
            if (st.dst >= 0) producer[st.dst] = i;
            for (int r : st.outs) producer[r] = i;
        }
        std::vector<size_t> idx(e - b);
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = b + i;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
            const Step &sx = net->steps[x], &sy = net->steps[y];
            if (level[x - b] != level[y - b]) return level[x - b] < level[y - b];
            if (kind_order(sx.kind) != kind_order(sy.kind)) return kind_order(sx.kind) < kind_order(sy.kind);
            if (sx.kind == ST_ROT && sx.a != sy.a) return sx.a < sy.a;
            return false;
        });
        std::vector<Step> sorted;
        sorted.reserve(idx.size());
        for (size_t i : idx) sorted.push_back(net->steps[i]);
        std::copy(sorted.begin(), sorted.end(), net->steps.begin() + b);
    }
}

}  // namespace

// Workspace words for grouped key switching with groups of E rotations (at
// the widest level and largest batch), single key switches, grouped squares
// and grouped rescales.
// Largest E * B of a grouped elementwise run over batches B <= max_batch when
// the executor groups E = min(UH_EW_GROUP_MAX, max(1, per / B)) steps.
static size_t max_group_batch(int max_batch, int per)
{
    size_t m = 0;
    for (int b = 1; b <= max_batch; ++b)
        m = std::max(m, (size_t)std::min(UH_EW_GROUP_MAX, std::max(1, per / b)) * (size_t)b);
    return m;
}

static size_t net_ws_words(const unihenn_ctx* c, const unihenn_net* net, int E_)
{
    const size_t L0 = (size_t)net->ws_nl, Bm = (size_t)net->max_batch, E = (size_t)E_;
    const size_t group_rows = Bm * (L0 + L0 * L0) + E * Bm * (L0 * L0 + 7 * L0 + 2);
    const int mb = net->max_batch;
    size_t ws_rows = std::max(ks_ws_rows(net->ws_nl, mb), group_rows);
    // grouped squares and products (E * B batches at once), grouped rescales and ModDowns
    ws_rows = std::max(ws_rows, group_square_ws_rows((int)max_group_batch(mb, 32), net->ws_nl, 1));
    ws_rows = std::max(ws_rows, max_group_batch(mb, 64) * 2 * (L0 + 1));
    return ws_rows * (size_t)c->n;
}

// Graphs are captured on the net's own stream, which then stays idle, and
// replayed on the caller's stream in order with the caller's other work.
static hipError_t begin_capture(unihenn_net* net)
{
    hipError_t e = hipStreamSynchronize(net->gstream);
    return e != hipSuccess ? e : hipStreamBeginCapture(net->gstream, hipStreamCaptureModeThreadLocal);
}

static void drop_graphs(unihenn_net* net)
{
    // a replay may still run on a caller's stream
    if (!net->graphs.empty() || !net->stage_graphs.empty()) (void)hipDeviceSynchronize();
    for (auto& g : net->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    net->graphs.clear();
    for (auto& g : net->stage_graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    net->stage_graphs.clear();
}

// ---------------------------------------------------------------- C ABI
extern "C" int unihenn_net_destroy(unihenn_net* net)
{
    if (!net) return UNIHENN_OK;
    // a replay still in flight reads the arenas: let it finish first
    drop_graphs(net);
    if (net->gstream) (void)hipStreamDestroy(net->gstream);
    (void)hipFree(net->pt_arena);
    (void)hipFree(net->reg_arena);
    (void)hipFree(net->ws);
    delete net;
    return UNIHENN_OK;
}

extern "C" int unihenn_net_create(const unihenn_ctx* c, const unihenn_input* in, const unihenn_layer* layers,
                                  uint32_t n_layers, uint32_t max_batch, unihenn_net** out)
{
    return unihenn_net_create_ex(c, in, layers, n_layers, max_batch, 0u, out);
}

extern "C" int unihenn_net_create_ex(const unihenn_ctx* c, const unihenn_input* in, const unihenn_layer* layers,
                                     uint32_t n_layers, uint32_t max_batch, uint32_t plan_flags, unihenn_net** out)
{
    if (!c || !in || !out || (n_layers && !layers)) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (plan_flags & ~(uint32_t)(UNIHENN_PLAN_LAZY_MODDOWN | UNIHENN_PLAN_FC_DOUBLING | UNIHENN_PLAN_CHANNEL_CTS))
        return uh_fail(UNIHENN_EINVAL, "unknown plan flag");
    const bool channel_cts = (plan_flags & UNIHENN_PLAN_CHANNEL_CTS) != 0;
    if (in->c < 1 || in->h < 1 || in->w < 1 || in->samples < 1 || max_batch < 1)
        return uh_fail(UNIHENN_EINVAL, "empty input shape, sample count or batch");
    if (in->pitch && in->pitch < in->w) return uh_fail(UNIHENN_EINVAL, "row pitch below the input width");
    for (uint32_t l = 0; l < n_layers; ++l)
        if (layers[l].kind < UNIHENN_LAYER_CONV || layers[l].kind > UNIHENN_LAYER_RELU_APPROX)
            return uh_fail(UNIHENN_EINVAL, "unknown layer kind");
    unihenn_net* net = new unihenn_net();
    net->ctx = c;
    net->lazy = (plan_flags & UNIHENN_PLAN_LAZY_MODDOWN) != 0;
    net->n_slots = c->n / 2;
    net->samples = (int)in->samples;
    net->max_batch = (int)max_batch;
    long fp = 0;
    if (footprint(*in, layers, (int)n_layers, &fp, channel_cts)) {
        delete net;
        return uh_fail(UNIHENN_EINVAL, "layer shapes do not chain");
    }
    if (in->samples == 1) {
        net->stride = net->n_slots;
        if (fp > net->n_slots) {
            delete net;
            return uh_fail(UNIHENN_ESLOTS, "the model's footprint exceeds the slots");
        }
    } else {
        net->stride = (int)in->stride;
        if ((long)in->stride < fp || (long)in->samples * in->stride > net->n_slots) {
            delete net;
            return uh_fail(UNIHENN_ESLOTS, "sample stride " + std::to_string(in->stride) + " below the footprint " +
                                               std::to_string(fp) + " or samples exceed the slots");
        }
    }
    net->depth = count_depth(*in, layers, (int)n_layers);
    net->in_limbs = net->depth + 1;
    if (net->depth < 0 || net->in_limbs > c->n_data) {
        delete net;
        return uh_fail(UNIHENN_ELEVEL, "the network needs " + std::to_string(net->in_limbs) + " limbs, the chain has " +
                                           std::to_string(c->n_data));
    }

    Planner P{net, c, c->scale, {}, "", 0};
    P.lazy = net->lazy;
    P.fc_doubling = (plan_flags & UNIHENN_PLAN_FC_DOUBLING) != 0;
    // the inputs, reduced to depth + 1 limbs: one ciphertext, or one per channel
    net->n_inputs = channel_cts ? (int)in->c : 1;
    std::vector<int> input_regs;
    for (int i = 0; i < net->n_inputs; ++i) {
        input_regs.push_back(P.newreg(net->in_limbs, c->scale));
        Step s;
        s.kind = ST_DROP;
        s.dst = input_regs.back();
        s.in_idx = i;
        net->steps.push_back(s);
    }
    net->input_reg = input_regs[0];
    // input layout: the sample's lead of zero slots (Section VI's padding
    // space), then the rows at pitch W_img (zero beyond the width)
    Layout L;
    L.C = (int)in->c;
    L.H = (int)in->h;
    L.W = (int)in->w;
    L.I = 1;
    L.W_img = in->pitch ? (int)in->pitch : (int)in->w;
    L.lead = (int)in->lead;
    for (uint32_t ch = 0; ch < in->c; ++ch) {
        L.ch_reg.push_back(channel_cts ? input_regs[ch] : net->input_reg);
        L.ch_off.push_back(L.lead + (channel_cts ? 0 : (int)(ch * in->h * (uint32_t)L.W_img)));
    }
    for (uint32_t l = 0; l < n_layers; ++l) {
        LayerRecord rec;
        rec.kind = layers[l].kind;
        rec.step_begin = net->steps.size();
        rec.in_regs = L.ch_reg;
        int rc = 0;
        switch (layers[l].kind) {
        case UNIHENN_LAYER_CONV: rc = P.conv(L, layers[l]); break;
        case UNIHENN_LAYER_SQUARE: rc = P.square_layer(L); break;
        case UNIHENN_LAYER_RELU_APPROX: rc = P.relu_layer(L, layers[l]); break;
        case UNIHENN_LAYER_AVGPOOL: rc = P.avgpool(L, layers[l]); break;
        case UNIHENN_LAYER_FLATTEN: rc = P.flatten(L); break;
        case UNIHENN_LAYER_FC: rc = P.fc(L, layers[l]); break;
        }
        // the network's outputs in normal form
        if (rc >= 0 && l + 1 == n_layers)
            for (int& r : L.ch_reg) r = P.norm(r);
        if (rc < 0 || P.err_code) {
            int code = P.err_code ? P.err_code : UNIHENN_EINVAL;
            std::string m = P.err;
            delete net;
            return uh_fail(code, "layer " + std::to_string(l) + ": " + m);
        }
        rec.step_end = net->steps.size();
        rec.out_regs = L.ch_reg;
        rec.interval_out = L.I;
        net->layers.push_back(rec);
    }
    // outputs: distinct registers in channel order
    for (int r : L.ch_reg)
        if (std::find(net->out_regs.begin(), net->out_regs.end(), r) == net->out_regs.end()) net->out_regs.push_back(r);
    for (int b = 0; b < net->samples; ++b) {
        long base = (long)b * net->stride;
        if (L.vec) {
            for (int v = 0; v < L.length; ++v) net->out_slots.push_back((uint64_t)(base + v));
        } else {
            for (int ch = 0; ch < L.C; ++ch) {
                uint64_t idx = std::find(net->out_regs.begin(), net->out_regs.end(), L.ch_reg[ch]) - net->out_regs.begin();
                for (int y = 0; y < L.H; ++y)
                    for (int x = 0; x < L.W; ++x)
                        net->out_slots.push_back((idx << 32) | (uint64_t)(base + L.ch_off[ch] + (long)L.I * (x + (long)L.W_img * y)));
            }
        }
    }
    net->n_values = L.vec ? L.length : L.C * L.H * L.W;
    for (auto& kv : P.rotset) net->rotations.push_back(kv.first);
    for (int r : net->out_regs)
        if (net->regs[r].nl != 1) {
            unihenn_net_destroy(net);
            return uh_fail(UNIHENN_ELEVEL, "output not at one limb");
        }

    if (max_batch <= 8 && !getenv("UNIHENN_NO_SCHEDULE")) schedule_layers(net);
    // device memory: plaintexts, registers, workspace
    std::vector<int> phys_nl;
    allocate(net, phys_nl);
    size_t reg_words = 0;
    for (int nl : phys_nl) {
        net->phys_off.push_back(reg_words);
        reg_words += (size_t)max_batch * 2 * nl * c->n;
    }
    net->ws_nl = net->in_limbs;
    net->group_max = net->group_alloc = std::max(1, std::min(UH_GROUP_MAX, 32 / (int)max_batch));
    net->ws_words = net_ws_words(c, net, net->group_alloc);
    if (hipMalloc(&net->pt_arena, sizeof(u64) * std::max<size_t>(net->pt_words, 1)) != hipSuccess ||
        hipMalloc(&net->reg_arena, sizeof(u64) * std::max<size_t>(reg_words, 1)) != hipSuccess ||
        hipMalloc(&net->ws, sizeof(u64) * net->ws_words) != hipSuccess) {
        unihenn_net_destroy(net);
        return uh_fail(UNIHENN_ENOMEM, "network buffers");
    }
    for (const PtRequest& r : net->requests) {
        int rc = encode_scaled_batch(c, r.z.data(), (int)r.z.size(), r.w.data(), (int)r.w.size(), r.scale, r.nl,
                                     r.mont, net->pt_arena + r.offset, nullptr, r.ext);
        if (rc) {
            unihenn_net_destroy(net);
            return rc;
        }
    }
    net->requests.clear();
    net->requests.shrink_to_fit();
    *out = net;
    return UNIHENN_OK;
}

extern "C" int unihenn_net_info(const unihenn_net* net, uint32_t* depth, uint32_t* n_rotations, uint32_t* n_outputs,
                                uint32_t* input_limbs)
{
    if (!net) return uh_fail(UNIHENN_EINVAL, "null net");
    if (depth) *depth = (uint32_t)net->depth;
    if (n_rotations) *n_rotations = (uint32_t)net->rotations.size();
    if (n_outputs) *n_outputs = (uint32_t)net->out_regs.size();
    if (input_limbs) *input_limbs = (uint32_t)net->in_limbs;
    return UNIHENN_OK;
}

extern "C" int unihenn_net_inputs(const unihenn_net* net, uint32_t* n_inputs)
{
    if (!net || !n_inputs) return uh_fail(UNIHENN_EINVAL, "null argument");
    *n_inputs = (uint32_t)net->n_inputs;
    return UNIHENN_OK;
}

extern "C" int unihenn_net_rotations(const unihenn_net* net, int32_t* steps)
{
    if (!net || !steps) return uh_fail(UNIHENN_EINVAL, "null argument");
    for (size_t i = 0; i < net->rotations.size(); ++i) steps[i] = net->rotations[i];
    return UNIHENN_OK;
}

extern "C" int unihenn_net_output_slots(const unihenn_net* net, uint64_t* positions, uint32_t* n_values)
{
    if (!net) return uh_fail(UNIHENN_EINVAL, "null net");
    if (n_values) *n_values = (uint32_t)net->n_values;
    if (positions) std::copy(net->out_slots.begin(), net->out_slots.end(), positions);
    return UNIHENN_OK;
}

extern "C" int unihenn_net_bind_keys(unihenn_net* net, const int32_t* steps, const unihenn_evk* gks, uint32_t n,
                                     const unihenn_evk* rlk)
{
    if (!net || (n && (!steps || !gks))) return uh_fail(UNIHENN_EINVAL, "null argument");
    const unihenn_ctx* c = net->ctx;
    std::map<int, const u64*> k;
    for (uint32_t i = 0; i < n; ++i) {
        if (!gks[i].data || (int)gks[i].n_data != c->n_data) return uh_fail(UNIHENN_EINVAL, "bad rotation key");
        long h = net->n_slots;
        k[(int)(((steps[i] % h) + h) % h)] = gks[i].data;
    }
    for (int r : net->rotations)
        if (!k.count(r)) return uh_fail(UNIHENN_ENOKEY, "no key for rotation " + std::to_string(r));
    bool needs_rlk = false;
    for (const Step& s : net->steps) needs_rlk |= s.kind == ST_SQUARE || s.kind == ST_MUL;
    if (needs_rlk && (!rlk || !rlk->data || (int)rlk->n_data != c->n_data))
        return uh_fail(UNIHENN_ENOKEY, "no relinearisation key");
    net->keys = k;
    net->rlk = rlk ? rlk->data : nullptr;
    net->key_version++;
    return UNIHENN_OK;
}

extern "C" int unihenn_net_set_mode(unihenn_net* net, int mode)
{
    if (!net || mode < 0 || mode > (UNIHENN_EVAL_HOISTED | UNIHENN_EVAL_GRAPH))
        return uh_fail(UNIHENN_EINVAL, "bad mode");
    net->mode = mode;
    return UNIHENN_OK;
}

// ---------------------------------------------------------------- execution
namespace {

struct Exec {
    unihenn_net* net;
    const unihenn_ctx* c;
    int B;
    hipStream_t s;
    std::map<int, u64*> bound;  // registers bound to caller buffers
    int modup_owner = -1;       // register whose digits the workspace holds
    std::vector<const u64*> ext_in;  // network inputs (ST_DROP sources), all at ext_in_limbs
    int ext_in_limbs = 0;
    size_t slot = 0;                 // first batch slot of the net's registers this evaluation uses

    u64* reg(int r)
    {
        auto it = bound.find(r);
        if (it != bound.end()) return it->second;
        return net->reg_arena + net->phys_off[net->regs[r].phys] + slot * 2 * net->regs[r].limbs() * c->n;
    }

    // workspace carve for grouped rotations (fixed offsets at the net's widest level)
    struct GroupWs {
        u64 *pdcoef, *pmodup, *aux, *dcoef, *modup, *U, *Up, *R;
    };
    GroupWs carve() const
    {
        const size_t rn = (size_t)c->n, L0 = (size_t)net->ws_nl, Bm = (size_t)net->max_batch,
                     E = (size_t)net->group_alloc;
        GroupWs w;
        u64* p = net->ws;
        w.pdcoef = p; p += Bm * L0 * rn;
        w.pmodup = p; p += Bm * L0 * L0 * rn;
        w.aux = p;    p += E * Bm * 2 * L0 * rn;
        w.dcoef = p;  p += E * Bm * L0 * rn;
        w.modup = p;  p += E * Bm * L0 * L0 * rn;
        w.U = p;      p += E * Bm * 2 * L0 * rn;
        w.Up = p;     p += E * Bm * 2 * rn;
        w.R = p;
        return w;
    }

    void fill(GroupArgs& ga, const std::vector<size_t>& run, size_t from, int count)
    {
        memset(&ga, 0, sizeof(ga));
        ga.E = count;
        for (int e = 0; e < count; ++e) {
            const Step& st = net->steps[run[from + e]];
            ga.src[e] = reg(st.a);
            ga.dst[e] = reg(st.dst);
            ga.key[e] = net->keys.at(st.rot);
            ga.g[e] = galois_elt(c, st.rot);
        }
    }

    // consecutive steps from `si` accepted by `ok`, at the same output level,
    // none reading a result of another; at most max_e steps (and max_e2)
    template <class F>
    std::vector<size_t> collect(size_t si, size_t end, int nl, F ok, int max_e, int max_e2)
    {
        std::vector<size_t> run;
        std::vector<int> made;
        int cap = std::max(1, std::min(max_e, max_e2));
        static const char* nog = getenv("UNIHENN_NO_GROUP");  // kinds (step enum digits) never grouped
        if (nog && strchr(nog, '0' + (int)net->steps[si].kind)) cap = 1;
        const bool ext = net->regs[net->steps[si].dst].ext;
        for (size_t sj = si; sj < end && (int)run.size() < cap; ++sj) {
            const Step& x = net->steps[sj];
            if (!ok(x) || net->regs[x.dst].nl != nl || net->regs[x.dst].ext != ext) break;
            bool dep = false;
            auto reads = [&](int r) { return r >= 0 && std::find(made.begin(), made.end(), r) != made.end(); };
            dep |= reads(x.a) || reads(x.b);
            for (const Term& t : x.terms) dep |= reads(t.src);
            if (dep) break;
            run.push_back(sj);
            made.push_back(x.dst);
        }
        return run;
    }

    // ext: the rotations stay extended (inner product only, no ModDown)
    void rotations(const std::vector<size_t>& run, int nl, bool ext)
    {
        const size_t rn = (size_t)c->n;
        GroupWs w = carve();
        const int Emax = net->group_max;
        if (net->mode & UNIHENN_EVAL_HOISTED) {
            // Launch sets of up to Emax rotations: whole runs of one source
            // while they fit, a source with more rotations alone in pieces of
            // Emax.  The distinct sources of a set are its ModUp blocks (each
            // decomposed once); every rotation reads its source's digits
            // through its automorphism.  A one-source set whose digits the
            // workspace still holds (the previous set's) skips the ModUp.
            size_t i = 0;
            while (i < run.size()) {
                std::vector<size_t> set;
                size_t j = i;
                while (j < run.size()) {
                    const int src = net->steps[run[j]].a;
                    size_t e = j;
                    while (e < run.size() && net->steps[run[e]].a == src) ++e;
                    if (set.empty()) {
                        const size_t take = std::min<size_t>(e - j, (size_t)Emax);
                        set.insert(set.end(), run.begin() + j, run.begin() + j + take);
                        j += take;
                        if (j < e) break;  // the source continues in the next set
                    } else if (set.size() + (e - j) <= (size_t)Emax) {
                        set.insert(set.end(), run.begin() + j, run.begin() + e);
                        j = e;
                    } else {
                        break;
                    }
                }
                i = j;
                GroupArgs ga;
                fill(ga, set, 0, (int)set.size());
                ga.dstride = 2 * nl;
                std::vector<int> srcs;
                for (int e = 0; e < ga.E; ++e) {
                    const int src = net->steps[set[e]].a;
                    int d = (int)(std::find(srcs.begin(), srcs.end(), src) - srcs.begin());
                    if (d == (int)srcs.size()) srcs.push_back(src);
                    ga.blk[e] = d;
                    ga.gin[e] = ga.gdig[e] = ga.g[e];
                }
                const u64* digits;
                if (srcs.size() == 1) {
                    const u64* d = reg(srcs[0]) + (size_t)nl * rn;
                    if (modup_owner != srcs[0]) {
                        group_modup(c, 1, &d, 2 * nl, B, nl, w.pdcoef, w.pmodup, s);
                        modup_owner = srcs[0];
                    }
                    ga.dsrc[0] = d;
                    digits = w.pmodup;
                } else {
                    std::vector<const u64*> d(srcs.size());
                    for (size_t q = 0; q < srcs.size(); ++q) d[q] = ga.dsrc[q] = reg(srcs[q]) + (size_t)nl * rn;
                    group_modup(c, (int)srcs.size(), d.data(), 2 * nl, B, nl, w.dcoef, w.modup, s);
                    digits = w.modup;
                }
                if (ext) group_switch_ext(c, ga, B, nl, digits, s);
                else group_switch(c, ga, B, nl, true, digits, w.aux, w.U, w.Up, w.R, s);
            }
        } else if (ntt_fusable(c)) {
            // each rotation decomposes its own tau(c1): the inverse NTT reads
            // c1 through the automorphism, the inner product reads the
            // digit of the same limb through it, and the ModDown takes tau(c0)
            // straight from the source
            for (size_t k = 0; k < run.size(); k += Emax) {
                GroupArgs ga;
                fill(ga, run, k, (int)std::min<size_t>(Emax, run.size() - k));
                ga.dstride = 2 * nl;
                std::vector<const u64*> d(ga.E);
                std::vector<u32> perm(ga.E);
                for (int e = 0; e < ga.E; ++e) {
                    ga.blk[e] = e;
                    ga.gin[e] = 1;                              // digits of tau(c1) itself
                    ga.gdig[e] = ga.g[e];                       // limb j of tau(c1), read from c1
                    ga.dsrc[e] = ga.src[e] + (size_t)nl * rn;  // c1 of src_e
                    d[e] = ga.dsrc[e];
                    perm[e] = ga.g[e];
                }
                // workgroup order 2: the row pass of the digits' forward NTT
                // runs inside the inner product
                const bool rf = group_modup(c, ga.E, d.data(), 2 * nl, B, nl, w.dcoef, w.modup, s, perm.data(),
                                            c->ks_order != 2);
                if (ext) group_switch_ext(c, ga, B, nl, w.modup, s, rf);
                else group_switch(c, ga, B, nl, true, w.modup, w.aux, w.U, w.Up, w.R, s, rf);
            }
            modup_owner = -1;
        } else {
            for (size_t k = 0; k < run.size(); k += Emax) {
                GroupArgs ga;
                fill(ga, run, k, (int)std::min<size_t>(Emax, run.size() - k));
                ga.dstride = 2 * nl;
                std::vector<const u64*> d(ga.E);
                for (int e = 0; e < ga.E; ++e) {
                    ga.blk[e] = e;
                    ga.gin[e] = ga.gdig[e] = 1;
                    ga.dsrc[e] = w.aux + ((size_t)e * B * 2 * nl + nl) * rn;  // c1 of tau(src_e)
                    d[e] = ga.dsrc[e];
                }
                group_auto_both(c, ga, B, nl, w.aux, s);
                group_modup(c, ga.E, d.data(), 2 * nl, B, nl, w.dcoef, w.modup, s);
                if (ext) group_switch_ext(c, ga, B, nl, w.modup, s);
                else group_switch(c, ga, B, nl, false, w.modup, w.aux, w.U, w.Up, w.R, s);
            }
            modup_owner = -1;
        }
    }

    int run(size_t begin, size_t end)
    {
        for (size_t si = begin; si < end; ++si) {
            const Step& st = net->steps[si];
            const int nl = net->regs[st.dst].nl;
            // rows per polynomial of the destination, and its P limb (extended) or -1
            const bool ext = net->regs[st.dst].ext;
            const int lim = net->regs[st.dst].limbs();
            const int pl = ext ? nl : -1;
            switch (st.kind) {
            case ST_DROP:
                launch_gather_rows(c, reg(st.dst), ext_in.at(st.in_idx), B * 2 * nl, nl, ext_in_limbs, 0, s);
                break;
            case ST_ROT: {
                // a run of consecutive rotations at this level, none reading another's result
                std::vector<size_t> run;
                size_t sj = si;
                while (sj < end && net->steps[sj].kind == ST_ROT && net->regs[net->steps[sj].dst].nl == nl &&
                       net->regs[net->steps[sj].dst].ext == ext) {
                    bool dep = false;
                    for (size_t x : run) dep |= net->steps[x].dst == net->steps[sj].a;
                    if (dep) break;
                    run.push_back(sj++);
                }
                rotations(run, nl, ext);
                si = sj - 1;
                break;
            }
            case ST_MAC: {
                // a run of independent single-output sums with the same term count
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) {
                    return x.kind == ST_MAC && !x.acc && x.terms.size() == st.terms.size() &&
                           x.terms.size() <= UH_MACG_MAX;
                }, UH_EW_GROUP_MAX, (int)(UH_MACG_MAX / std::max<size_t>(1, st.terms.size())));
                if (run.size() > 1) {
                    MacGroup m;
                    memset(&m, 0, sizeof(m));
                    m.E = (int)run.size();
                    m.T = (int)st.terms.size();
                    for (int e = 0; e < m.E; ++e) {
                        const Step& x = net->steps[run[e]];
                        m.acc[e] = reg(x.dst);
                        for (int t = 0; t < m.T; ++t) {
                            m.ct[e * m.T + t] = reg(x.terms[t].src);
                            m.pt[e * m.T + t] = net->pt_arena + x.terms[t].pt;
                        }
                    }
                    launch_mac_group(c, m, lim, B, s, pl);
                    si = run.back();
                    break;
                }
                const size_t nt = st.terms.size();
                for (size_t t0 = 0; t0 < nt; t0 += UH_MAC_MAX_TERMS) {
                    MacTerms mt;
                    int k = (int)std::min<size_t>(UH_MAC_MAX_TERMS, nt - t0);
                    for (int t = 0; t < k; ++t) {
                        mt.ct[t] = reg(st.terms[t0 + t].src);
                        mt.pt[t] = net->pt_arena + st.terms[t0 + t].pt;
                    }
                    launch_mac(c, reg(st.dst), mt, k, lim, B, (st.acc || t0 > 0) ? 1 : 0, s, pl);
                }
                break;
            }
            case ST_MACM: {
                const int O = (int)st.outs.size(), T = (int)st.srcs.size();
                for (int o0 = 0; o0 < O; o0 += UH_MACM_MAX_OUT) {
                    const int no = std::min(UH_MACM_MAX_OUT, O - o0);
                    for (int t0 = 0; t0 < T; t0 += UH_MAC_MAX_TERMS) {
                        const int nt = std::min(UH_MAC_MAX_TERMS, T - t0);
                        MacMulti m;
                        memset(&m, 0, sizeof(m));
                        for (int o = 0; o < no; ++o) m.acc[o] = reg(st.outs[o0 + o]);
                        for (int t = 0; t < nt; ++t) m.ct[t] = reg(st.srcs[t0 + t]);
                        m.pt_base = net->pt_arena + st.pt + (size_t)o0 * st.pt_ostride * lim * c->n;
                        m.o_stride = st.pt_ostride;
                        m.t_off = st.pt_toff + t0;
                        launch_mac_multi(c, m, no, nt, lim, B, (st.acc || t0 > 0) ? 1 : 0, s, pl);
                    }
                }
                break;
            }
            case ST_RESCALE: {
                const int nla = net->regs[st.a].nl;
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) { return x.kind == ST_RESCALE; },
                                                  UH_EW_GROUP_MAX, std::max(1, 64 / B));
                std::vector<const u64*> ins;
                std::vector<u64*> outs;
                for (size_t x : run) {
                    ins.push_back(reg(net->steps[x].a));
                    outs.push_back(reg(net->steps[x].dst));
                }
                group_rescale(c, (int)run.size(), ins.data(), outs.data(), B, nla, net->ws, s);
                modup_owner = -1;
                si = run.back();
                break;
            }
            case ST_ADD:
            case ST_ADD_PLAIN: {
                const StepKind kind = st.kind;
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) { return x.kind == kind; },
                                                  UH_EW_GROUP_MAX, UH_EW_GROUP_MAX);
                EwGroup g;
                memset(&g, 0, sizeof(g));
                g.E = (int)run.size();
                for (int e = 0; e < g.E; ++e) {
                    const Step& x = net->steps[run[e]];
                    g.out[e] = reg(x.dst);
                    g.a[e] = reg(x.a);
                    g.b[e] = kind == ST_ADD ? reg(x.b) : net->pt_arena + x.pt;
                }
                launch_group_add(c, g, B, lim, kind == ST_ADD_PLAIN, s, pl);
                si = run.back();
                break;
            }
            case ST_SUM: {
                // independent sums with the same term count, one launch per
                // UH_SUM_MAX_TERMS terms of the group
                const int T = (int)st.srcs.size();
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) {
                    return x.kind == ST_SUM && (int)x.srcs.size() == T;
                }, UH_EW_GROUP_MAX, std::max(1, UH_SUM_MAX_TERMS / T));
                SumGroup g;
                memset(&g, 0, sizeof(g));
                g.E = (int)run.size();
                for (int t0 = 0; t0 < T; t0 += UH_SUM_MAX_TERMS) {
                    g.T = std::min(UH_SUM_MAX_TERMS, T - t0);
                    for (int e = 0; e < g.E; ++e) {
                        const Step& x = net->steps[run[e]];
                        g.out[e] = reg(x.dst);
                        for (int t = 0; t < g.T; ++t) g.in[e * g.T + t] = reg(x.srcs[t0 + t]);
                    }
                    launch_group_sum(c, g, B, lim, t0 > 0, s, pl);
                }
                si = run.back();
                break;
            }
            case ST_EXT: {
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) { return x.kind == ST_EXT; },
                                                  UH_EW_GROUP_MAX, UH_EW_GROUP_MAX);
                EwGroup g;
                memset(&g, 0, sizeof(g));
                g.E = (int)run.size();
                for (int e = 0; e < g.E; ++e) {
                    g.a[e] = reg(net->steps[run[e]].a);
                    g.out[e] = reg(net->steps[run[e]].dst);
                }
                launch_group_to_ext(c, g, B, nl, s);
                si = run.back();
                break;
            }
            case ST_MODDOWN: {
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) { return x.kind == ST_MODDOWN; },
                                                  UH_EW_GROUP_MAX, std::max(1, 64 / B));
                std::vector<const u64*> ins;
                std::vector<u64*> outs;
                for (size_t x : run) {
                    ins.push_back(reg(net->steps[x].a));
                    outs.push_back(reg(net->steps[x].dst));
                }
                group_moddown(c, (int)run.size(), ins.data(), outs.data(), B, nl, net->ws, s);
                modup_owner = -1;
                si = run.back();
                break;
            }
            case ST_SQUARE: {
                const int nla = net->regs[st.a].nl;
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) { return x.kind == ST_SQUARE; },
                                                  UH_EW_GROUP_MAX, std::max(1, 32 / B));
                std::vector<const u64*> ins;
                std::vector<u64*> outs;
                for (size_t x : run) {
                    ins.push_back(reg(net->steps[x].a));
                    outs.push_back(reg(net->steps[x].dst));
                }
                group_square(c, (int)run.size(), ins.data(), outs.data(), net->rlk, B, nla, net->ws, s);
                modup_owner = -1;
                si = run.back();
                break;
            }
            case ST_MUL: {
                const int nla = net->regs[st.a].nl, nlb = net->regs[st.b].nl;
                std::vector<size_t> run = collect(si, end, nl, [&](const Step& x) {
                    return x.kind == ST_MUL && net->regs[x.a].nl == nla && net->regs[x.b].nl == nlb;
                }, UH_EW_GROUP_MAX, std::max(1, 32 / B));
                std::vector<const u64*> ins, in2;
                std::vector<u64*> outs;
                for (size_t x : run) {
                    ins.push_back(reg(net->steps[x].a));
                    in2.push_back(reg(net->steps[x].b));
                    outs.push_back(reg(net->steps[x].dst));
                }
                group_square(c, (int)run.size(), ins.data(), outs.data(), net->rlk, B, nla, net->ws, s, in2.data(),
                             nlb);
                modup_owner = -1;
                si = run.back();
                break;
            }
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return uh_fail(UNIHENN_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
        return UNIHENN_OK;
    }
};

int check_keys(const unihenn_net* net)
{
    if (net->keys.size() < net->rotations.size()) return uh_fail(UNIHENN_ENOKEY, "keys not bound");
    for (const Step& s : net->steps)
        if ((s.kind == ST_SQUARE || s.kind == ST_MUL) && !net->rlk)
            return uh_fail(UNIHENN_ENOKEY, "relinearisation key not bound");
    return UNIHENN_OK;
}

}  // namespace

extern "C" int unihenn_eval_network(const unihenn_ctx* c, unihenn_net* net, const unihenn_ct* in, unihenn_ct* out,
                                    void* stream)
{
    if (!c || !net || !in || !in->data || !out) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (net->ctx != c) return uh_fail(UNIHENN_EINVAL, "net made for another context");
    if (in->batch < 1 || (int)in->batch > net->max_batch) return uh_fail(UNIHENN_EINVAL, "batch exceeds max_batch");
    if ((int)in->n_limbs < net->in_limbs) return uh_fail(UNIHENN_ELEVEL, "input has fewer limbs than the depth needs");
    if ((int)in->n_limbs > c->n_data) return uh_fail(UNIHENN_ELEVEL, "bad input limb count");
    if (in->scale != c->scale) return uh_fail(UNIHENN_ESCALE, "input scale differs from the encoding scale");
    std::vector<const u64*> ins;
    for (int i = 0; i < net->n_inputs; ++i) {
        if (!in[i].data) return uh_fail(UNIHENN_EINVAL, "null input " + std::to_string(i));
        if (in[i].batch != in->batch || in[i].n_limbs != in->n_limbs || in[i].scale != in->scale)
            return uh_fail(UNIHENN_EINVAL, "input " + std::to_string(i) + " differs in batch, limbs or scale");
        ins.push_back(in[i].data);
    }
    int rc = check_keys(net);
    if (rc) return rc;
    for (size_t i = 0; i < net->out_regs.size(); ++i)
        if (!out[i].data) return uh_fail(UNIHENN_EINVAL, "null output buffer");
    const bool graph = (net->mode & UNIHENN_EVAL_GRAPH) && !stats_enabled();
    hipStream_t cs = (hipStream_t)stream;
    if (!graph) {
        Exec ex{net, c, (int)in->batch, cs, {}, -1, ins, (int)in->n_limbs};
        for (size_t i = 0; i < net->out_regs.size(); ++i) ex.bound[net->out_regs[i]] = out[i].data;
        rc = ex.run(0, net->steps.size());
        if (rc) return rc;
    } else {
        if (!net->gstream) UH_CHECK_HIP(hipStreamCreateWithFlags(&net->gstream, hipStreamNonBlocking));
        std::vector<u64*> outs;
        for (size_t i = 0; i < net->out_regs.size(); ++i) outs.push_back(out[i].data);
        unihenn_net::GraphEntry* hit = nullptr;
        for (auto& g : net->graphs)
            if (g.exec && g.batch == (int)in->batch && g.in == ins && g.in_limbs == (int)in->n_limbs &&
                g.outs == outs && g.mode == net->mode && g.key_version == net->key_version)
                hit = &g;
        if (!hit) {
            // capture into a free slot, or replace the least recently used of 16
            if (net->graphs.size() < 16) {
                net->graphs.emplace_back();
                hit = &net->graphs.back();
            } else {
                hit = &net->graphs[0];
                for (auto& g : net->graphs)
                    if (g.last_use < hit->last_use) hit = &g;
                // it may still run on a caller's stream
                UH_CHECK_HIP(hipDeviceSynchronize());
                if (hit->exec) (void)hipGraphExecDestroy(hit->exec);
                hit->exec = nullptr;
            }
            Exec ex{net, c, (int)in->batch, net->gstream, {}, -1, ins, (int)in->n_limbs};
            for (size_t i = 0; i < net->out_regs.size(); ++i) ex.bound[net->out_regs[i]] = out[i].data;
            UH_CHECK_HIP(begin_capture(net));
            int rc2 = ex.run(0, net->steps.size());
            hipGraph_t graph_obj = nullptr;
            hipError_t e = hipStreamEndCapture(net->gstream, &graph_obj);
            if (rc2) {
                if (graph_obj) (void)hipGraphDestroy(graph_obj);
                return rc2;
            }
            if (e != hipSuccess) return uh_fail(UNIHENN_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&hit->exec, graph_obj, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph_obj);
            if (e != hipSuccess) {
                hit->exec = nullptr;
                return uh_fail(UNIHENN_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            hit->batch = (int)in->batch;
            hit->in = ins;
            hit->in_limbs = (int)in->n_limbs;
            hit->outs = outs;
            hit->mode = net->mode;
            hit->key_version = net->key_version;
        }
        hit->last_use = ++net->graph_clock;
        UH_CHECK_HIP(hipGraphLaunch(hit->exec, cs));
    }
    for (size_t i = 0; i < net->out_regs.size(); ++i) {
        out[i].n_limbs = 1;
        out[i].batch = in->batch;
        out[i].scale = net->regs[net->out_regs[i]].scale;
    }
    return UNIHENN_OK;
}

extern "C" int unihenn_conv(const unihenn_ctx* c, unihenn_net* net, uint32_t layer, const unihenn_ct* in,
                            uint32_t n_in, unihenn_ct* out, uint32_t* interval_out, void* stream)
{
    if (!c || !net || !in || !out) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (layer >= net->layers.size() || net->layers[layer].kind != UNIHENN_LAYER_CONV)
        return uh_fail(UNIHENN_EINVAL, "layer is not a convolution");
    const LayerRecord& L = net->layers[layer];
    std::vector<int> uniq;
    for (int r : L.in_regs)
        if (std::find(uniq.begin(), uniq.end(), r) == uniq.end()) uniq.push_back(r);
    if (n_in != uniq.size()) return uh_fail(UNIHENN_EINVAL, "expected " + std::to_string(uniq.size()) + " inputs");
    const int B = (int)in[0].batch;
    if (B < 1 || B > net->max_batch) return uh_fail(UNIHENN_EINVAL, "batch exceeds max_batch");
    for (uint32_t i = 0; i < n_in; ++i) {
        const VReg& r = net->regs[uniq[i]];
        if (r.ext) return uh_fail(UNIHENN_EINVAL, "the layer's input is an extended sum in this plan");
        if (!in[i].data || (int)in[i].n_limbs != r.nl || (int)in[i].batch != B)
            return uh_fail(UNIHENN_ELEVEL, "input " + std::to_string(i) + " not at the layer's level");
        if (in[i].scale != r.scale) return uh_fail(UNIHENN_ESCALE, "input scale differs from the plan");
    }
    int rc = check_keys(net);
    if (rc) return rc;
    Exec ex{net, c, B, (hipStream_t)stream, {}, -1, {}, 0};
    for (uint32_t i = 0; i < n_in; ++i) ex.bound[uniq[i]] = in[i].data;
    for (size_t o = 0; o < L.out_regs.size(); ++o) {
        if (!out[o].data) return uh_fail(UNIHENN_EINVAL, "null output buffer");
        ex.bound[L.out_regs[o]] = out[o].data;
    }
    rc = ex.run(L.step_begin, L.step_end);
    if (rc) return rc;
    for (size_t o = 0; o < L.out_regs.size(); ++o) {
        const VReg& r = net->regs[L.out_regs[o]];
        out[o].n_limbs = (uint32_t)r.nl;
        out[o].batch = (uint32_t)B;
        out[o].scale = r.scale;
    }
    if (interval_out) *interval_out = (uint32_t)L.interval_out;
    return UNIHENN_OK;
}

// ---------------------------------------------------------------- layer stages
// Stage k is layer k of the plan (stage 0 also reduces the inputs to the
// network's level).  A group of batch slots of the net's registers runs its
// stages in order; groups at different stages interleave on the net's stream,
// each launch touching only its own slots.
extern "C" int unihenn_net_stages(const unihenn_net* net, uint32_t* n_stages)
{
    if (!net || !n_stages) return uh_fail(UNIHENN_EINVAL, "null argument");
    *n_stages = (uint32_t)net->layers.size();
    return UNIHENN_OK;
}

extern "C" int unihenn_net_memory(const unihenn_net* net, size_t* fixed_bytes, size_t* per_slot_bytes)
{
    if (!net || !fixed_bytes || !per_slot_bytes) return uh_fail(UNIHENN_EINVAL, "null argument");
    // every physical register holds max_batch slots of 2 * limbs rows; the
    // workspace is laid out for max_batch slots too
    size_t slot_words = 0;
    std::vector<char> seen(net->phys_off.size(), 0);
    for (const VReg& r : net->regs)
        if (r.phys >= 0 && !seen[r.phys]) {
            seen[r.phys] = 1;
            slot_words += (size_t)2 * r.limbs() * net->ctx->n;
        }
    slot_words += (net->ws_words + net->max_batch - 1) / net->max_batch;
    *per_slot_bytes = sizeof(u64) * slot_words;
    *fixed_bytes = sizeof(u64) * net->pt_words;
    return UNIHENN_OK;
}

extern "C" int unihenn_workspace_size(const unihenn_ctx* c, const unihenn_net* net, uint32_t batch, size_t* bytes)
{
    if (!c || !net || !bytes) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (net->ctx != c) return uh_fail(UNIHENN_EINVAL, "net made for another context");
    if (batch < 1 || (int)batch > net->max_batch) return uh_fail(UNIHENN_EINVAL, "batch outside 1..max_batch");
    *bytes = sizeof(u64) * net->ws_words;
    return UNIHENN_OK;
}

extern "C" int unihenn_eval_stage(const unihenn_ctx* c, unihenn_net* net, uint32_t stage, uint32_t slot,
                                  uint32_t batch, const unihenn_ct* in, unihenn_ct* out, void* stream)
{
    if (!c || !net) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (net->ctx != c) return uh_fail(UNIHENN_EINVAL, "net made for another context");
    const uint32_t ns = (uint32_t)net->layers.size();
    if (stage >= ns) return uh_fail(UNIHENN_EINVAL, "stage out of range");
    if (batch < 1 || (size_t)slot + batch > (size_t)net->max_batch)
        return uh_fail(UNIHENN_EINVAL, "slots [slot, slot + batch) exceed max_batch");
    std::vector<const u64*> ins;
    int in_limbs = 0;
    if (stage == 0) {
        if (!in || !in->data) return uh_fail(UNIHENN_EINVAL, "stage 0 needs the input ciphertexts");
        if ((int)in->n_limbs < net->in_limbs) return uh_fail(UNIHENN_ELEVEL, "input has fewer limbs than the depth needs");
        if ((int)in->n_limbs > c->n_data) return uh_fail(UNIHENN_ELEVEL, "bad input limb count");
        if (in->scale != c->scale) return uh_fail(UNIHENN_ESCALE, "input scale differs from the encoding scale");
        for (int i = 0; i < net->n_inputs; ++i) {
            if (!in[i].data || in[i].batch != batch || in[i].n_limbs != in->n_limbs || in[i].scale != in->scale)
                return uh_fail(UNIHENN_EINVAL, "input " + std::to_string(i) + " differs in batch, limbs or scale");
            ins.push_back(in[i].data);
        }
        in_limbs = (int)in->n_limbs;
    }
    if (stage + 1 == ns) {
        if (!out) return uh_fail(UNIHENN_EINVAL, "the last stage needs the output buffers");
        for (size_t i = 0; i < net->out_regs.size(); ++i)
            if (!out[i].data) return uh_fail(UNIHENN_EINVAL, "null output buffer");
    }
    int rc = check_keys(net);
    if (rc) return rc;
    std::vector<u64*> outs;
    if (stage + 1 == ns)
        for (size_t i = 0; i < net->out_regs.size(); ++i) outs.push_back(out[i].data);
    const size_t b = stage == 0 ? 0 : net->layers[stage].step_begin;
    const bool graph = (net->mode & UNIHENN_EVAL_GRAPH) && !stats_enabled();
    hipStream_t cs = (hipStream_t)stream;
    if (!graph) {
        Exec ex{net, c, (int)batch, cs, {}, -1, ins, in_limbs, slot};
        for (size_t i = 0; i < outs.size(); ++i) ex.bound[net->out_regs[i]] = outs[i];
        rc = ex.run(b, net->layers[stage].step_end);
        if (rc) return rc;
    } else {
        // one captured graph per stage, slot range and buffer set (up to 256, least recently used replaced)
        if (!net->gstream) UH_CHECK_HIP(hipStreamCreateWithFlags(&net->gstream, hipStreamNonBlocking));
        unihenn_net::GraphEntry* hit = nullptr;
        for (auto& g : net->stage_graphs)
            if (g.exec && g.stage == (int)stage && g.slot == (int)slot && g.batch == (int)batch && g.in == ins &&
                g.in_limbs == in_limbs && g.outs == outs && g.mode == net->mode && g.key_version == net->key_version)
                hit = &g;
        if (!hit) {
            if (net->stage_graphs.size() < 256) {
                net->stage_graphs.emplace_back();
                hit = &net->stage_graphs.back();
            } else {
                hit = &net->stage_graphs[0];
                for (auto& g : net->stage_graphs)
                    if (g.last_use < hit->last_use) hit = &g;
                UH_CHECK_HIP(hipDeviceSynchronize());
                if (hit->exec) (void)hipGraphExecDestroy(hit->exec);
                hit->exec = nullptr;
            }
            Exec ex{net, c, (int)batch, net->gstream, {}, -1, ins, in_limbs, slot};
            for (size_t i = 0; i < outs.size(); ++i) ex.bound[net->out_regs[i]] = outs[i];
            UH_CHECK_HIP(begin_capture(net));
            int rc2 = ex.run(b, net->layers[stage].step_end);
            hipGraph_t graph_obj = nullptr;
            hipError_t e = hipStreamEndCapture(net->gstream, &graph_obj);
            if (rc2) {
                if (graph_obj) (void)hipGraphDestroy(graph_obj);
                return rc2;
            }
            if (e != hipSuccess) return uh_fail(UNIHENN_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&hit->exec, graph_obj, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph_obj);
            if (e != hipSuccess) {
                hit->exec = nullptr;
                return uh_fail(UNIHENN_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
            }
            hit->stage = (int)stage;
            hit->slot = (int)slot;
            hit->batch = (int)batch;
            hit->in = ins;
            hit->in_limbs = in_limbs;
            hit->outs = outs;
            hit->mode = net->mode;
            hit->key_version = net->key_version;
        }
        hit->last_use = ++net->graph_clock;
        UH_CHECK_HIP(hipGraphLaunch(hit->exec, cs));
    }
    if (stage + 1 == ns)
        for (size_t i = 0; i < net->out_regs.size(); ++i) {
            out[i].n_limbs = 1;
            out[i].batch = batch;
            out[i].scale = net->regs[net->out_regs[i]].scale;
        }
    return UNIHENN_OK;
}

// ---------------------------------------------------------------- tuner hooks
int net_ks_group(const unihenn_net* net) { return net->group_max; }

// Largest group size worth trying: the library cap, limited so that the
// grouped workspace stays within 16 GiB.
int net_ks_group_cap(const unihenn_ctx* c, const unihenn_net* net)
{
    int e = 1;
    while (e * 2 <= UH_GROUP_MAX && sizeof(u64) * net_ws_words(c, net, e * 2) <= (16ull << 30)) e *= 2;
    return e;
}

// Use groups of e rotations; grows the workspace when its layout holds fewer.
// Captured graphs are dropped (they hold launch shapes and buffer addresses).
int net_set_ks_group(const unihenn_ctx* c, unihenn_net* net, int e)
{
    if (e < 1 || e > UH_GROUP_MAX) return uh_fail(UNIHENN_EINVAL, "group size out of range");
    drop_graphs(net);
    if (e > net->group_alloc) {
        const size_t words = net_ws_words(c, net, e);
        u64* ws = nullptr;
        UH_CHECK_HIP(hipDeviceSynchronize());
        if (hipMalloc(&ws, sizeof(u64) * words) != hipSuccess) return uh_fail(UNIHENN_ENOMEM, "grouped workspace");
        (void)hipFree(net->ws);
        net->ws = ws;
        net->ws_words = words;
        net->group_alloc = e;
    }
    net->group_max = e;
    return UNIHENN_OK;
}

void net_drop_graphs(unihenn_net* net) { drop_graphs(net); }

int net_max_batch(const unihenn_net* net) { return net->max_batch; }
int net_in_limbs(const unihenn_net* net) { return net->in_limbs; }
int net_n_out(const unihenn_net* net) { return (int)net->out_regs.size(); }
int net_n_inputs(const unihenn_net* net) { return net->n_inputs; }
int net_mode(const unihenn_net* net) { return net->mode; }
void net_set_mode_raw(unihenn_net* net, int mode) { net->mode = mode; }

// FNV-1a over the plan: step kinds, levels, term / output / source counts
uint64_t net_fingerprint(const unihenn_net* net)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix(net->steps.size());
    mix((uint64_t)net->in_limbs);
    mix((uint64_t)net->max_batch);
    for (const Step& st : net->steps) {
        mix((uint64_t)st.kind);
        mix((uint64_t)net->regs[st.dst].nl);
        mix((uint64_t)net->regs[st.dst].ext);
        mix(st.terms.size());
        mix(st.outs.size());
        mix(st.srcs.size());
        mix((uint64_t)(int64_t)st.rot);
    }
    return h;
}
