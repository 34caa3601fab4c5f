// CKKS evaluator primitives: key switching (hybrid, one digit per data prime,
// special prime P), rotation (plain and hoisted), plaintext multiply-
// accumulate, square + relinearisation, rescale, additions, limb drop, and
// the import / export conversions of the C ABI.
#include <algorithm>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

// ---------------------------------------------------------------- helpers
u32 galois_elt(const unihenn_ctx* c, long steps)
{
    long h = c->n / 2;
    long r = ((steps % h) + h) % h;
    u64 g = 1, two_n = 2 * (u64)c->n;
    for (long i = 0; i < r; ++i) g = g * 5 % two_n;
    return (u32)g;
}

size_t ks_ws_rows(int nl, int batch) { return (size_t)batch * ((size_t)nl * nl + 8 * (size_t)nl + 2); }

KsWs ks_ws_carve(u64* base, int nl, int batch, int n)
{
    KsWs w;
    size_t rn = (size_t)n;
    u64* p = base;
    w.dcoef = p; p += (size_t)batch * nl * rn;
    w.modup = p; p += (size_t)batch * nl * nl * rn;
    w.U = p;     p += (size_t)batch * 2 * nl * rn;
    w.Up = p;    p += (size_t)batch * 2 * rn;
    w.R = p;     p += (size_t)batch * 2 * nl * rn;
    w.aux = p;
    return w;
}

void ks_modup(const unihenn_ctx* c, const u64* d, int d_stride, int batch, int nl, KsWs& ws, hipStream_t s)
{
    launch_gather_rows(c, ws.dcoef, d, batch * nl, nl, d_stride, 0, s);
    launch_ntt_inv(c, ws.dcoef, batch * nl, rowmap_ct(nl), s);
    if (launch_ntt_fwd_modup(c, ws.modup, ws.dcoef, batch * nl, nl, s)) return;
    launch_modup(c, ws.modup, ws.dcoef, batch, nl, s);
    launch_ntt_fwd(c, ws.modup, batch * nl * nl, rowmap_modup(nl, c->n_data), s);
}

void ks_finish(const unihenn_ctx* c, const u64* d, int d_stride, const u64* key, int nd, int batch, int nl, u32 g,
               u64* out, const u64* add0, const u64* add1, int add_stride, KsWs& ws, hipStream_t s)
{
    launch_ks_inner(c, ws.U, ws.Up, d, d_stride, ws.modup, key, nd, batch, nl, g, s);
    launch_ntt_inv(c, ws.Up, batch * 2, rowmap_list({c->n_data}), s);
    FuseArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.src = ws.Up;
    fa.src_mod = c->n_data;
    fa.nl = nl;
    fa.polys = batch * 2;
    fa.x[0] = ws.U;
    fa.x_limbs = nl;
    fa.add[0][0] = add0;
    fa.add[0][1] = add1;
    fa.add_stride = add_stride;
    fa.add_perm[0] = 1;
    fa.out[0] = out;
    fa.inv = c->d_p_inv;
    if (launch_ntt_fwd_fused(c, ws.R, fa, batch * 2 * nl, KF_MODDOWN, s)) return;
    launch_lift_last(c, ws.R, ws.Up, batch * 2, nl, c->n_data, KF_MODDOWN, s);
    launch_ntt_fwd(c, ws.R, batch * 2 * nl, rowmap_ct(nl), s);
    launch_sub_scale(c, out, ws.U, nl, ws.R, c->d_p_inv, batch * 2, nl, add0, add1, add_stride, KF_MODDOWN, s);
}

void rescale_core(const unihenn_ctx* c, const u64* in, int batch, int nl, u64* out, KsWs& ws, hipStream_t s)
{
    const int l = nl - 1;
    launch_gather_rows(c, ws.Up, in, batch * 2, 1, nl, l, s);
    launch_ntt_inv(c, ws.Up, batch * 2, rowmap_list({l}), s);
    const u64* inv = c->d_inv_last + (size_t)l * c->primes.size() * 2;
    FuseArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.src = ws.Up;
    fa.src_mod = l;
    fa.nl = l;
    fa.polys = batch * 2;
    fa.x[0] = in;
    fa.x_limbs = nl;
    fa.add_perm[0] = 1;
    fa.out[0] = out;
    fa.inv = inv;
    if (launch_ntt_fwd_fused(c, ws.R, fa, batch * 2 * l, KF_RESCALE, s)) return;
    launch_lift_last(c, ws.R, ws.Up, batch * 2, l, l, KF_RESCALE, s);
    launch_ntt_fwd(c, ws.R, batch * 2 * l, rowmap_ct(l), s);
    launch_sub_scale(c, out, in, nl, ws.R, inv, batch * 2, l, nullptr, nullptr, 0, KF_RESCALE, s);
}

static int check_ct(const unihenn_ctx* c, const unihenn_ct* x, const char* what)
{
    if (!c || !x || !x->data) return uh_fail(UNIHENN_EINVAL, std::string("null ") + what);
    if (x->n_limbs < 1 || (int)x->n_limbs > c->n_data) return uh_fail(UNIHENN_ELEVEL, std::string(what) + ": bad limb count");
    if (x->batch < 1) return uh_fail(UNIHENN_EINVAL, std::string(what) + ": empty batch");
    return UNIHENN_OK;
}

static int check_ws(const unihenn_ctx* c, int nl, int batch, size_t ws_bytes, void* ws)
{
    size_t need = ks_ws_rows(nl, batch) * c->n * sizeof(u64);
    if (!ws || ws_bytes < need)
        return uh_fail(UNIHENN_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    return UNIHENN_OK;
}

static int check_key(const unihenn_ctx* c, const unihenn_evk* k, int nl)
{
    if (!k || !k->data) return uh_fail(UNIHENN_ENOKEY, "missing switching key");
    if ((int)k->n_data != c->n_data) return uh_fail(UNIHENN_EINVAL, "key made for another chain");
    if (nl > (int)k->n_data) return uh_fail(UNIHENN_ELEVEL, "key has fewer limbs than the ciphertext");
    return UNIHENN_OK;
}

static hipError_t last_launch() { return hipGetLastError(); }

#define UH_LAUNCH_CHECK()                                                                           \
    do {                                                                                            \
        hipError_t _e = last_launch();                                                              \
        if (_e != hipSuccess) return uh_fail(UNIHENN_EDEVICE, std::string("launch: ") + hipGetErrorString(_e)); \
    } while (0)

// ---------------------------------------------------------------- C ABI
extern "C" int unihenn_to_ntt(const unihenn_ctx* c, uint64_t* data, uint32_t n_limbs, uint32_t n_polys,
                              void* stream)
{
    if (!c || !data) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (n_limbs < 1 || (int)n_limbs > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    launch_ntt_fwd(c, data, (int)(n_limbs * n_polys), rowmap_ct((int)n_limbs), (hipStream_t)stream);
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_from_ntt(const unihenn_ctx* c, uint64_t* data, uint32_t n_limbs, uint32_t n_polys,
                                void* stream)
{
    if (!c || !data) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (n_limbs < 1 || (int)n_limbs > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    launch_ntt_inv(c, data, (int)(n_limbs * n_polys), rowmap_ct((int)n_limbs), (hipStream_t)stream);
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_import_ct(const unihenn_ctx* c, const uint64_t* coeff, unihenn_ct* dst, void* stream)
{
    if (!c || !coeff || !dst || !dst->data) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (dst->n_limbs < 1 || (int)dst->n_limbs > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    if (dst->batch < 1) return uh_fail(UNIHENN_EINVAL, "empty batch");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t polys = 2 * dst->batch;
    if (coeff != dst->data)
        UH_CHECK_HIP(hipMemcpyAsync(dst->data, coeff, sizeof(u64) * polys * dst->n_limbs * c->n, hipMemcpyDefault, s));
    launch_ntt_fwd(c, dst->data, (int)(dst->n_limbs * polys), rowmap_ct((int)dst->n_limbs), s);
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_export_ct(const unihenn_ctx* c, const unihenn_ct* src, uint64_t* coeff, void* stream)
{
    if (!c || !src || !src->data || !coeff) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (src->n_limbs < 1 || (int)src->n_limbs > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    if (src->batch < 1) return uh_fail(UNIHENN_EINVAL, "empty batch");
    hipStream_t s = (hipStream_t)stream;
    const uint32_t polys = 2 * src->batch;
    if (coeff != src->data)
        UH_CHECK_HIP(hipMemcpyAsync(coeff, src->data, sizeof(u64) * polys * src->n_limbs * c->n,
                                    hipMemcpyDeviceToDevice, s));
    launch_ntt_inv(c, coeff, (int)(src->n_limbs * polys), rowmap_ct((int)src->n_limbs), s);
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_import_evk(const unihenn_ctx* c, const uint64_t* coeff, uint32_t n_data, uint64_t* out,
                                  void* stream)
{
    if (!c || !coeff || !out) return uh_fail(UNIHENN_EINVAL, "null argument");
    if ((int)n_data != c->n_data) return uh_fail(UNIHENN_EINVAL, "key made for another chain");
    hipStream_t s = (hipStream_t)stream;
    const int nb = c->n_data + 1;
    const int rows = c->n_data * 2 * nb;
    if (out != coeff)
        UH_CHECK_HIP(hipMemcpyAsync(out, coeff, sizeof(u64) * rows * c->n, hipMemcpyDeviceToDevice, s));
    std::vector<int> mods;
    for (int i = 0; i < nb; ++i) mods.push_back(i);  // basis q_0..q_L, P: index i (P = n_data)
    RowMap m = rowmap_list(mods);
    launch_ntt_fwd(c, out, rows, m, s);
    launch_mont_convert(c, out, rows, m, 1, s);
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" size_t unihenn_ks_workspace_size(const unihenn_ctx* c, uint32_t n_limbs, uint32_t batch)
{
    if (!c) return 0;
    return ks_ws_rows((int)n_limbs, (int)batch) * c->n * sizeof(u64);
}

static int rotate_checks(const unihenn_ctx* c, const unihenn_ct* in, const unihenn_ct* out)
{
    int rc = check_ct(c, in, "input");
    if (rc) return rc;
    if (!out || !out->data) return uh_fail(UNIHENN_EINVAL, "null output");
    if (out->data == in->data) return uh_fail(UNIHENN_EINVAL, "output aliases input");
    return UNIHENN_OK;
}

extern "C" int unihenn_rotate(const unihenn_ctx* c, const unihenn_ct* in, int32_t steps, const unihenn_evk* gk,
                              unihenn_ct* out, void* ws, size_t ws_bytes, void* stream)
{
    int rc = rotate_checks(c, in, out);
    if (rc) return rc;
    const int nl = (int)in->n_limbs, B = (int)in->batch;
    hipStream_t s = (hipStream_t)stream;
    out->n_limbs = in->n_limbs;
    out->batch = in->batch;
    out->scale = in->scale;
    u32 g = galois_elt(c, steps);
    if (g == 1) {
        UH_CHECK_HIP(hipMemcpyAsync(out->data, in->data, sizeof(u64) * (size_t)B * 2 * nl * c->n,
                                    hipMemcpyDeviceToDevice, s));
        return UNIHENN_OK;
    }
    if ((rc = check_key(c, gk, nl))) return rc;
    if ((rc = check_ws(c, nl, B, ws_bytes, ws))) return rc;
    KsWs w = ks_ws_carve((u64*)ws, nl, B, c->n);
    // tau_g of both components, then key-switch tau_g(c1)
    launch_automorphism(c, w.aux, in->data, B * 2 * nl, g, s);
    ks_modup(c, w.aux + (size_t)nl * c->n, 2 * nl, B, nl, w, s);
    ks_finish(c, w.aux + (size_t)nl * c->n, 2 * nl, gk->data, c->n_data, B, nl, 1, out->data, w.aux, nullptr, 2 * nl,
              w, s);
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

// ---- rotation without allocation: a fixed device scratch array per GPU
// holds the key-switching workspace instead of a caller buffer.
#define UH_SCRATCH_BYTES (64ull << 20)
static __device__ __align__(256) u64 scratch[UH_SCRATCH_BYTES / sizeof(u64)];
namespace {
std::mutex g_scratch_mu;
std::vector<u64*> g_scratch_dev;  // device address of `scratch`, by device ordinal (null until looked up)
}  // namespace

// The device address of this GPU's copy of `scratch`, looked up once per
// device with that device current.  The host-side name of the array is only a
// stand-in: kernels and copies take the address found here.
static int scratch_address(const unihenn_ctx* c, u64** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return uh_fail(UNIHENN_EDEVICE, "hipGetDevice failed");
    if (dev != c->device)
        return uh_fail(UNIHENN_EINVAL, "the context's device must be current (context on device " +
                                           std::to_string(c->device) + ", current " + std::to_string(dev) + ")");
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return uh_fail(UNIHENN_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = (u64*)p;
    }
    *out = g_scratch_dev[dev];
    return UNIHENN_OK;
}

extern "C" int unihenn_rotate_noalloc(const unihenn_ctx* c, const unihenn_ct* in, int32_t steps,
                                      const unihenn_evk* gk, unihenn_ct* out, void* stream)
{
    int rc = rotate_checks(c, in, out);
    if (rc) return rc;
    const size_t need = ks_ws_rows((int)in->n_limbs, (int)in->batch) * c->n * sizeof(u64);
    if (need > UH_SCRATCH_BYTES)
        return uh_fail(UNIHENN_EINVAL, "rotation needs " + std::to_string(need) +
                                           " bytes of workspace, above the fixed scratch of " +
                                           std::to_string(UH_SCRATCH_BYTES) + " bytes (use unihenn_rotate)");
    if (galois_elt(c, steps) != 1 && (rc = check_key(c, gk, (int)in->n_limbs))) return rc;
    u64* ws = nullptr;
    if ((rc = scratch_address(c, &ws))) return rc;
    return unihenn_rotate(c, in, steps, gk, out, ws, UH_SCRATCH_BYTES, stream);
}

extern "C" int unihenn_rotate_hoisted(const unihenn_ctx* c, const unihenn_ct* in, const int32_t* steps,
                                      uint32_t n_steps, const unihenn_evk* gks, unihenn_ct* outs, void* ws,
                                      size_t ws_bytes, void* stream)
{
    if (!steps || !outs || (n_steps && !gks)) return uh_fail(UNIHENN_EINVAL, "null argument");
    int rc = check_ct(c, in, "input");
    if (rc) return rc;
    const int nl = (int)in->n_limbs, B = (int)in->batch;
    hipStream_t s = (hipStream_t)stream;
    bool any = false;
    for (uint32_t i = 0; i < n_steps; ++i) {
        if ((rc = rotate_checks(c, in, &outs[i]))) return rc;
        if (galois_elt(c, steps[i]) != 1) {
            any = true;
            if ((rc = check_key(c, &gks[i], nl))) return rc;
        }
    }
    if (any && (rc = check_ws(c, nl, B, ws_bytes, ws))) return rc;
    KsWs w = any ? ks_ws_carve((u64*)ws, nl, B, c->n) : KsWs{};
    if (any) ks_modup(c, in->data + (size_t)nl * c->n, 2 * nl, B, nl, w, s);
    for (uint32_t i = 0; i < n_steps; ++i) {
        unihenn_ct* o = &outs[i];
        o->n_limbs = in->n_limbs;
        o->batch = in->batch;
        o->scale = in->scale;
        u32 g = galois_elt(c, steps[i]);
        if (g == 1) {
            UH_CHECK_HIP(hipMemcpyAsync(o->data, in->data, sizeof(u64) * (size_t)B * 2 * nl * c->n,
                                        hipMemcpyDeviceToDevice, s));
            continue;
        }
        // tau_g(c0) into aux, then the inner product reads the lifted digits of
        // c1 through the permutation
        launch_automorphism(c, w.aux, in->data, B * 2 * nl, g, s);
        ks_finish(c, in->data + (size_t)nl * c->n, 2 * nl, gks[i].data, c->n_data, B, nl, g, o->data, w.aux, nullptr,
                  2 * nl, w, s);
    }
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_mul_plain_acc(const unihenn_ctx* c, const unihenn_ct* cts, const uint64_t* const* pts,
                                     uint32_t n_terms, int overwrite, unihenn_ct* acc, void* stream)
{
    if (!c || !cts || !pts || !acc || !acc->data || n_terms == 0) return uh_fail(UNIHENN_EINVAL, "null argument");
    const int nl = (int)cts[0].n_limbs, B = (int)cts[0].batch;
    for (uint32_t t = 0; t < n_terms; ++t) {
        int rc = check_ct(c, &cts[t], "term");
        if (rc) return rc;
        if ((int)cts[t].n_limbs != nl) return uh_fail(UNIHENN_ELEVEL, "terms at different levels");
        if ((int)cts[t].batch != B) return uh_fail(UNIHENN_EINVAL, "terms with different batch sizes");
        if (cts[t].scale != cts[0].scale) return uh_fail(UNIHENN_ESCALE, "terms at different scales");
        if (!pts[t]) return uh_fail(UNIHENN_EINVAL, "null plaintext");
    }
    if (!overwrite && ((int)acc->n_limbs != nl || (int)acc->batch != B))
        return uh_fail(UNIHENN_ELEVEL, "accumulator shape differs");
    if (!overwrite && acc->scale != cts[0].scale * c->scale)
        return uh_fail(UNIHENN_ESCALE, "accumulator scale differs");
    hipStream_t s = (hipStream_t)stream;
    for (uint32_t t0 = 0; t0 < n_terms; t0 += UH_MAC_MAX_TERMS) {
        MacTerms mt;
        int nt = (int)std::min<uint32_t>(UH_MAC_MAX_TERMS, n_terms - t0);
        for (int t = 0; t < nt; ++t) {
            mt.ct[t] = cts[t0 + t].data;
            mt.pt[t] = pts[t0 + t];
        }
        launch_mac(c, acc->data, mt, nt, nl, B, (t0 > 0 || !overwrite) ? 1 : 0, s);
    }
    acc->n_limbs = (uint32_t)nl;
    acc->batch = (uint32_t)B;
    acc->scale = cts[0].scale * c->scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_rescale(const unihenn_ctx* c, const unihenn_ct* in, unihenn_ct* out, void* ws,
                               size_t ws_bytes, void* stream)
{
    int rc = check_ct(c, in, "input");
    if (rc) return rc;
    if (in->n_limbs < 2) return uh_fail(UNIHENN_ELEVEL, "level exhausted: one limb left");
    if (!out || !out->data) return uh_fail(UNIHENN_EINVAL, "null output");
    if (out->data == in->data) return uh_fail(UNIHENN_EINVAL, "output aliases input");
    const int nl = (int)in->n_limbs, B = (int)in->batch;
    if ((rc = check_ws(c, nl, B, ws_bytes, ws))) return rc;
    KsWs w = ks_ws_carve((u64*)ws, nl, B, c->n);
    rescale_core(c, in->data, B, nl, out->data, w, (hipStream_t)stream);
    out->n_limbs = in->n_limbs - 1;
    out->batch = in->batch;
    out->scale = in->scale / (double)c->primes[nl - 1];
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_mul_relin(const unihenn_ctx* c, const unihenn_ct* a, const unihenn_ct* b,
                                 const unihenn_evk* rlk, unihenn_ct* out, void* ws, size_t ws_bytes, void* stream)
{
    int rc = rotate_checks(c, a, out);
    if (rc) return rc;
    if ((rc = check_ct(c, b, "second operand"))) return rc;
    if (out->data == b->data) return uh_fail(UNIHENN_EINVAL, "output aliases input");
    if (b->batch != a->batch) return uh_fail(UNIHENN_EINVAL, "operands of different batch sizes");
    if (b->n_limbs < a->n_limbs) return uh_fail(UNIHENN_ELEVEL, "second operand has fewer limbs than the first");
    const int nl = (int)a->n_limbs, B = (int)a->batch;
    if ((rc = check_key(c, rlk, nl))) return rc;
    if ((rc = check_ws(c, nl, B, ws_bytes, ws))) return rc;
    hipStream_t s = (hipStream_t)stream;
    KsWs w = ks_ws_carve((u64*)ws, nl, B, c->n);
    u64* d0 = w.aux;
    u64* d1 = w.aux + (size_t)B * nl * c->n;
    u64* d2 = w.aux + (size_t)2 * B * nl * c->n;
    launch_tensor_mul(c, d0, d1, d2, a->data, b->data, (int)b->n_limbs, B, nl, s);
    ks_modup(c, d2, nl, B, nl, w, s);
    ks_finish(c, d2, nl, rlk->data, c->n_data, B, nl, 1, out->data, d0, d1, nl, w, s);
    out->n_limbs = a->n_limbs;
    out->batch = a->batch;
    out->scale = a->scale * b->scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" size_t unihenn_drop_level_workspace_size(const unihenn_ctx* c, uint32_t n_limbs, uint32_t batch)
{
    if (!c) return 0;
    return (ks_ws_rows((int)n_limbs, (int)batch) + (size_t)4 * batch * n_limbs) * c->n * sizeof(u64);
}

// Drop-Level as Section IV-A states it: n_ones products with encryptions of
// all-ones vectors, each relinearised and rescaled (one level each).  The
// workspace holds the key-switch scratch, the product t and the running
// value x, which alternate so that no launch reads what it writes.
extern "C" int unihenn_drop_level(const unihenn_ctx* c, const unihenn_ct* in, const unihenn_ct* ones,
                                  uint32_t n_ones, const unihenn_evk* rlk, unihenn_ct* out, void* ws, size_t ws_bytes,
                                  void* stream)
{
    int rc = rotate_checks(c, in, out);
    if (rc) return rc;
    if (n_ones < 1 || n_ones >= in->n_limbs) return uh_fail(UNIHENN_ELEVEL, "drop count must be in 1 .. limbs - 1");
    if (!ones) return uh_fail(UNIHENN_EINVAL, "null all-ones ciphertexts");
    const int nl0 = (int)in->n_limbs, B = (int)in->batch;
    for (uint32_t k = 0; k < n_ones; ++k) {
        if ((rc = check_ct(c, &ones[k], "all-ones ciphertext"))) return rc;
        if ((int)ones[k].batch != B) return uh_fail(UNIHENN_EINVAL, "all-ones ciphertext of another batch size");
        if ((int)ones[k].n_limbs < nl0 - (int)k)
            return uh_fail(UNIHENN_ELEVEL, "all-ones ciphertext " + std::to_string(k) + " below its product's level");
        if (ones[k].data == out->data) return uh_fail(UNIHENN_EINVAL, "output aliases an all-ones ciphertext");
    }
    if ((rc = check_key(c, rlk, nl0))) return rc;
    const size_t need = unihenn_drop_level_workspace_size(c, (uint32_t)nl0, (uint32_t)B);
    if (!ws || ws_bytes < need) return uh_fail(UNIHENN_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    const size_t rn = (size_t)c->n;
    u64* base = (u64*)ws;
    u64* t = base + ks_ws_rows(nl0, B) * rn;       // [B][2][nl] product
    u64* x = t + (size_t)2 * B * nl0 * rn;         // [B][2][nl - 1] running value
    const u64* cur = in->data;
    double scale = in->scale;
    for (uint32_t k = 0; k < n_ones; ++k) {
        const int nl = nl0 - (int)k;
        KsWs w = ks_ws_carve(base, nl, B, c->n);
        u64* d0 = w.aux;
        u64* d1 = w.aux + (size_t)B * nl * rn;
        u64* d2 = w.aux + (size_t)2 * B * nl * rn;
        launch_tensor_mul(c, d0, d1, d2, cur, ones[k].data, (int)ones[k].n_limbs, B, nl, s);
        ks_modup(c, d2, nl, B, nl, w, s);
        ks_finish(c, d2, nl, rlk->data, c->n_data, B, nl, 1, t, d0, d1, nl, w, s);
        u64* dst = k + 1 == n_ones ? out->data : x;
        rescale_core(c, t, B, nl, dst, w, s);
        cur = dst;
        scale = scale * ones[k].scale / (double)c->primes[nl - 1];
    }
    out->n_limbs = in->n_limbs - n_ones;
    out->batch = in->batch;
    out->scale = scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_square_relin(const unihenn_ctx* c, const unihenn_ct* in, const unihenn_evk* rlk,
                                    unihenn_ct* out, void* ws, size_t ws_bytes, void* stream)
{
    int rc = rotate_checks(c, in, out);
    if (rc) return rc;
    const int nl = (int)in->n_limbs, B = (int)in->batch;
    if ((rc = check_key(c, rlk, nl))) return rc;
    if ((rc = check_ws(c, nl, B, ws_bytes, ws))) return rc;
    hipStream_t s = (hipStream_t)stream;
    KsWs w = ks_ws_carve((u64*)ws, nl, B, c->n);
    u64* d0 = w.aux;
    u64* d1 = w.aux + (size_t)B * nl * c->n;
    u64* d2 = w.aux + (size_t)2 * B * nl * c->n;
    launch_tensor_square(c, d0, d1, d2, in->data, B, nl, s);
    ks_modup(c, d2, nl, B, nl, w, s);
    ks_finish(c, d2, nl, rlk->data, c->n_data, B, nl, 1, out->data, d0, d1, nl, w, s);
    out->n_limbs = in->n_limbs;
    out->batch = in->batch;
    out->scale = in->scale * in->scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_add(const unihenn_ctx* c, const unihenn_ct* a, const unihenn_ct* b, unihenn_ct* out,
                           void* stream)
{
    int rc = check_ct(c, a, "a");
    if (rc || (rc = check_ct(c, b, "b"))) return rc;
    if (!out || !out->data) return uh_fail(UNIHENN_EINVAL, "null output");
    if (a->n_limbs != b->n_limbs) return uh_fail(UNIHENN_ELEVEL, "operands at different levels");
    if (a->batch != b->batch) return uh_fail(UNIHENN_EINVAL, "operands with different batch sizes");
    if (a->scale != b->scale) return uh_fail(UNIHENN_ESCALE, "operands at different scales");
    launch_add(c, out->data, a->data, b->data, (int)(a->batch * 2 * a->n_limbs), (int)a->n_limbs,
               (hipStream_t)stream);
    out->n_limbs = a->n_limbs;
    out->batch = a->batch;
    out->scale = a->scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_add_plain(const unihenn_ctx* c, const unihenn_ct* a, const uint64_t* pt, unihenn_ct* out,
                                 void* stream)
{
    int rc = check_ct(c, a, "a");
    if (rc) return rc;
    if (!pt || !out || !out->data) return uh_fail(UNIHENN_EINVAL, "null argument");
    launch_add_plain(c, out->data, a->data, pt, (int)a->batch, (int)a->n_limbs, (hipStream_t)stream);
    out->n_limbs = a->n_limbs;
    out->batch = a->batch;
    out->scale = a->scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}

extern "C" int unihenn_mod_drop(const unihenn_ctx* c, const unihenn_ct* in, uint32_t n_limbs_out, unihenn_ct* out,
                                void* stream)
{
    int rc = check_ct(c, in, "input");
    if (rc) return rc;
    if (!out || !out->data) return uh_fail(UNIHENN_EINVAL, "null output");
    if (n_limbs_out < 1 || n_limbs_out > in->n_limbs) return uh_fail(UNIHENN_ELEVEL, "cannot raise the level");
    if (out->data == in->data && n_limbs_out != in->n_limbs) return uh_fail(UNIHENN_EINVAL, "output aliases input");
    const int B = (int)in->batch;
    launch_gather_rows(c, out->data, in->data, B * 2 * (int)n_limbs_out, (int)n_limbs_out, (int)in->n_limbs, 0,
                       (hipStream_t)stream);
    out->n_limbs = n_limbs_out;
    out->batch = in->batch;
    out->scale = in->scale;
    UH_LAUNCH_CHECK();
    return UNIHENN_OK;
}
