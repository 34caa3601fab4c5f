// Elementwise kernels of the key-switching, rescaling and multiply-accumulate
// path.  Every kernel is memory-streaming over limb rows of N words; threads
// map to consecutive coefficients so each wavefront touches 512 contiguous
// bytes of a row.
#include <cstring>
#include <vector>

#include "kernels.h"

namespace {

constexpr int EW_THREADS = 256;

// Consecutive hardware workgroup ids are dealt to the 8 XCDs in turn (each
// with its own L2).  For a 1D grid padded to a multiple of 8, hardware id w
// runs logical workgroup (w mod 8) * (grid / 8) + w / 8, so every XCD holds a
// contiguous logical range; kernels order their logical index with the
// dimension whose workgroups share input rows fastest.  Returns -1 for the
// padding workgroups.
constexpr int UH_XCDS = 8;
__device__ __forceinline__ int xcd_logical(int W)
{
    const int wp = (int)gridDim.x, w = (int)blockIdx.x;
    const int L = (w % UH_XCDS) * (wp / UH_XCDS) + w / UH_XCDS;
    return L < W ? L : -1;
}

inline unsigned xcd_grid(long W) { return (unsigned)((W + UH_XCDS - 1) / UH_XCDS * UH_XCDS); }

// Key-switch inner products: split the batch into Zb chunks so that a
// launch has about min_wg workgroups (8 per CU by default); the chunks of one
// (coefficient chunk, target limb, rotation) share its key rows.
inline void inner_split(long C, int T, int E, int batch, int min_wg, int* bb, int* zb)
{
    int z = 1;
    while (C * T * E * z < min_wg && z < batch) z *= 2;
    *bb = (batch + z - 1) / z;
    *zb = (batch + *bb - 1) / *bb;
}

__global__ void k_automorphism(u64* __restrict__ out, const u64* __restrict__ in, int log_n, u32 g)
{
    const int n = 1 << log_n;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= (u32)n) return;
    const size_t row = blockIdx.y;
    out[row * n + k] = in[row * n + auto_perm(k, g, log_n)];
}

// digits of the ModUp: out[b][j][s] = centered([d]_{q_j}) mod q_t, t = s < j ? s : s+1 (t = n: P)
__global__ void k_modup(u64* __restrict__ out, const u64* __restrict__ dcoef, DevCtx ctx, const u64* __restrict__ qmod,
                        int nl, int n_mod)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // (b * nl + j) * nl + s
    const int s = r % nl, j = (r / nl) % nl, b = r / (nl * nl);
    const int t = s < j ? s : s + 1;
    const int tm = t == nl ? ctx.p_index : t;
    const Modulus mt = ctx.mod[tm];
    const u64 x = dcoef[((size_t)b * nl + j) * n + k];
    out[(size_t)r * n + k] = centered_lift(x, ctx.mod[j].half, qmod[(size_t)j * n_mod + tm], mt.q, mt.ratio);
}

// U_c[t] = sum_j D_j[t] (*) evk_{j,c}[t] over t in {q_0..q_{nl-1}, P}.  D_j[j]
// is limb j of the NTT-form input itself; the other targets come from the
// ModUp rows.  With g != 1 the digits are read through the automorphism
// permutation (hoisted rotation).  The thread keeps its 2 nl key words in
// registers and loops over the batch.
template <int MAXL>
__global__ void __launch_bounds__(EW_THREADS) k_ks_inner(u64* __restrict__ U, u64* __restrict__ Up,
                                                         const u64* __restrict__ dntt, int d_stride,
                                                         const u64* __restrict__ modup, const u64* __restrict__ key,
                                                         DevCtx ctx, int nl, int nd, int batch, u32 g, int BB, int Zb,
                                                         int C, int W)
{
    const int L = xcd_logical(W);
    if (L < 0) return;
    const int zb = L % Zb;
    const int x = (L / Zb) % C;
    const int t = L / (Zb * C);  // 0..nl
    const int n = ctx.n;
    const int k = x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int b_lo = zb * BB, b_hi = min(batch, b_lo + BB);
    const int tm = t == nl ? ctx.p_index : t;
    const int klimb = t == nl ? nd : t;
    const Modulus M = ctx.mod[tm];
    const int period = wide_period(M.ratio);
    const u32 src = g == 1 ? (u32)k : auto_perm((u32)k, g, ctx.log_n);
    u64 k0[MAXL], k1[MAXL];
#pragma unroll
    for (int j = 0; j < MAXL; ++j) {
        if (j < nl) {
            k0[j] = key[(((size_t)j * 2 + 0) * (nd + 1) + klimb) * n + k];
            k1[j] = key[(((size_t)j * 2 + 1) * (nd + 1) + klimb) * n + k];
        }
    }
    // entry b + 1's digits load while entry b's products run
    u64 dn[MAXL] = {};
    auto fetch = [&](int b) {
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < nl) {
                if (t == j) {
                    dn[j] = dntt[((size_t)b * d_stride + j) * n + src];
                } else {
                    const int s = t < j ? t : t - 1;
                    dn[j] = modup[(((size_t)b * nl + j) * nl + s) * n + src];
                }
            }
        }
    };
    if (b_lo < b_hi) fetch(b_lo);
    for (int b = b_lo; b < b_hi; ++b) {
        WideAcc a0, a1;
        wide_init(a0, 0);
        wide_init(a1, 0);
        int since = 0;
        u64 dc[MAXL];
#pragma unroll
        for (int j = 0; j < MAXL; ++j) dc[j] = dn[j];
        if (b + 1 < b_hi) fetch(b + 1);
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < nl) {
                const u64 d = dc[j];
                wide_mac(a0, d, k0[j]);
                wide_mac(a1, d, k1[j]);
                if (++since == period) {
                    wide_fold(a0, M.q, M.qinv_neg);
                    wide_fold(a1, M.q, M.qinv_neg);
                    since = 0;
                }
            }
        }
        const u64 r0 = wide_redc(a0, M.q, M.qinv_neg), r1 = wide_redc(a1, M.q, M.qinv_neg);
        if (t < nl) {
            U[(((size_t)b * 2 + 0) * nl + t) * n + k] = r0;
            U[(((size_t)b * 2 + 1) * nl + t) * n + k] = r1;
        } else {
            Up[((size_t)b * 2 + 0) * n + k] = r0;
            Up[((size_t)b * 2 + 1) * n + k] = r1;
        }
    }
}

// out[row = p * nl + i] = centered(src[p]) mod q_i, src rows in the modulus
// src_mod (P for ModDown, q_l for rescale)
__global__ void k_lift_last(u64* __restrict__ out, const u64* __restrict__ src, DevCtx ctx,
                            const u64* __restrict__ qmod, int n_mod, int nl, int src_mod)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;
    const int i = r % nl, p = r / nl;
    const Modulus mi = ctx.mod[i];
    out[(size_t)r * n + k] = centered_lift(src[(size_t)p * n + k], ctx.mod[src_mod].half,
                                           qmod[(size_t)src_mod * n_mod + i], mi.q, mi.ratio);
}

// out[p][i] = (x[p][i] - r[p][i]) * inv_i (+ add_c[b][i]),  p = b * 2 + c,
// x rows have stride x_limbs per polynomial, out and r have nl.
__global__ void k_sub_scale(u64* __restrict__ out, const u64* __restrict__ x, int x_limbs, const u64* __restrict__ r,
                            const u64* __restrict__ inv, DevCtx ctx, int nl, const u64* __restrict__ add0,
                            const u64* __restrict__ add1, int add_stride)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int row = blockIdx.y;
    const int i = row % nl, p = row / nl;
    const int b = p >> 1, c = p & 1;
    const u64 q = ctx.mod[i].q;
    u64 v = sub_mod(x[((size_t)p * x_limbs + i) * n + k], r[(size_t)row * n + k], q);
    v = mul_shoup(v, inv[2 * i], inv[2 * i + 1], q);
    const u64* add = c == 0 ? add0 : add1;
    if (add) v = add_mod(v, add[((size_t)b * add_stride + i) * n + k], q);
    out[(size_t)row * n + k] = v;
}

// dst row r <- src row (r / per) * src_stride + r % per + off
__global__ void k_gather_rows(u64* __restrict__ dst, const u64* __restrict__ src, int n, int per, int src_stride,
                              int off)
{
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;
    const size_t sr = (size_t)(r / per) * src_stride + r % per + off;
    dst[(size_t)r * n + k] = src[sr * n + k];
}

template <int BCH>
__global__ void __launch_bounds__(EW_THREADS) k_mac(u64* __restrict__ acc, MacTerms terms, int n_terms, DevCtx ctx,
                                                    int nl, int batch, int accumulate, int pl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int i = blockIdx.y;
    const int b0 = blockIdx.z * BCH;
    const Modulus M = ctx.mod[i == pl ? ctx.p_index : i];
    const int period = wide_period(M.ratio);
    WideAcc a[2 * BCH];
#pragma unroll
    for (int u = 0; u < 2 * BCH; ++u) {
        const int b = b0 + u / 2, c = u & 1;
        wide_init(a[u], (accumulate && b < batch) ? acc[(((size_t)b * 2 + c) * nl + i) * n + k] : 0);
    }
    // term t + 1's words load while term t's products run
    u64 pn = 0, vn[2 * BCH];
    auto fetch = [&](int t) {
        pn = terms.pt[t][(size_t)i * n + k];
        const u64* ct = terms.ct[t];
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) {
            const int b = b0 + u / 2, c = u & 1;
            vn[u] = b < batch ? ct[(((size_t)b * 2 + c) * nl + i) * n + k] : 0;
        }
    };
    if (n_terms > 0) fetch(0);
    int since = 0;
    for (int t = 0; t < n_terms; ++t) {
        const u64 p = pn;
        u64 v[2 * BCH];
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) v[u] = vn[u];
        if (t + 1 < n_terms) fetch(t + 1);
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) wide_mac(a[u], p, v[u]);
        if (++since == period) {
#pragma unroll
            for (int u = 0; u < 2 * BCH; ++u) wide_fold(a[u], M.q, M.qinv_neg);
            since = 0;
        }
    }
#pragma unroll
    for (int u = 0; u < 2 * BCH; ++u) {
        const int b = b0 + u / 2, c = u & 1;
        if (b < batch) acc[(((size_t)b * 2 + c) * nl + i) * n + k] = wide_redc(a[u], M.q, M.qinv_neg);
    }
}

// (c0, c1) -> d0 = c0^2, d1 = 2 c0 c1, d2 = c1^2, each [B][nl][N]
__global__ void k_tensor_square(u64* __restrict__ d0, u64* __restrict__ d1, u64* __restrict__ d2,
                                const u64* __restrict__ ct, DevCtx ctx, int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // b * nl + i
    const int i = r % nl, b = r / nl;
    const Modulus M = ctx.mod[i];
    const u64 c0 = ct[(((size_t)b * 2 + 0) * nl + i) * n + k];
    const u64 c1 = ct[(((size_t)b * 2 + 1) * nl + i) * n + k];
    // x y = mont(mont(x, y), 2^128 mod q)
    const u64 s00 = mont_mul(mont_mul(c0, c0, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    const u64 s01 = mont_mul(mont_mul(c0, c1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    const u64 s11 = mont_mul(mont_mul(c1, c1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    d0[(size_t)r * n + k] = s00;
    d1[(size_t)r * n + k] = add_mod(s01, s01, M.q);
    d2[(size_t)r * n + k] = s11;
}

// out = a + b over rows with modulus = row % nl
__global__ void k_add(u64* __restrict__ out, const u64* __restrict__ a, const u64* __restrict__ b, DevCtx ctx, int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const size_t r = blockIdx.y;
    const u64 q = ctx.mod[r % nl].q;
    out[r * n + k] = add_mod(a[r * n + k], b[r * n + k], q);
}

// c0 of every ciphertext += pt ([nl][N]); c1 copied when out != a
__global__ void k_add_plain(u64* __restrict__ out, const u64* __restrict__ a, const u64* __restrict__ pt, DevCtx ctx,
                            int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // (b * 2 + c) * nl + i
    const int i = r % nl, c = (r / nl) & 1;
    const u64 q = ctx.mod[i].q;
    u64 v = a[(size_t)r * n + k];
    if (c == 0) v = add_mod(v, pt[(size_t)i * n + k], q);
    out[(size_t)r * n + k] = v;
}

// x -> x 2^64 mod q (to_mont) or x 2^-64 mod q (from_mont), modulus by row map
__global__ void k_mont_convert(u64* __restrict__ data, DevCtx ctx, RowMap map, int to_mont)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const size_t r = blockIdx.y;
    const Modulus M = ctx.mod[rowmap_mod(map, (int)r)];
    const u64 x = data[r * n + k];
    data[r * n + k] = mont_mul(x, to_mont ? M.r2 : 1, M.q, M.qinv_neg);
}

inline dim3 grid_rows(int n, int rows, int z = 1) { return dim3((n + EW_THREADS - 1) / EW_THREADS, rows, z); }

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_automorphism(const unihenn_ctx* c, u64* out, const u64* in, int rows, u32 g, hipStream_t s)
{
    if (rows <= 0) return;
    LaunchTimer tm(KF_AUTO, 16.0 * c->n * rows, s);
    k_automorphism<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(out, in, c->log_n, g);
}

void launch_modup(const unihenn_ctx* c, u64* out, const u64* dcoef, int batch, int nl, hipStream_t s)
{
    int rows = batch * nl * nl;
    LaunchTimer tm(KF_MODUP, 8.0 * c->n * (batch * nl + rows), s);
    k_modup<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(out, dcoef, c->dev, c->d_qmod, nl,
                                                         (int)c->primes.size());
}

void launch_ks_inner(const unihenn_ctx* c, u64* U, u64* Up, const u64* dntt, int d_stride, const u64* modup,
                     const u64* key, int nd, int batch, int nl, u32 g, hipStream_t s)
{
    // algorithmic bytes: key limbs (2 nl (nl+1)), digits (nl (nl+1) per ct), output 2 (nl+1) per ct
    double rows = 2.0 * nl * (nl + 1) + (double)batch * (nl * (nl + 1) + 2 * (nl + 1));
    LaunchTimer tm(KF_KS_INNER, 8.0 * c->n * rows, s);
    const int C = (c->n + EW_THREADS - 1) / EW_THREADS;
    int bb, zb;
    inner_split(C, nl + 1, 1, batch, c->ks_min_wg, &bb, &zb);
    const int W = zb * C * (nl + 1);
    const unsigned gx = xcd_grid(W);
#define KSI(M) k_ks_inner<M><<<gx, EW_THREADS, 0, s>>>(U, Up, dntt, d_stride, modup, key, c->dev, nl, nd, batch, g, \
                                                       bb, zb, C, W)
    if (nl <= 4) KSI(4);
    else if (nl <= 8) KSI(8);
    else if (nl <= 12) KSI(12);
    else KSI(UH_MAX_MODULI);
#undef KSI
}

void launch_lift_last(const unihenn_ctx* c, u64* out, const u64* src, int n_src_rows, int nl, int src_mod,
                      KernelFamily fam, hipStream_t s)
{
    int rows = n_src_rows * nl;
    LaunchTimer tm(fam, 8.0 * c->n * (n_src_rows + rows), s);
    k_lift_last<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(out, src, c->dev, c->d_qmod, (int)c->primes.size(), nl,
                                                             src_mod);
}

void launch_sub_scale(const unihenn_ctx* c, u64* out, const u64* x, int x_limbs, const u64* r, const u64* inv,
                      int n_polys, int nl, const u64* add0, const u64* add1, int add_stride, KernelFamily fam,
                      hipStream_t s)
{
    int rows = n_polys * nl;
    LaunchTimer tm(fam, 8.0 * c->n * rows * (3 + (add0 ? 0.5 : 0) + (add1 ? 0.5 : 0)), s);
    k_sub_scale<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(out, x, x_limbs, r, inv, c->dev, nl, add0, add1, add_stride);
}

void launch_gather_rows(const unihenn_ctx* c, u64* dst, const u64* src, int rows, int per, int src_stride, int off,
                        hipStream_t s)
{
    if (rows <= 0) return;
    LaunchTimer tm(KF_OTHER, 16.0 * c->n * rows, s);
    k_gather_rows<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(dst, src, c->n, per, src_stride, off);
}

void launch_mac(const unihenn_ctx* c, u64* acc, const MacTerms& terms, int n_terms, int nl, int batch, int accumulate,
                hipStream_t s, int pl)
{
    // algorithmic bytes: plaintexts once, ciphertexts once, acc written (and read when accumulating)
    double rows = (double)n_terms * nl + (double)n_terms * batch * 2 * nl + (1 + accumulate) * batch * 2.0 * nl;
    LaunchTimer tm(KF_MAC, 8.0 * c->n * rows, s);
    if (batch >= 4) {
        k_mac<4><<<grid_rows(c->n, nl, (batch + 3) / 4), EW_THREADS, 0, s>>>(acc, terms, n_terms, c->dev, nl, batch,
                                                                             accumulate, pl);
    } else {
        k_mac<1><<<grid_rows(c->n, nl, batch), EW_THREADS, 0, s>>>(acc, terms, n_terms, c->dev, nl, batch,
                                                                   accumulate, pl);
    }
}

// (a0, a1) x (b0, b1) -> d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1, each
// [B][nl][N]; b rows have b_limbs limbs per polynomial (its first nl used)
__global__ void k_tensor_mul(u64* __restrict__ d0, u64* __restrict__ d1, u64* __restrict__ d2,
                             const u64* __restrict__ a, const u64* __restrict__ bct, int b_limbs, DevCtx ctx, int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // b * nl + i
    const int i = r % nl, b = r / nl;
    const Modulus M = ctx.mod[i];
    const u64 a0 = a[(((size_t)b * 2 + 0) * nl + i) * n + k];
    const u64 a1 = a[(((size_t)b * 2 + 1) * nl + i) * n + k];
    const u64 b0 = bct[(((size_t)b * 2 + 0) * b_limbs + i) * n + k];
    const u64 b1 = bct[(((size_t)b * 2 + 1) * b_limbs + i) * n + k];
    const u64 s00 = mont_mul(mont_mul(a0, b0, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    const u64 s01 = mont_mul(mont_mul(a0, b1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    const u64 s10 = mont_mul(mont_mul(a1, b0, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    const u64 s11 = mont_mul(mont_mul(a1, b1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    d0[(size_t)r * n + k] = s00;
    d1[(size_t)r * n + k] = add_mod(s01, s10, M.q);
    d2[(size_t)r * n + k] = s11;
}

void launch_tensor_mul(const unihenn_ctx* c, u64* d0, u64* d1, u64* d2, const u64* a, const u64* b, int b_limbs,
                       int batch, int nl, hipStream_t s)
{
    LaunchTimer tm(KF_TENSOR, 8.0 * c->n * batch * nl * 7, s);
    k_tensor_mul<<<grid_rows(c->n, batch * nl), EW_THREADS, 0, s>>>(d0, d1, d2, a, b, b_limbs, c->dev, nl);
}

void launch_tensor_square(const unihenn_ctx* c, u64* d0, u64* d1, u64* d2, const u64* ct, int batch, int nl,
                          hipStream_t s)
{
    LaunchTimer tm(KF_TENSOR, 8.0 * c->n * batch * nl * 5, s);
    k_tensor_square<<<grid_rows(c->n, batch * nl), EW_THREADS, 0, s>>>(d0, d1, d2, ct, c->dev, nl);
}

void launch_add(const unihenn_ctx* c, u64* out, const u64* a, const u64* b, int rows, int nl, hipStream_t s)
{
    LaunchTimer tm(KF_ADD, 24.0 * c->n * rows, s);
    k_add<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(out, a, b, c->dev, nl);
}

void launch_add_plain(const unihenn_ctx* c, u64* out, const u64* a, const u64* pt, int batch, int nl, hipStream_t s)
{
    LaunchTimer tm(KF_ADD, 8.0 * c->n * (batch * 4.0 * nl + nl), s);
    k_add_plain<<<grid_rows(c->n, batch * 2 * nl), EW_THREADS, 0, s>>>(out, a, pt, c->dev, nl);
}

void launch_mont_convert(const unihenn_ctx* c, u64* data, int rows, const RowMap& map, int to_mont, hipStream_t s)
{
    if (rows <= 0) return;
    LaunchTimer tm(KF_OTHER, 16.0 * c->n * rows, s);
    k_mont_convert<<<grid_rows(c->n, rows), EW_THREADS, 0, s>>>(data, c->dev, map, to_mont);
}

// ------------------------------------------------------------------ grouped rotations
namespace {

// aux[e][b][c][i] = tau_{g_e}(src_e)[b][c][i]; c0_only: c = 0 rows only
__global__ void k_group_auto(u64* __restrict__ aux, GroupArgs ga, int nl, int batch, int log_n, int c0_only)
{
    const int n = 1 << log_n;
    const u32 k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= (u32)n) return;
    const int e = blockIdx.z;
    const int r = blockIdx.y;  // (b * 2 + c) * nl + i  (c0_only: b * nl + i)
    int b, c, i;
    if (c0_only) { i = r % nl; b = r / nl; c = 0; }
    else { i = r % nl; c = (r / nl) & 1; b = r / (2 * nl); }
    const size_t row = ((size_t)b * 2 + c) * nl + i;
    aux[((size_t)e * batch * 2 * nl + row) * n + k] = ga.src[e][row * n + auto_perm(k, ga.g[e], log_n)];
}

// dcoef[blk][b][j] = dsrc_blk rows (b, j)
__global__ void k_group_gather(u64* __restrict__ dcoef, GroupArgs ga, int nl, int batch, int n)
{
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // b * nl + j
    const int blk = blockIdx.z;
    const int j = r % nl, b = r / nl;
    dcoef[(((size_t)blk * batch + b) * nl + j) * n + k] = ga.dsrc[blk][((size_t)b * ga.dstride + j) * n + k];
}

// Inner product of the ModUp digits with each element's key, limb t of
// {q_0..q_{nl-1}, P} per thread.  EXT = false: U [E][B][2][nl] and Up
// [E][B][2] for the ModDown that follows.  EXT = true: the extended rotation
// (P tau(c0) + U_0, U_1) straight into dst_e [B][2][nl+1] (limb nl = P),
// with tau(c0) read from src_e through the automorphism.
//
// Logical workgroup order (each XCD runs a contiguous range): order 0 varies
// the batch chunk fastest, then the coefficient chunk, the limb and the
// element (keys re-read from L2 across batch chunks); order 1 varies the
// element fastest, then the coefficient chunk, the batch chunk and the limb,
// so that the elements of a group gather the same digit rows back to back
// (digits re-read from L2 across rotations).
template <int MAXL, bool EXT>
__global__ void __launch_bounds__(EW_THREADS) k_group_inner(u64* __restrict__ U, u64* __restrict__ Up,
                                                            const u64* __restrict__ modup, GroupArgs ga, DevCtx ctx,
                                                            int nl, int nd, int batch, int BB, int Zb, int C, int W,
                                                            int order)
{
    const int L = xcd_logical(W);
    if (L < 0) return;
    int zb, x, t, e;
    if (order == 0) {
        zb = L % Zb;
        x = (L / Zb) % C;
        t = (L / (Zb * C)) % (nl + 1);  // 0..nl
        e = L / (Zb * C * (nl + 1));
    } else {
        e = L % ga.E;
        x = (L / ga.E) % C;
        zb = (L / (ga.E * C)) % Zb;
        t = L / (ga.E * C * Zb);
    }
    const int n = ctx.n;
    const int k = x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int b_lo = zb * BB, b_hi = min(batch, b_lo + BB);
    const int tm = t == nl ? ctx.p_index : t;
    const int klimb = t == nl ? nd : t;
    const Modulus M = ctx.mod[tm];
    const int period = wide_period(M.ratio);
    const u32 g = ga.gin[e], gd = ga.gdig[e];
    const u32 src = g == 1 ? (u32)k : auto_perm((u32)k, g, ctx.log_n);
    const u32 srcd = gd == 1 ? (u32)k : (gd == g ? src : auto_perm((u32)k, gd, ctx.log_n));
    const u64* __restrict__ key = ga.key[e];
    const u64* __restrict__ dsrc = ga.dsrc[ga.blk[e]];
    const int blk = ga.blk[e];
    u32 c0i = 0;
    u64 pm = 0, pm_sh = 0;
    if (EXT && t < nl) {
        c0i = auto_perm((u32)k, ga.g[e], ctx.log_n);
        pm = ctx.p_mod[2 * t];
        pm_sh = ctx.p_mod[2 * t + 1];
    }
    u64 k0[MAXL], k1[MAXL];
#pragma unroll
    for (int j = 0; j < MAXL; ++j) {
        if (j < nl) {
            k0[j] = key[(((size_t)j * 2 + 0) * (nd + 1) + klimb) * n + k];
            k1[j] = key[(((size_t)j * 2 + 1) * (nd + 1) + klimb) * n + k];
        }
    }
    // the digits of batch entry b + 1 are loaded while entry b's products
    // run, so their latency overlaps the arithmetic
    u64 dn[MAXL] = {};
    auto fetch = [&](int b) {
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < nl) {
                if (t == j) {
                    dn[j] = dsrc[((size_t)b * ga.dstride + j) * n + srcd];
                } else {
                    const int s = t < j ? t : t - 1;
                    dn[j] = modup[((((size_t)blk * batch + b) * nl + j) * nl + s) * n + src];
                }
            }
        }
    };
    if (b_lo < b_hi) fetch(b_lo);
    for (int b = b_lo; b < b_hi; ++b) {
        WideAcc a0, a1;
        wide_init(a0, 0);
        wide_init(a1, 0);
        int since = 0;
        u64 dc[MAXL];
#pragma unroll
        for (int j = 0; j < MAXL; ++j) dc[j] = dn[j];
        if (b + 1 < b_hi) fetch(b + 1);
#pragma unroll
        for (int j = 0; j < MAXL; ++j) {
            if (j < nl) {
                const u64 d = dc[j];
                wide_mac(a0, d, k0[j]);
                wide_mac(a1, d, k1[j]);
                if (++since == period) {
                    wide_fold(a0, M.q, M.qinv_neg);
                    wide_fold(a1, M.q, M.qinv_neg);
                    since = 0;
                }
            }
        }
        u64 r0 = wide_redc(a0, M.q, M.qinv_neg);
        const u64 r1 = wide_redc(a1, M.q, M.qinv_neg);
        if (EXT) {
            u64* __restrict__ dst = ga.dst[e];
            const size_t base = (size_t)b * 2 * (nl + 1);
            if (t < nl) {
                const u64 x = ga.src[e][((size_t)b * 2 * nl + t) * n + c0i];
                r0 = add_mod(r0, mul_shoup(x, pm, pm_sh, M.q), M.q);
            }
            dst[(base + t) * n + k] = r0;
            dst[(base + nl + 1 + t) * n + k] = r1;
            continue;
        }
        const size_t eb = (size_t)e * batch + b;
        if (t < nl) {
            U[((eb * 2 + 0) * nl + t) * n + k] = r0;
            U[((eb * 2 + 1) * nl + t) * n + k] = r1;
        } else {
            Up[(eb * 2 + 0) * n + k] = r0;
            Up[(eb * 2 + 1) * n + k] = r1;
        }
    }
}

// dst_e[b][c][i] = (U - R) P^-1 (+ aux c0 on c = 0)
__global__ void k_group_sub_scale(GroupArgs ga, const u64* __restrict__ U, const u64* __restrict__ R,
                                  const u64* __restrict__ aux, const u64* __restrict__ inv, DevCtx ctx, int nl,
                                  int batch)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // (b * 2 + c) * nl + i
    const int e = blockIdx.z;
    const int i = r % nl, c = (r / nl) & 1, b = r / (2 * nl);
    const u64 q = ctx.mod[i].q;
    const size_t row = (size_t)e * batch * 2 * nl + r;
    u64 v = sub_mod(U[row * n + k], R[row * n + k], q);
    v = mul_shoup(v, inv[2 * i], inv[2 * i + 1], q);
    if (c == 0) v = add_mod(v, aux[(((size_t)e * batch + b) * 2 * nl + i) * n + k], q);
    ga.dst[e][(size_t)r * n + k] = v;
}

}  // namespace

bool group_modup(const unihenn_ctx* c, int D, const u64* const* dsrc, int dstride, int B, int nl, u64* dcoef,
                 u64* modup, hipStream_t s, const u32* perm, bool row_pass)
{
    if (ntt_fusable(c)) {
        const bool skip = !row_pass && ks_rowfusable(c, nl, D * B);
        // the inverse NTT gathers (and permutes) its rows, the forward NTT lifts them
        GatherArgs gta;
        memset(&gta, 0, sizeof(gta));
        for (int d = 0; d < D; ++d) {
            gta.src[d] = dsrc[d];
            gta.perm[d] = perm ? perm[d] : 1u;
        }
        gta.stride = dstride;
        if (launch_ntt_inv_gather(c, dcoef, gta, D, B, nl, s) &&
            launch_ntt_fwd_modup(c, modup, dcoef, D * B * nl, nl, s, !skip))
            return skip;
    }
    GroupArgs ga;
    memset(&ga, 0, sizeof(ga));
    for (int d = 0; d < D; ++d) ga.dsrc[d] = dsrc[d];
    ga.dstride = dstride;
    {
        LaunchTimer tm(KF_OTHER, 16.0 * c->n * D * B * nl, s);
        dim3 g3((c->n + EW_THREADS - 1) / EW_THREADS, B * nl, D);
        k_group_gather<<<g3, EW_THREADS, 0, s>>>(dcoef, ga, nl, B, c->n);
    }
    launch_ntt_inv(c, dcoef, D * B * nl, rowmap_ct(nl), s);
    if (launch_ntt_fwd_modup(c, modup, dcoef, D * B * nl, nl, s)) return false;
    launch_modup(c, modup, dcoef, D * B, nl, s);
    launch_ntt_fwd(c, modup, D * B * nl * nl, rowmap_modup(nl, c->n_data), s);
    return false;
}

namespace {
template <bool EXT>
void launch_group_inner(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, const u64* modup, u64* U, u64* Up,
                        hipStream_t s)
{
    const int E = ga.E;
    const unsigned gx = (c->n + EW_THREADS - 1) / EW_THREADS;
    // keys, digits, the outputs (and the c0 rows of the sources when extended)
    double rows = (double)E * 2.0 * nl * (nl + 1) + (double)E * B * (nl * (nl + 1) + 2 * (nl + 1) + (EXT ? nl : 0));
    LaunchTimer tm(KF_KS_INNER, 8.0 * c->n * rows, s);
    int bb, zb;
    inner_split((long)gx, nl + 1, E, B, c->ks_min_wg, &bb, &zb);
    const int W = zb * (int)gx * (nl + 1) * E;
    const unsigned gw = xcd_grid(W);
#define GI(M)                                                                                                  \
    k_group_inner<M, EXT><<<gw, EW_THREADS, 0, s>>>(U, Up, modup, ga, c->dev, nl, c->n_data, B, bb, zb, (int)gx, W, \
                                                    c->ks_order == 1 ? 1 : 0)
    if (nl <= 4) GI(4);
    else if (nl <= 8) GI(8);
    else if (nl <= 12) GI(12);
    else GI(UH_MAX_MODULI);
#undef GI
}
}  // namespace

void group_switch_ext(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, const u64* modup, hipStream_t s,
                      bool row_fused)
{
    if (row_fused) launch_ks_rowfused(c, ga, B, nl, modup, nullptr, nullptr, true, s);
    else launch_group_inner<true>(c, ga, B, nl, modup, nullptr, nullptr, s);
}

void group_switch(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, bool c0_only, const u64* modup, u64* aux,
                  u64* U, u64* Up, u64* R, hipStream_t s, bool row_fused)
{
    const int E = ga.E;
    const unsigned gx = (c->n + EW_THREADS - 1) / EW_THREADS;
    if (row_fused) launch_ks_rowfused(c, ga, B, nl, modup, U, Up, false, s);
    else launch_group_inner<false>(c, ga, B, nl, modup, U, Up, s);
    launch_ntt_inv(c, Up, E * B * 2, rowmap_list({c->n_data}), s);
    {
        // the c0 addend: tau(c0) read straight from the source (c0_only), or
        // the automorphism already in aux
        FuseArgs fa;
        memset(&fa, 0, sizeof(fa));
        fa.src = Up;
        fa.src_mod = c->n_data;
        fa.nl = nl;
        fa.polys = B * 2;
        fa.x_limbs = nl;
        fa.add_stride = 2 * nl;
        fa.inv = c->d_p_inv;
        const size_t per = (size_t)B * 2 * nl * c->n;
        // reading c0 from the sources while other workgroups write the
        // destinations needs the two sets of buffers to be disjoint
        bool disjoint = true;
        for (int e = 0; e < E && c0_only; ++e)
            for (int f = 0; f < E; ++f)
                if (ga.dst[e] < ga.src[f] + per && ga.src[f] < ga.dst[e] + per) disjoint = false;
        for (int e = 0; e < E; ++e) {
            fa.x[e] = U + e * per;
            fa.out[e] = ga.dst[e];
            fa.add[e][0] = c0_only ? ga.src[e] : aux + e * per;
            fa.add_perm[e] = c0_only ? ga.g[e] : 1u;
        }
        if (disjoint && launch_ntt_fwd_fused(c, R, fa, E * B * 2 * nl, KF_MODDOWN, s)) return;
    }
    if (c0_only) {
        LaunchTimer tm(KF_AUTO, 16.0 * c->n * E * B * nl, s);
        dim3 g3(gx, B * nl, E);
        k_group_auto<<<g3, EW_THREADS, 0, s>>>(aux, ga, nl, B, c->log_n, 1);
    }
    launch_lift_last(c, R, Up, E * B * 2, nl, c->n_data, KF_MODDOWN, s);
    launch_ntt_fwd(c, R, E * B * 2 * nl, rowmap_ct(nl), s);
    {
        LaunchTimer tm(KF_MODDOWN, 8.0 * c->n * E * B * 2 * nl * 3.5, s);
        dim3 g3(gx, B * 2 * nl, E);
        k_group_sub_scale<<<g3, EW_THREADS, 0, s>>>(ga, U, R, aux, c->d_p_inv, c->dev, nl, B);
    }
}

void group_auto_both(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, u64* aux, hipStream_t s)
{
    LaunchTimer tm(KF_AUTO, 16.0 * c->n * ga.E * B * 2 * nl, s);
    dim3 g3((c->n + EW_THREADS - 1) / EW_THREADS, B * 2 * nl, ga.E);
    k_group_auto<<<g3, EW_THREADS, 0, s>>>(aux, ga, nl, B, c->log_n, 0);
}

// ------------------------------------------------------------------ multi-output MAC
// acc[o][b] (+)= sum_t pt(o, t) (*) ct[t][b] for every coefficient k and limb i:
// per (i, k) a small product of an n_out x n_terms plaintext matrix and an
// n_terms x 2B ciphertext matrix.  A thread owns OPT outputs x BCH batch
// entries (2 OPT BCH accumulators) of one (i, k); the output groups g and
// batch chunks z that share a (k-chunk, limb) read the same ciphertext rows
// (across g) and the same plaintext rows (across z).
//
// Workgroup numbering is XCD-aware: consecutive hardware workgroup ids go to
// the 8 XCDs in turn, so hardware id w runs logical workgroup
// (w mod 8) * (W / 8) + w / 8.  Each XCD then holds a contiguous logical range
// in which (g, z) vary fastest, and the rows shared across g and z are
// re-read from that XCD's L2 rather than from HBM.
namespace {
template <int OPT, int BCH>
__global__ void __launch_bounds__(EW_THREADS) k_mac_multi(MacMulti m, int n_out, int n_terms, DevCtx ctx, int nl,
                                                          int batch, int accumulate, int G, int Z, int C, int W,
                                                          int pl)
{
    const int L = xcd_logical(W);
    if (L < 0) return;
    const int g = L % G;
    const int z = (L / G) % Z;
    const int x = (L / (G * Z)) % C;
    const int i = L / (G * Z * C);
    const int n = ctx.n;
    const int k = x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int o0 = g * OPT, b0 = z * BCH;
    const Modulus M = ctx.mod[i == pl ? ctx.p_index : i];
    const int period = wide_period(M.ratio);
    WideAcc a[OPT][2 * BCH];
#pragma unroll
    for (int o = 0; o < OPT; ++o)
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) {
            const int b = b0 + u / 2, c = u & 1;
            wide_init(a[o][u], (accumulate && o0 + o < n_out && b < batch)
                                   ? m.acc[o0 + o][(((size_t)b * 2 + c) * nl + i) * n + k] : 0);
        }
    const size_t row = (size_t)nl * n;
    // Terms go in chunks of UNR whose loads are all issued before their
    // products, so that a thread with few accumulators still keeps several
    // rows in flight (the one-image MAC is bound by plaintext reads; each
    // plaintext word is read once, so those loads are non-temporal).  A fold
    // comes before any chunk that would take the products since the last one
    // past the period.
    constexpr int UNR = OPT * BCH <= 2 ? 4 : (OPT * BCH <= 4 ? 2 : 1);
    int since = 0;
    for (int t0 = 0; t0 < n_terms; t0 += UNR) {
        const int nt = n_terms - t0 < UNR ? n_terms - t0 : UNR;
        if (since + nt > period) {
#pragma unroll
            for (int o = 0; o < OPT; ++o)
#pragma unroll
                for (int u = 0; u < 2 * BCH; ++u) wide_fold(a[o][u], M.q, M.qinv_neg);
            since = 0;
        }
        u64 v[UNR][2 * BCH], p[UNR][OPT];
#pragma unroll
        for (int h = 0; h < UNR; ++h) {
            const int t = t0 + h;
            const bool live = h < nt;
#pragma unroll
            for (int u = 0; u < 2 * BCH; ++u) {
                const int b = b0 + u / 2, c = u & 1;
                v[h][u] = live && b < batch ? m.ct[t][(((size_t)b * 2 + c) * nl + i) * n + k] : 0;
            }
            const u64* p0 = m.pt_base + (size_t)(m.t_off + t) * row + (size_t)i * n + k;
#pragma unroll
            for (int o = 0; o < OPT; ++o)
                p[h][o] = live && o0 + o < n_out
                              ? __builtin_nontemporal_load(p0 + (size_t)(o0 + o) * m.o_stride * row) : 0;
        }
#pragma unroll
        for (int h = 0; h < UNR; ++h) {
            if (h < nt) {
#pragma unroll
                for (int o = 0; o < OPT; ++o)
#pragma unroll
                    for (int u = 0; u < 2 * BCH; ++u) wide_mac(a[o][u], p[h][o], v[h][u]);
            }
        }
        since += nt;
    }
#pragma unroll
    for (int o = 0; o < OPT; ++o)
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) {
            const int b = b0 + u / 2, c = u & 1;
            if (o0 + o < n_out && b < batch)
                m.acc[o0 + o][(((size_t)b * 2 + c) * nl + i) * n + k] = wide_redc(a[o][u], M.q, M.qinv_neg);
        }
}

template <int OPT, int BCH>
void launch_mm(const MacMulti& m, int n_out, int n_terms, DevCtx dev, int nl, int batch, int accumulate, int G,
               int Z, int C, int pl, hipStream_t s)
{
    const int W = G * Z * C * nl;
    k_mac_multi<OPT, BCH><<<xcd_grid(W), EW_THREADS, 0, s>>>(m, n_out, n_terms, dev, nl, batch, accumulate, G, Z, C, W,
                                                              pl);
}
}  // namespace

// Outputs per thread and batch entries per thread: at most 32 accumulators,
// and enough workgroups (min_wg, about 8 per CU by default) to keep the
// memory system busy.
void mac_multi_shape(int n_out, int nl, int batch, int n, int min_wg, int* opt, int* bch)
{
    const int b = batch >= 4 ? 4 : (batch >= 2 ? 2 : 1);
    int o = 16 / b;
    const long C = (n + EW_THREADS - 1) / EW_THREADS;
    const long Z = (batch + b - 1) / b;
    while (o > 1 && (long)((n_out + o - 1) / o) * Z * C * nl < min_wg) o /= 2;
    while (o > 1 && o / 2 >= n_out) o /= 2;
    *opt = o;
    *bch = b;
}

void launch_mac_multi(const unihenn_ctx* c, const MacMulti& m, int n_out, int n_terms, int nl, int batch,
                      int accumulate, hipStream_t s, int pl)
{
    // algorithmic bytes: each term ciphertext once, each plaintext once, outputs written (read when accumulating)
    double rows = (double)n_terms * batch * 2 * nl + (double)n_out * n_terms * nl +
                  (1.0 + accumulate) * n_out * batch * 2 * nl;
    LaunchTimer tm(KF_MAC, 8.0 * c->n * rows, s);
    int opt, bch;
    mac_multi_shape(n_out, nl, batch, c->n, c->mac_min_wg, &opt, &bch);
    const int G = (n_out + opt - 1) / opt, Z = (batch + bch - 1) / bch, C = (c->n + EW_THREADS - 1) / EW_THREADS;
#define MM(O, B) launch_mm<O, B>(m, n_out, n_terms, c->dev, nl, batch, accumulate, G, Z, C, pl, s)
    switch (bch * 100 + opt) {
    case 101: MM(1, 1); break;
    case 102: MM(2, 1); break;
    case 104: MM(4, 1); break;
    case 108: MM(8, 1); break;
    case 116: MM(16, 1); break;
    case 201: MM(1, 2); break;
    case 202: MM(2, 2); break;
    case 204: MM(4, 2); break;
    case 208: MM(8, 2); break;
    case 401: MM(1, 4); break;
    case 402: MM(2, 4); break;
    default: MM(4, 4); break;
    }
#undef MM
}

// ------------------------------------------------------------------ grouped elementwise steps
namespace {
__global__ void k_group_add(EwGroup g, DevCtx ctx, int nl, int plain, int pl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // (b * 2 + c) * nl + i
    const int e = blockIdx.z;
    const int i = r % nl, c = (r / nl) & 1;
    const u64 q = ctx.mod[i == pl ? ctx.p_index : i].q;
    const u64 x = g.a[e][(size_t)r * n + k];
    u64 v;
    if (plain) v = c == 0 ? add_mod(x, g.b[e][(size_t)i * n + k], q) : x;
    else v = add_mod(x, g.b[e][(size_t)r * n + k], q);
    g.out[e][(size_t)r * n + k] = v;
}

// last[e][b][c] <- in_e[b][c][nl-1]
__global__ void k_group_last(u64* __restrict__ last, EwGroup g, int nl, int n)
{
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int p = blockIdx.y;  // b * 2 + c
    const int e = blockIdx.z;
    last[((size_t)e * gridDim.y + p) * n + k] = g.a[e][((size_t)p * nl + nl - 1) * n + k];
}

__global__ void k_group_sum(SumGroup g, DevCtx ctx, int nl, int accumulate, int pl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const size_t r = blockIdx.y;  // (b * 2 + c) * nl + i
    const int e = blockIdx.z;
    const int i = (int)(r % nl);
    const u64 q = ctx.mod[i == pl ? ctx.p_index : i].q;
    const size_t o = r * n + k;
    u64 v = accumulate ? g.out[e][o] : 0;
    // four independent loads per step, not one load per dependent addition
    int t = 0;
    for (; t + 4 <= g.T; t += 4) {
        const u64 x0 = g.in[e * g.T + t][o], x1 = g.in[e * g.T + t + 1][o];
        const u64 x2 = g.in[e * g.T + t + 2][o], x3 = g.in[e * g.T + t + 3][o];
        v = add_mod(add_mod(v, x0, q), add_mod(x1, add_mod(x2, x3, q), q), q);
    }
    for (; t < g.T; ++t) v = add_mod(v, g.in[e * g.T + t][o], q);
    g.out[e][o] = v;
}

// out_e[(b * 2 + c) * (nl + 1) + i] = P in_e[(b * 2 + c) * nl + i] (i < nl), 0 (i = nl)
__global__ void k_group_to_ext(EwGroup g, DevCtx ctx, int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // p * (nl + 1) + i
    const int e = blockIdx.z;
    const int i = r % (nl + 1), p = r / (nl + 1);
    u64 v = 0;
    if (i < nl)
        v = mul_shoup(g.a[e][((size_t)p * nl + i) * n + k], ctx.p_mod[2 * i], ctx.p_mod[2 * i + 1], ctx.mod[i].q);
    g.out[e][(size_t)r * n + k] = v;
}

// out_e[p][i] = (in_e[p][i] - r[e][p][i]) * inv_i (+ d0 / d1 addends: relinearisation)
__global__ void k_group_sub_scale2(EwGroup g, const u64* __restrict__ r, int x_limbs, const u64* __restrict__ inv,
                                   DevCtx ctx, int nl, int polys)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int row = blockIdx.y;  // p * nl + i
    const int e = blockIdx.z;
    const int i = row % nl, p = row / nl;
    const u64 q = ctx.mod[i].q;
    u64 v = sub_mod(g.a[e][((size_t)p * x_limbs + i) * n + k], r[((size_t)e * polys * nl + row) * n + k], q);
    v = mul_shoup(v, inv[2 * i], inv[2 * i + 1], q);
    g.out[e][(size_t)row * n + k] = v;
}

// relinearised product: out[e][b][c][i] = (U - R) P^-1 + d_c[e][b][i]
__global__ void k_relin_combine(u64* __restrict__ out, const u64* __restrict__ U, const u64* __restrict__ R,
                                const u64* __restrict__ d0, const u64* __restrict__ d1, const u64* __restrict__ inv,
                                DevCtx ctx, int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const size_t row = blockIdx.y;  // ((e * B + b) * 2 + c) * nl + i
    const int i = (int)(row % nl);
    const size_t p = row / nl, eb = p >> 1;
    const int c = (int)(p & 1);
    const u64 q = ctx.mod[i].q;
    u64 v = sub_mod(U[row * n + k], R[row * n + k], q);
    v = mul_shoup(v, inv[2 * i], inv[2 * i + 1], q);
    const u64* d = c == 0 ? d0 : d1;
    v = add_mod(v, d[(eb * nl + i) * n + k], q);
    out[row * n + k] = v;
}

// tensor of E ciphertext batches: d0/d1/d2 [E][B][nl]
// tensor of E ciphertext batches: a[e] x b[e] (b[e] null: a[e] squared; b rows
// with b_limbs limbs per polynomial, its first nl used); d0/d1/d2 [E][B][nl]
__global__ void k_group_tensor(u64* __restrict__ d0, u64* __restrict__ d1, u64* __restrict__ d2, EwGroup g, DevCtx ctx,
                               int nl, int batch, int b_limbs)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // b * nl + i
    const int e = blockIdx.z;
    const int i = r % nl, b = r / nl;
    const Modulus M = ctx.mod[i];
    const u64 c0 = g.a[e][(((size_t)b * 2 + 0) * nl + i) * n + k];
    const u64 c1 = g.a[e][(((size_t)b * 2 + 1) * nl + i) * n + k];
    const size_t o = ((size_t)e * batch * nl + r) * n + k;
    if (!g.b[e]) {
        const u64 s00 = mont_mul(mont_mul(c0, c0, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        const u64 s01 = mont_mul(mont_mul(c0, c1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        const u64 s11 = mont_mul(mont_mul(c1, c1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        d0[o] = s00;
        d1[o] = add_mod(s01, s01, M.q);
        d2[o] = s11;
    } else {
        const u64 e0 = g.b[e][(((size_t)b * 2 + 0) * b_limbs + i) * n + k];
        const u64 e1 = g.b[e][(((size_t)b * 2 + 1) * b_limbs + i) * n + k];
        const u64 s00 = mont_mul(mont_mul(c0, e0, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        const u64 s01 = mont_mul(mont_mul(c0, e1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        const u64 s10 = mont_mul(mont_mul(c1, e0, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        const u64 s11 = mont_mul(mont_mul(c1, e1, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        d0[o] = s00;
        d1[o] = add_mod(s01, s10, M.q);
        d2[o] = s11;
    }
}

template <int BCH>
__global__ void __launch_bounds__(EW_THREADS) k_mac_group(MacGroup m, DevCtx ctx, int nl, int batch, int pl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * EW_THREADS + threadIdx.x;
    if (k >= n) return;
    const int i = blockIdx.y;
    const int e = blockIdx.z % m.E;
    const int b0 = (blockIdx.z / m.E) * BCH;
    const Modulus M = ctx.mod[i == pl ? ctx.p_index : i];
    const int period = wide_period(M.ratio);
    WideAcc a[2 * BCH];
#pragma unroll
    for (int u = 0; u < 2 * BCH; ++u) wide_init(a[u], 0);
    // term t + 1's words load while term t's products run
    u64 pn = 0, vn[2 * BCH];
    auto fetch = [&](int t) {
        pn = m.pt[e * m.T + t][(size_t)i * n + k];
        const u64* ct = m.ct[e * m.T + t];
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) {
            const int b = b0 + u / 2, c = u & 1;
            vn[u] = b < batch ? ct[(((size_t)b * 2 + c) * nl + i) * n + k] : 0;
        }
    };
    if (m.T > 0) fetch(0);
    int since = 0;
    for (int t = 0; t < m.T; ++t) {
        const u64 p = pn;
        u64 v[2 * BCH];
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) v[u] = vn[u];
        if (t + 1 < m.T) fetch(t + 1);
#pragma unroll
        for (int u = 0; u < 2 * BCH; ++u) wide_mac(a[u], p, v[u]);
        if (++since == period) {
#pragma unroll
            for (int u = 0; u < 2 * BCH; ++u) wide_fold(a[u], M.q, M.qinv_neg);
            since = 0;
        }
    }
#pragma unroll
    for (int u = 0; u < 2 * BCH; ++u) {
        const int b = b0 + u / 2, c = u & 1;
        if (b < batch) m.acc[e][(((size_t)b * 2 + c) * nl + i) * n + k] = wide_redc(a[u], M.q, M.qinv_neg);
    }
}
}  // namespace

void launch_group_add(const unihenn_ctx* c, const EwGroup& g, int batch, int nl, bool plain, hipStream_t s, int pl)
{
    LaunchTimer tm(KF_ADD, 8.0 * c->n * g.E * (batch * 2.0 * nl * (plain ? 2.0 : 3.0) + (plain ? nl : 0)), s);
    dim3 g3((c->n + EW_THREADS - 1) / EW_THREADS, batch * 2 * nl, g.E);
    k_group_add<<<g3, EW_THREADS, 0, s>>>(g, c->dev, nl, plain ? 1 : 0, pl);
}

void launch_group_sum(const unihenn_ctx* c, const SumGroup& g, int batch, int nl, bool accumulate, hipStream_t s,
                      int pl)
{
    LaunchTimer tm(KF_ADD, 8.0 * c->n * g.E * batch * 2.0 * nl * (g.T + 1 + (accumulate ? 1 : 0)), s);
    dim3 g3((c->n + EW_THREADS - 1) / EW_THREADS, batch * 2 * nl, g.E);
    k_group_sum<<<g3, EW_THREADS, 0, s>>>(g, c->dev, nl, accumulate ? 1 : 0, pl);
}

void launch_group_to_ext(const unihenn_ctx* c, const EwGroup& g, int batch, int nl, hipStream_t s)
{
    LaunchTimer tm(KF_OTHER, 8.0 * c->n * g.E * batch * 2.0 * (2 * nl + 1), s);
    dim3 g3((c->n + EW_THREADS - 1) / EW_THREADS, batch * 2 * (nl + 1), g.E);
    k_group_to_ext<<<g3, EW_THREADS, 0, s>>>(g, c->dev, nl);
}

// ModDown of extended sums: the P rows gathered and inverse transformed, then
// lifted, forward transformed and combined, (x - R) P^-1, in one fused pass
// last[e][b][c] = INTT of limb `limb` (modulus index `mi`) of polynomial
// (b, c) of in_e (rows of `limbs` limbs), read straight from in_e by the
// gathering inverse NTT's first pass; false (nothing launched) when that
// pass is outside the radix-8 kernels.
static bool inv_ntt_of_limb(const unihenn_ctx* c, u64* last, const u64* const* in, int E, int B, int limbs,
                            int limb, int mi, hipStream_t s)
{
    if (E > UH_FUSE_MAX || !ntt_fusable(c)) return false;
    GatherArgs gta;
    memset(&gta, 0, sizeof(gta));
    for (int e = 0; e < E; ++e) {
        gta.src[e] = in[e] + (size_t)limb * c->n;
        gta.perm[e] = 1;
    }
    gta.stride = limbs;
    gta.mod0 = mi;
    return launch_ntt_inv_gather(c, last, gta, E, B * 2, 1, s);
}

void group_moddown(const unihenn_ctx* c, int E, const u64* const* in, u64* const* out, int B, int nl, u64* ws,
                   hipStream_t s)
{
    const size_t rn = (size_t)c->n;
    EwGroup g;
    memset(&g, 0, sizeof(g));
    g.E = E;
    for (int e = 0; e < E; ++e) {
        g.a[e] = in[e];
        g.out[e] = out[e];
    }
    u64* last = ws;                               // [E][B][2]
    u64* R = ws + (size_t)E * B * 2 * rn;         // [E][B][2][nl]
    const unsigned gx = (c->n + EW_THREADS - 1) / EW_THREADS;
    if (!inv_ntt_of_limb(c, last, in, E, B, nl + 1, nl, c->n_data, s)) {
        {
            LaunchTimer tm(KF_OTHER, 16.0 * c->n * E * B * 2, s);
            k_group_last<<<dim3(gx, B * 2, E), EW_THREADS, 0, s>>>(last, g, nl + 1, c->n);
        }
        launch_ntt_inv(c, last, E * B * 2, rowmap_list({c->n_data}), s);
    }
    {
        FuseArgs fa;
        memset(&fa, 0, sizeof(fa));
        fa.src = last;
        fa.src_mod = c->n_data;
        fa.nl = nl;
        fa.polys = B * 2;
        fa.x_limbs = nl + 1;
        fa.inv = c->d_p_inv;
        for (int e = 0; e < E; ++e) {
            fa.x[e] = in[e];
            fa.out[e] = out[e];
            fa.add_perm[e] = 1;
        }
        if (launch_ntt_fwd_fused(c, R, fa, E * B * 2 * nl, KF_MODDOWN, s)) return;
    }
    launch_lift_last(c, R, last, E * B * 2, nl, c->n_data, KF_MODDOWN, s);
    launch_ntt_fwd(c, R, E * B * 2 * nl, rowmap_ct(nl), s);
    {
        LaunchTimer tm(KF_MODDOWN, 8.0 * c->n * E * B * 2 * nl * 3, s);
        k_group_sub_scale2<<<dim3(gx, B * 2 * nl, E), EW_THREADS, 0, s>>>(g, R, nl + 1, c->d_p_inv, c->dev, nl, B * 2);
    }
}

void group_rescale(const unihenn_ctx* c, int E, const u64* const* in, u64* const* out, int B, int nl, u64* ws,
                   hipStream_t s)
{
    const int l = nl - 1;
    const size_t rn = (size_t)c->n;
    EwGroup g;
    memset(&g, 0, sizeof(g));
    g.E = E;
    for (int e = 0; e < E; ++e) {
        g.a[e] = in[e];
        g.out[e] = out[e];
    }
    u64* last = ws;                               // [E][B][2]
    u64* R = ws + (size_t)E * B * 2 * rn;         // [E][B][2][l]
    const unsigned gx = (c->n + EW_THREADS - 1) / EW_THREADS;
    if (!inv_ntt_of_limb(c, last, in, E, B, nl, l, l, s)) {
        {
            LaunchTimer tm(KF_OTHER, 16.0 * c->n * E * B * 2, s);
            k_group_last<<<dim3(gx, B * 2, E), EW_THREADS, 0, s>>>(last, g, nl, c->n);
        }
        launch_ntt_inv(c, last, E * B * 2, rowmap_list({l}), s);
    }
    const u64* inv = c->d_inv_last + (size_t)l * c->primes.size() * 2;
    {
        FuseArgs fa;
        memset(&fa, 0, sizeof(fa));
        fa.src = last;
        fa.src_mod = l;
        fa.nl = l;
        fa.polys = B * 2;
        fa.x_limbs = nl;
        fa.inv = inv;
        for (int e = 0; e < E; ++e) {
            fa.x[e] = in[e];
            fa.out[e] = out[e];
            fa.add_perm[e] = 1;
        }
        if (launch_ntt_fwd_fused(c, R, fa, E * B * 2 * l, KF_RESCALE, s)) return;
    }
    launch_lift_last(c, R, last, E * B * 2, l, l, KF_RESCALE, s);
    launch_ntt_fwd(c, R, E * B * 2 * l, rowmap_ct(l), s);
    {
        LaunchTimer tm(KF_RESCALE, 8.0 * c->n * E * B * 2 * l * 3, s);
        k_group_sub_scale2<<<dim3(gx, B * 2 * l, E), EW_THREADS, 0, s>>>(g, R, nl, inv, c->dev, l, B * 2);
    }
}

size_t group_square_ws_rows(int E, int nl, int batch)
{
    // d0, d1, d2 [E][B][nl]; dcoef [E][B][nl]; modup [E][B][nl][nl]; U [E][B][2][nl]; Up [E][B][2];
    // R [E][B][2][nl]; relinearised [E][B][2][nl]; rescale scratch E*B*2*nl
    return (size_t)E * batch * (3 * nl + nl + (size_t)nl * nl + 2 * nl + 2 + 2 * nl + 2 * nl + 2 * nl);
}

void group_square(const unihenn_ctx* c, int E, const u64* const* in, u64* const* out, const u64* rlk, int B, int nl,
                  u64* ws, hipStream_t s, const u64* const* in2, int in2_limbs)
{
    const size_t rn = (size_t)c->n, EB = (size_t)E * B;
    u64* d0 = ws;
    u64* d1 = d0 + EB * nl * rn;
    u64* d2 = d1 + EB * nl * rn;
    u64* dcoef = d2 + EB * nl * rn;
    u64* modup = dcoef + EB * nl * rn;
    u64* U = modup + EB * nl * nl * rn;
    u64* Up = U + EB * 2 * nl * rn;
    u64* R = Up + EB * 2 * rn;
    u64* rel = R + EB * 2 * nl * rn;
    u64* scratch = rel + EB * 2 * nl * rn;
    const unsigned gx = (c->n + EW_THREADS - 1) / EW_THREADS;
    EwGroup g;
    memset(&g, 0, sizeof(g));
    g.E = E;
    for (int e = 0; e < E; ++e) {
        g.a[e] = in[e];
        g.b[e] = in2 ? in2[e] : nullptr;
    }
    {
        LaunchTimer tm(KF_TENSOR, 8.0 * c->n * EB * nl * (in2 ? 7 : 5), s);
        k_group_tensor<<<dim3(gx, B * nl, E), EW_THREADS, 0, s>>>(d0, d1, d2, g, c->dev, nl, B, in2 ? in2_limbs : nl);
    }
    // ModUp of every d2 (E * B ciphertext-polys as one batch), inner product with the relinearisation key
    launch_gather_rows(c, dcoef, d2, (int)EB * nl, nl, nl, 0, s);
    launch_ntt_inv(c, dcoef, (int)EB * nl, rowmap_ct(nl), s);
    if (!launch_ntt_fwd_modup(c, modup, dcoef, (int)EB * nl, nl, s)) {
        launch_modup(c, modup, dcoef, (int)EB, nl, s);
        launch_ntt_fwd(c, modup, (int)EB * nl * nl, rowmap_modup(nl, c->n_data), s);
    }
    launch_ks_inner(c, U, Up, d2, nl, modup, rlk, c->n_data, (int)EB, nl, 1, s);
    launch_ntt_inv(c, Up, (int)EB * 2, rowmap_list({c->n_data}), s);
    FuseArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.src = Up;
    fa.src_mod = c->n_data;
    fa.nl = nl;
    fa.polys = (int)EB * 2;
    fa.x[0] = U;
    fa.x_limbs = nl;
    fa.add[0][0] = d0;
    fa.add[0][1] = d1;
    fa.add_stride = nl;
    fa.add_perm[0] = 1;
    fa.out[0] = rel;
    fa.inv = c->d_p_inv;
    if (!launch_ntt_fwd_fused(c, R, fa, (int)EB * 2 * nl, KF_MODDOWN, s)) {
        launch_lift_last(c, R, Up, (int)EB * 2, nl, c->n_data, KF_MODDOWN, s);
        launch_ntt_fwd(c, R, (int)EB * 2 * nl, rowmap_ct(nl), s);
        LaunchTimer tm(KF_MODDOWN, 8.0 * c->n * EB * 2 * nl * 3.5, s);
        k_relin_combine<<<dim3(gx, (unsigned)(EB * 2 * nl)), EW_THREADS, 0, s>>>(rel, U, R, d0, d1, c->d_p_inv, c->dev,
                                                                                 nl);
    }
    std::vector<const u64*> ins(E);
    for (int e = 0; e < E; ++e) ins[e] = rel + (size_t)e * B * 2 * nl * rn;
    group_rescale(c, E, ins.data(), out, B, nl, scratch, s);
}

void launch_mac_group(const unihenn_ctx* c, const MacGroup& m, int nl, int batch, hipStream_t s, int pl)
{
    double rows = (double)m.E * m.T * (nl + batch * 2.0 * nl) + m.E * batch * 2.0 * nl;
    LaunchTimer tm(KF_MAC, 8.0 * c->n * rows, s);
    const unsigned gx = (c->n + EW_THREADS - 1) / EW_THREADS;
    if (batch >= 4)
        k_mac_group<4><<<dim3(gx, nl, m.E * ((batch + 3) / 4)), EW_THREADS, 0, s>>>(m, c->dev, nl, batch, pl);
    else
        k_mac_group<1><<<dim3(gx, nl, m.E * batch), EW_THREADS, 0, s>>>(m, c->dev, nl, batch, pl);
}
