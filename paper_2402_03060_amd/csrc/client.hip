// Client side (UniHENN Section III and Fig. 1: the client encrypts its inputs
// and decrypts the returned results; the server holds the evaluation keys).
// Keys, encryptions and decryptions computed on the GPU, in NTT form.
//
// Randomness is a counter-based hash (the SplitMix64 output function applied
// twice to seed + golden-ratio multiples of (stream, index)): a research
// generator, not a cryptographic one.
#include <cmath>
#include <vector>

#include "dd.h"
#include "kernels.h"

namespace {
constexpr int CL_THREADS = 256;

__device__ __forceinline__ u64 mix64(u64 z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ u64 rng64(u64 seed, u64 stream, u64 idx)
{
    return mix64(mix64(seed + 0x9e3779b97f4a7c15ull * ((stream << 40) + idx + 1)) ^ (stream * 0xd1b54a32d192ed03ull));
}
// uniform ternary in {-1, 0, 1}
__device__ __forceinline__ int ternary(u64 seed, u64 stream, u64 idx)
{
    return (int)((((rng64(seed, stream, idx) >> 32) * 3ull) >> 32)) - 1;
}
// rounded Gaussian, sigma = 3.2, redrawn when |e| > 19 (Box-Muller)
__device__ __forceinline__ int gauss(u64 seed, u64 stream, u64 idx)
{
    for (u64 t = 0; t < 64; ++t) {
        const u64 r1 = rng64(seed, stream, 2 * (idx * 64 + t)), r2 = rng64(seed, stream, 2 * (idx * 64 + t) + 1);
        const double u1 = ((r1 >> 11) + 1) * 0x1p-53, u2 = (r2 >> 11) * 0x1p-53;
        const double e = rint(3.2 * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
        if (fabs(e) <= 19.0) return (int)e;
    }
    return 0;
}
__device__ __forceinline__ u64 small_mod(int v, u64 q) { return v < 0 ? q - (u64)(-v) : (u64)v; }

// rows [n_rows][N]: small signed values (ternary or Gaussian) reduced mod the row's modulus
__global__ void k_sample_small(u64* __restrict__ out, DevCtx ctx, RowMap map, int rows_per_poly, u64 seed, u64 stream,
                               int gaussian)
{
    const int n = ctx.n;
    const int k = blockIdx.x * CL_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;
    const int poly = r / rows_per_poly;
    const u64 q = ctx.mod[rowmap_mod(map, r)].q;
    const u64 idx = (u64)poly * n + k;
    const int v = gaussian ? gauss(seed, stream, idx) : ternary(seed, stream, idx);
    out[(size_t)r * n + k] = small_mod(v, q);
}

// key[d][0][i] = -a s + e + [i == d] (P mod q_i) t, key[d][1][i] = a   (NTT form, plain)
__global__ void k_keygen_combine(u64* __restrict__ key, const u64* __restrict__ e, const u64* __restrict__ s,
                                 const u64* __restrict__ t, DevCtx ctx, const u64* __restrict__ qmod, int n_mod,
                                 u64 seed)
{
    const int n = ctx.n;
    const int k = blockIdx.x * CL_THREADS + threadIdx.x;
    if (k >= n) return;
    const int nb = ctx.n_data + 1;
    const int r = blockIdx.y;  // d * nb + i
    const int i = r % nb, d = r / nb;
    const Modulus M = ctx.mod[i];
    const u64 a = umulhi64(rng64(seed, 1000 + d, (u64)i * n + k), M.q);
    const u64 as = mont_mul(mont_mul(a, s[(size_t)i * n + k], M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    u64 v = sub_mod(e[(size_t)r * n + k], as, M.q);
    if (i == d) {
        const u64 pm = qmod[(size_t)ctx.p_index * n_mod + i];
        const u64 pt = mont_mul(mont_mul(pm, t[(size_t)i * n + k], M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
        v = add_mod(v, pt, M.q);
    }
    key[(((size_t)d * 2 + 0) * nb + i) * n + k] = v;
    key[(((size_t)d * 2 + 1) * nb + i) * n + k] = a;
}

// t = s (*) s over every modulus (relinearisation target)
__global__ void k_square_rows(u64* __restrict__ t, const u64* __restrict__ s, DevCtx ctx)
{
    const int n = ctx.n;
    const int k = blockIdx.x * CL_THREADS + threadIdx.x;
    if (k >= n) return;
    const int i = blockIdx.y;
    const Modulus M = ctx.mod[i];
    const u64 x = s[(size_t)i * n + k];
    t[(size_t)i * n + k] = mont_mul(mont_mul(x, x, M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
}

// ct[b] = (-a s + e + m_b, a) over nl limbs, NTT form
__global__ void k_encrypt_combine(u64* __restrict__ ct, const u64* __restrict__ e, const u64* __restrict__ s,
                                  const u64* __restrict__ pts, DevCtx ctx, int nl, u64 seed)
{
    const int n = ctx.n;
    const int k = blockIdx.x * CL_THREADS + threadIdx.x;
    if (k >= n) return;
    const int r = blockIdx.y;  // b * nl + i
    const int i = r % nl, b = r / nl;
    const Modulus M = ctx.mod[i];
    const u64 a = umulhi64(rng64(seed, 2000000 + b, (u64)i * n + k), M.q);
    const u64 as = mont_mul(mont_mul(a, s[(size_t)i * n + k], M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    const u64 v = add_mod(sub_mod(e[(size_t)r * n + k], as, M.q), pts[(size_t)r * n + k], M.q);
    ct[(((size_t)b * 2 + 0) * nl + i) * n + k] = v;
    ct[(((size_t)b * 2 + 1) * nl + i) * n + k] = a;
}

// m[b] = c0 + c1 s on limb 0 (NTT form)
__global__ void k_decrypt_limb0(u64* __restrict__ m, const u64* __restrict__ ct, const u64* __restrict__ s, DevCtx ctx,
                                int nl)
{
    const int n = ctx.n;
    const int k = blockIdx.x * CL_THREADS + threadIdx.x;
    if (k >= n) return;
    const int b = blockIdx.y;
    const Modulus M = ctx.mod[0];
    const u64 c0 = ct[(((size_t)b * 2 + 0) * nl) * n + k];
    const u64 c1 = ct[(((size_t)b * 2 + 1) * nl) * n + k];
    const u64 cs = mont_mul(mont_mul(c1, s[k], M.q, M.qinv_neg), M.r2, M.q, M.qinv_neg);
    m[(size_t)b * n + k] = add_mod(c0, cs, M.q);
}

// values[b][i] = (1/scale) sum_j centered(m_j) cos(pi e_i j / N), one block per (b, i)
__global__ void k_decode_slots(double* __restrict__ out, const u64* __restrict__ m, const uint32_t* __restrict__ slot_e,
                               int n_slots, const double* __restrict__ cos_tab, DevCtx ctx, double inv_scale)
{
    __shared__ double red[CL_THREADS];
    const int n = ctx.n;
    const int i = blockIdx.x, b = blockIdx.y;
    const u64 q = ctx.mod[0].q, half = ctx.mod[0].half;
    const u64 e = slot_e[i];
    const u64 mask = 2ull * n - 1;
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += CL_THREADS) {
        const u64 x = m[(size_t)b * n + j];
        const double v = x > half ? -(double)(q - x) : (double)x;
        acc += v * cos_tab[2 * ((e * (u64)j) & mask)];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = CL_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)b * n_slots + i] = red[0] * inv_scale;
}

inline dim3 grid_rows(int n, int rows) { return dim3((n + CL_THREADS - 1) / CL_THREADS, rows); }

}  // namespace

extern "C" int unihenn_keygen_secret(const unihenn_ctx* c, uint64_t seed, uint64_t* sk, void* stream)
{
    if (!c || !sk) return uh_fail(UNIHENN_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = c->n_data + 1;
    RowMap m = rowmap_ct(nb);
    // every row holds the same ternary polynomial (poly index 0) mod its prime
    k_sample_small<<<grid_rows(c->n, nb), CL_THREADS, 0, s>>>(sk, c->dev, m, nb, seed, 1, 0);
    launch_ntt_fwd(c, sk, nb, m, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return uh_fail(UNIHENN_EDEVICE, hipGetErrorString(e));
    return UNIHENN_OK;
}

extern "C" int unihenn_gen_switch_key(const unihenn_ctx* c, const uint64_t* sk, uint64_t seed, int32_t steps, int relin,
                                      uint64_t* out, void* stream)
{
    if (!c || !sk || !out) return uh_fail(UNIHENN_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const int nb = c->n_data + 1, nd = c->n_data;
    const u32 g = galois_elt(c, steps);
    if (!relin && g == 1) return uh_fail(UNIHENN_EINVAL, "rotation by 0 needs no key");
    u64 *t = nullptr, *e = nullptr;
    if (hipMalloc(&t, sizeof(u64) * nb * c->n) != hipSuccess ||
        hipMalloc(&e, sizeof(u64) * (size_t)nd * nb * c->n) != hipSuccess) {
        (void)hipFree(t);
        (void)hipFree(e);
        return uh_fail(UNIHENN_ENOMEM, "key generation buffers");
    }
    if (relin)
        k_square_rows<<<grid_rows(c->n, nb), CL_THREADS, 0, s>>>(t, sk, c->dev);
    else
        launch_automorphism(c, t, sk, nb, g, s);
    // one Gaussian polynomial per digit, the same integers reduced mod every prime
    RowMap m = rowmap_ct(nb);
    const u64 stream_id = 10 + (relin ? 0 : (u64)g);
    k_sample_small<<<grid_rows(c->n, nd * nb), CL_THREADS, 0, s>>>(e, c->dev, m, nb, seed, stream_id, 1);
    launch_ntt_fwd(c, e, nd * nb, m, s);
    k_keygen_combine<<<grid_rows(c->n, nd * nb), CL_THREADS, 0, s>>>(out, e, sk, t, c->dev, c->d_qmod,
                                                                      (int)c->primes.size(), seed ^ (stream_id << 20));
    launch_mont_convert(c, out, nd * 2 * nb, m, 1, s);
    hipError_t err = hipStreamSynchronize(s);
    (void)hipFree(t);
    (void)hipFree(e);
    if (err != hipSuccess) return uh_fail(UNIHENN_EDEVICE, hipGetErrorString(err));
    return UNIHENN_OK;
}

extern "C" int unihenn_encrypt_sk(const unihenn_ctx* c, const uint64_t* sk, const uint64_t* pts, uint64_t seed,
                                  unihenn_ct* ct, void* stream)
{
    if (!c || !sk || !pts || !ct || !ct->data) return uh_fail(UNIHENN_EINVAL, "null argument");
    const int nl = (int)ct->n_limbs, B = (int)ct->batch;
    if (nl < 1 || nl > c->n_data || B < 1) return uh_fail(UNIHENN_EINVAL, "bad ciphertext shape");
    hipStream_t s = (hipStream_t)stream;
    u64* e = nullptr;
    if (hipMalloc(&e, sizeof(u64) * (size_t)B * nl * c->n) != hipSuccess)
        return uh_fail(UNIHENN_ENOMEM, "encryption buffers");
    RowMap m = rowmap_ct(nl);
    k_sample_small<<<grid_rows(c->n, B * nl), CL_THREADS, 0, s>>>(e, c->dev, m, nl, seed, 3000000, 1);
    launch_ntt_fwd(c, e, B * nl, m, s);
    k_encrypt_combine<<<grid_rows(c->n, B * nl), CL_THREADS, 0, s>>>(ct->data, e, sk, pts, c->dev, nl, seed);
    hipError_t err = hipStreamSynchronize(s);
    (void)hipFree(e);
    if (err != hipSuccess) return uh_fail(UNIHENN_EDEVICE, hipGetErrorString(err));
    return UNIHENN_OK;
}

extern "C" int unihenn_decrypt_slots(const unihenn_ctx* c, const uint64_t* sk, const unihenn_ct* ct,
                                     const uint32_t* slot_index, uint32_t n_slots, double* values, void* stream)
{
    if (!c || !sk || !ct || !ct->data || !values || (n_slots && !slot_index)) return uh_fail(UNIHENN_EINVAL, "null argument");
    const int B = (int)ct->batch, nl = (int)ct->n_limbs;
    if (B < 1 || nl < 1 || nl > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad ciphertext shape");
    if (n_slots == 0) return UNIHENN_OK;
    std::vector<uint32_t> es(n_slots);
    for (uint32_t i = 0; i < n_slots; ++i) {
        if (slot_index[i] >= (uint32_t)c->n / 2) return uh_fail(UNIHENN_EINVAL, "slot index out of range");
        es[i] = galois_elt(c, slot_index[i]);
    }
    hipStream_t s = (hipStream_t)stream;
    u64* m = nullptr;
    uint32_t* de = nullptr;
    double* dv = nullptr;
    if (hipMalloc(&m, sizeof(u64) * (size_t)B * c->n) != hipSuccess || hipMalloc(&de, sizeof(uint32_t) * n_slots) != hipSuccess ||
        hipMalloc(&dv, sizeof(double) * (size_t)B * n_slots) != hipSuccess) {
        (void)hipFree(m);
        (void)hipFree(de);
        (void)hipFree(dv);
        return uh_fail(UNIHENN_ENOMEM, "decryption buffers");
    }
    hipError_t cerr = hipMemcpyAsync(de, es.data(), sizeof(uint32_t) * n_slots, hipMemcpyHostToDevice, s);
    k_decrypt_limb0<<<grid_rows(c->n, B), CL_THREADS, 0, s>>>(m, ct->data, sk, c->dev, nl);
    launch_ntt_inv(c, m, B, rowmap_list({0}), s);
    k_decode_slots<<<dim3(n_slots, B), CL_THREADS, 0, s>>>(dv, m, de, (int)n_slots, c->d_cos, c->dev, 1.0 / ct->scale);
    if (cerr == hipSuccess) cerr = hipMemcpyAsync(values, dv, sizeof(double) * (size_t)B * n_slots, hipMemcpyDeviceToHost, s);
    hipError_t err = hipStreamSynchronize(s);
    if (err == hipSuccess) err = cerr;
    (void)hipFree(m);
    (void)hipFree(de);
    (void)hipFree(dv);
    if (err != hipSuccess) return uh_fail(UNIHENN_EDEVICE, hipGetErrorString(err));
    return UNIHENN_OK;
}
