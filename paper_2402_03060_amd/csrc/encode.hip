// Encoding of real slot vectors into plaintexts (Section II-B, III-A):
//   m_j = (2/N) sum_k z_k cos(pi (5^k mod 2N) j / N),  pt_j = round(scale m_j)
// The sum runs over the non-zero slots only, one thread per coefficient j,
// in double-double arithmetic against a double-double cosine table; the
// rounding (half away from zero) is decided on that value, then the integer
// is reduced mod each prime and the rows are transformed to NTT form.
#include <algorithm>
#include <vector>

#include "dd.h"
#include "kernels.h"

namespace {
constexpr int ENC_THREADS = 256;

__global__ void k_encode_sum(double* __restrict__ m_out, const uint32_t* __restrict__ ek,
                             const double* __restrict__ zv, int nnz, const double* __restrict__ cos_tab, int log_n)
{
    const int n = 1 << log_n;
    const int j = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (j >= n) return;
    const u64 mask = (2ull << log_n) - 1;
    dd acc = dd_make(0.0, 0.0);
    for (int t = 0; t < nnz; ++t) {
        const u64 idx = ((u64)ek[t] * (u64)j) & mask;
        const dd cs = dd_make(cos_tab[2 * idx], cos_tab[2 * idx + 1]);
        acc = dd_add(acc, dd_mul_d(cs, zv[t]));
    }
    const double f = ldexp(1.0, 1 - log_n);  // 2/N, exact
    m_out[2 * j] = acc.hi * f;
    m_out[2 * j + 1] = acc.lo * f;
}

// round half away from zero of |v| < 2^52; false when out of range
__device__ __forceinline__ bool dd_round(dd v, i64* out)
{
    double hi = v.hi, lo = v.lo;
    const bool neg = hi < 0.0 || (hi == 0.0 && lo < 0.0);
    if (neg) { hi = -hi; lo = -lo; }
    if (!(hi < 4503599627370496.0)) return false;
    const double f = floor(hi);
    const dd r = two_sum(hi - f, lo);  // hi - f is exact
    i64 k = (i64)f;
    if (r.hi > 0.5 || (r.hi == 0.5 && r.lo >= 0.0)) k += 1;
    *out = neg ? -k : k;
    return true;
}

// pt[w][i][j] = round(s_w * m_j) mod q_i with s_w = scale * w (exact double-double);
// with ext the last of the nl rows is taken mod P
__global__ void k_encode_round(u64* __restrict__ pt, const double* __restrict__ m, const double* __restrict__ ws,
                               int n_w, double scale, DevCtx ctx, int nl, int ext, int* __restrict__ overflow)
{
    const int n = ctx.n;
    const int j = blockIdx.x * ENC_THREADS + threadIdx.x;
    if (j >= n) return;
    const int w = blockIdx.y;
    const dd sw = two_prod(scale, ws[w]);
    const dd v = dd_mul(dd_make(m[2 * j], m[2 * j + 1]), sw);
    i64 iv = 0;
    if (!dd_round(v, &iv)) {
        atomicOr(overflow, 1);
        iv = 0;
    }
    const u64 mag = (u64)(iv < 0 ? -iv : iv);
    for (int i = 0; i < nl; ++i) {
        const Modulus M = ctx.mod[(ext && i == nl - 1) ? ctx.p_index : i];
        u64 r = reduce64(mag, M.q, M.ratio);
        if (iv < 0 && r) r = M.q - r;
        pt[(((size_t)w * nl) + i) * n + j] = r;
    }
}
}  // namespace

// Device buffers of one encoding job, released by the destructor after a
// stream synchronisation.
struct EncodeJob {
    uint32_t* ek = nullptr;
    double* zv = nullptr;
    double* m = nullptr;
    double* ws = nullptr;
    int* ovf = nullptr;
    ~EncodeJob()
    {
        (void)hipFree(ek);
        (void)hipFree(zv);
        (void)hipFree(m);
        (void)hipFree(ws);
        (void)hipFree(ovf);
    }
};

// Encode(w_t * z) for every weight (n_w plaintexts, [n_w][nl][N], or with
// ext [n_w][nl+1][N] whose limb nl is the residue mod P, for products with
// extended ciphertexts); internal entry used by the network builder and
// unihenn_encode.
int encode_scaled_batch(const unihenn_ctx* c, const double* z, int n_slots, const double* w, int n_w, double scale,
                        int nl, int mont, u64* out, hipStream_t s, int ext)
{
    if (n_slots > c->n / 2) return uh_fail(UNIHENN_EINVAL, "more values than slots");
    if (nl < 1 || nl > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    std::vector<uint32_t> ek;
    std::vector<double> zv;
    u64 e = 1, two_n = 2 * (u64)c->n;
    for (int k = 0; k < n_slots; ++k) {
        if (z[k] != 0.0) {
            ek.push_back((uint32_t)e);
            zv.push_back(z[k]);
        }
        e = e * 5 % two_n;
    }
    EncodeJob job;
    const int nnz = (int)ek.size();
    if (hipMalloc(&job.m, sizeof(double) * 2 * c->n) != hipSuccess ||
        hipMalloc(&job.ws, sizeof(double) * std::max(n_w, 1)) != hipSuccess ||
        hipMalloc(&job.ovf, sizeof(int)) != hipSuccess)
        return uh_fail(UNIHENN_ENOMEM, "encode buffers");
    if (nnz > 0 && (hipMalloc(&job.ek, sizeof(uint32_t) * nnz) != hipSuccess ||
                    hipMalloc(&job.zv, sizeof(double) * nnz) != hipSuccess))
        return uh_fail(UNIHENN_ENOMEM, "encode buffers");
    if (nnz > 0) {
        UH_CHECK_HIP(hipMemcpyAsync(job.ek, ek.data(), sizeof(uint32_t) * nnz, hipMemcpyHostToDevice, s));
        UH_CHECK_HIP(hipMemcpyAsync(job.zv, zv.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, s));
    }
    UH_CHECK_HIP(hipMemcpyAsync(job.ws, w, sizeof(double) * n_w, hipMemcpyHostToDevice, s));
    const int zero = 0;
    UH_CHECK_HIP(hipMemcpyAsync(job.ovf, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    {
        LaunchTimer tm(KF_ENCODE, 8.0 * (2.0 * c->n + (double)n_w * (nl + ext) * c->n), s);
        dim3 g1((c->n + ENC_THREADS - 1) / ENC_THREADS);
        k_encode_sum<<<g1, ENC_THREADS, 0, s>>>(job.m, job.ek, job.zv, nnz, c->d_cos, c->log_n);
        dim3 g2((c->n + ENC_THREADS - 1) / ENC_THREADS, n_w);
        k_encode_round<<<g2, ENC_THREADS, 0, s>>>(out, job.m, job.ws, n_w, scale, c->dev, nl + ext, ext, job.ovf);
    }
    std::vector<int> mods;
    for (int i = 0; i < nl; ++i) mods.push_back(i);
    if (ext) mods.push_back(c->n_data);
    const RowMap map = rowmap_list(mods);
    launch_ntt_fwd(c, out, n_w * (nl + ext), map, s);
    if (mont) launch_mont_convert(c, out, n_w * (nl + ext), map, 1, s);
    int ovf = 0;
    UH_CHECK_HIP(hipMemcpyAsync(&ovf, job.ovf, sizeof(int), hipMemcpyDeviceToHost, s));
    UH_CHECK_HIP(hipStreamSynchronize(s));
    if (ovf) return uh_fail(UNIHENN_EINVAL, "encoded coefficient exceeds 2^52");
    return UNIHENN_OK;
}

extern "C" int unihenn_encode(const unihenn_ctx* c, const double* slots, uint32_t n_slots, double scale,
                              uint32_t n_limbs, int mont, uint64_t* pt, void* stream)
{
    if (!c || !pt || (n_slots && !slots)) return uh_fail(UNIHENN_EINVAL, "null argument");
    const double one = 1.0;
    return encode_scaled_batch(c, slots, (int)n_slots, &one, 1, scale, (int)n_limbs, mont, pt, (hipStream_t)stream, 0);
}

extern "C" int unihenn_import_pt(const unihenn_ctx* c, const uint64_t* coeff, uint32_t n_limbs, int mont,
                                 uint64_t* pt, void* stream)
{
    if (!c || !coeff || !pt) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (n_limbs < 1 || (int)n_limbs > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    hipStream_t s = (hipStream_t)stream;
    if (pt != coeff)
        UH_CHECK_HIP(hipMemcpyAsync(pt, coeff, sizeof(u64) * n_limbs * c->n, hipMemcpyDeviceToDevice, s));
    launch_ntt_fwd(c, pt, (int)n_limbs, rowmap_ct((int)n_limbs), s);
    if (mont) launch_mont_convert(c, pt, (int)n_limbs, rowmap_ct((int)n_limbs), 1, s);
    return UNIHENN_OK;
}

extern "C" int unihenn_export_pt(const unihenn_ctx* c, const uint64_t* pt, uint32_t n_limbs, int mont,
                                 uint64_t* coeff_out, void* stream)
{
    if (!c || !pt || !coeff_out) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (n_limbs < 1 || (int)n_limbs > c->n_data) return uh_fail(UNIHENN_EINVAL, "bad limb count");
    hipStream_t s = (hipStream_t)stream;
    if (coeff_out != pt)
        UH_CHECK_HIP(hipMemcpyAsync(coeff_out, pt, sizeof(u64) * n_limbs * c->n, hipMemcpyDeviceToDevice, s));
    if (mont) launch_mont_convert(c, coeff_out, (int)n_limbs, rowmap_ct((int)n_limbs), 0, s);
    launch_ntt_inv(c, coeff_out, (int)n_limbs, rowmap_ct((int)n_limbs), s);
    return UNIHENN_OK;
}
