// Negacyclic NTT / inverse NTT of batched limb rows.
//
// Forward: Cooley-Tukey butterflies with the 2N-th root psi merged into the
// twiddles (stage s uses psi^brev(2^s + i)), output in bit-reversed order,
// so that entry k holds a(psi^(2 brev(k) + 1)).  Inverse: Gentleman-Sande
// butterflies with psi^-brev(.), then the factor N^-1.  Values stay lazily
// reduced (forward in [0, 4q), inverse in [0, 2q)) and are made canonical
// at the end; q < 2^61 keeps every intermediate below 2^64.
//
// The log N stages are split into two passes over LDS tiles:
//   column pass  stages [0, L1): 2^L1-point transforms of elements strided by
//                N / 2^L1; a tile holds COLS consecutive columns so every
//                global row access is COLS contiguous words;
//   row pass     stages [L1, log N): contiguous 2^(log N - L1)-point blocks.
// The generic kernels (sub-transforms below 8 points) use tiles of TILE
// words (16 KiB) of LDS and 256 threads; the radix-8 kernels take the tile
// size (2^11 or 2^12 words, with 2^8 or 2^9 threads) as a launch parameter.
#include <cstring>
#include <type_traits>

#include "kernels.h"

namespace {

constexpr int TILE = 2048;
constexpr int NTT_THREADS = 256;

struct PassGeom {
    int log_r;    // log2 of the sub-transform size
    int cols;     // sub-transforms per tile
    int sigma0;   // first global stage of the pass
    bool strided; // column pass
};

__device__ __forceinline__ int lds_index(bool strided, int u, int c, int cols, int r)
{
    return strided ? u * cols + c : c * r + u;
}

template <bool STRIDED, bool LAST>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_fwd(u64* __restrict__ data, DevCtx ctx, RowMap map,
                                                         int log_r, int cols, int sigma0)
{
    __shared__ u64 s[TILE];
    const int n = ctx.n, log_n = ctx.log_n;
    const int r = 1 << log_r;
    const int row = blockIdx.y;
    const int mi = rowmap_mod(map, row);
    const u64 q = ctx.mod[mi].q, q2 = 2 * q;
    const u64* tw = ctx.tw + (size_t)mi * n;
    const u64* tw_sh = ctx.tw_sh + (size_t)mi * n;
    u64* a = data + (size_t)row * n;
    const int tid = threadIdx.x;
    const int elems = r * cols;
    const int col0 = blockIdx.x * cols;  // first column (strided) or first block (contiguous)
    const int stride = n >> log_r;

    for (int e = tid; e < elems; e += NTT_THREADS) {
        if (STRIDED) {
            int c = e % cols, u = e / cols;
            s[e] = a[col0 + c + (size_t)u * stride];
        } else {
            s[e] = a[(size_t)col0 * r + e];
        }
    }
    __syncthreads();
    for (int tau = 0; tau < log_r; ++tau) {
        const int sigma = sigma0 + tau;
        const int hb = log_r - tau - 1;  // half-size bit
        const int t = 1 << hb;
        for (int b = tid; b < elems / 2; b += NTT_THREADS) {
            int c, p;
            if (STRIDED) { c = b % cols; p = b / cols; }
            else { c = b / (r / 2); p = b % (r / 2); }
            const int u = ((p >> hb) << (hb + 1)) | (p & (t - 1));
            const int j = STRIDED ? (col0 + c) + u * stride : (col0 + c) * r + u;  // global index
            const int ti = (1 << sigma) + (j >> (log_n - sigma));
            const int i0 = lds_index(STRIDED, u, c, cols, r), i1 = lds_index(STRIDED, u + t, c, cols, r);
            u64 U = s[i0];
            U = U >= q2 ? U - q2 : U;
            const u64 V = mul_shoup_lazy(s[i1], tw[ti], tw_sh[ti], q);
            s[i0] = U + V;
            s[i1] = U - V + q2;
        }
        __syncthreads();
    }
    for (int e = tid; e < elems; e += NTT_THREADS) {
        u64 v = s[e];
        if (LAST) {
            v = v >= q2 ? v - q2 : v;
            v = v >= q ? v - q : v;
        }
        if (STRIDED) {
            int c = e % cols, u = e / cols;
            a[col0 + c + (size_t)u * stride] = v;
        } else {
            a[(size_t)col0 * r + e] = v;
        }
    }
}

template <bool STRIDED, bool LAST>
__global__ void __launch_bounds__(NTT_THREADS) k_ntt_inv(u64* __restrict__ data, DevCtx ctx, RowMap map,
                                                         int log_r, int cols, int sigma0)
{
    __shared__ u64 s[TILE];
    const int n = ctx.n, log_n = ctx.log_n;
    const int r = 1 << log_r;
    const int row = blockIdx.y;
    const int mi = rowmap_mod(map, row);
    const Modulus M = ctx.mod[mi];
    const u64 q = M.q, q2 = 2 * q;
    const u64* tw = ctx.itw + (size_t)mi * n;
    const u64* tw_sh = ctx.itw_sh + (size_t)mi * n;
    u64* a = data + (size_t)row * n;
    const int tid = threadIdx.x;
    const int elems = r * cols;
    const int col0 = blockIdx.x * cols;
    const int stride = n >> log_r;

    for (int e = tid; e < elems; e += NTT_THREADS) {
        if (STRIDED) {
            int c = e % cols, u = e / cols;
            s[e] = a[col0 + c + (size_t)u * stride];
        } else {
            s[e] = a[(size_t)col0 * r + e];
        }
    }
    __syncthreads();
    for (int tau = log_r - 1; tau >= 0; --tau) {
        const int sigma = sigma0 + tau;
        const int hb = log_r - tau - 1;
        const int t = 1 << hb;
        for (int b = tid; b < elems / 2; b += NTT_THREADS) {
            int c, p;
            if (STRIDED) { c = b % cols; p = b / cols; }
            else { c = b / (r / 2); p = b % (r / 2); }
            const int u = ((p >> hb) << (hb + 1)) | (p & (t - 1));
            const int j = STRIDED ? (col0 + c) + u * stride : (col0 + c) * r + u;
            const int ti = (1 << sigma) + (j >> (log_n - sigma));
            const int i0 = lds_index(STRIDED, u, c, cols, r), i1 = lds_index(STRIDED, u + t, c, cols, r);
            const u64 U = s[i0], V = s[i1];
            u64 x = U + V;
            s[i0] = x >= q2 ? x - q2 : x;
            s[i1] = mul_shoup_lazy(U - V + q2, tw[ti], tw_sh[ti], q);
        }
        __syncthreads();
    }
    for (int e = tid; e < elems; e += NTT_THREADS) {
        u64 v = s[e];
        if (LAST) v = mul_shoup(v, M.n_inv, M.n_inv_sh, q);
        if (STRIDED) {
            int c = e % cols, u = e / cols;
            a[col0 + c + (size_t)u * stride] = v;
        } else {
            a[(size_t)col0 * r + e] = v;
        }
    }
}


// Shoup product for primes below 2^40, with x of any size below 2^64: the
// quotient estimate is the usual floor(x w' / 2^64), and since the remainder
// r = x w - qh q lies in [0, 2q) below 2^41, only r mod 2^42 is formed.  Its
// upper ten bits need the cross products only mod 2^10, which full-rate
// 24-bit multiplies give (they use the low 24 bits of each operand).
// v_mul_u32_u24: low 32 bits of the product of the operands' low 24 bits (a
// full-rate VALU instruction; the compiler folds the masked C form into
// 64-bit multiply-adds instead).  Register operands only, no memory access.
__device__ __forceinline__ u32 mul_u24(u32 a, u32 b)
{
    u32 r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ u64 mul_shoup_lazy_small(u64 x, u64 w, u64 w_sh, u64 nq)
{
    const u64 qh = umulhi64(x, w_sh);
    const u32 x0 = (u32)x, x1 = (u32)(x >> 32), w0 = (u32)w, w1 = (u32)(w >> 32);
    const u32 h0 = (u32)qh, h1 = (u32)(qh >> 32), n0 = (u32)nq, n1 = (u32)(nq >> 32);
    u64 acc = (u64)h0 * n0;          // - qh q = qh (2^64 - q) mod 2^64
    acc += (u64)x0 * w0;
    const u32 c = mul_u24(x0, w1) + mul_u24(x1, w0) + mul_u24(h0, n1) + mul_u24(h1, n0);
    const u32 hi = ((u32)(acc >> 32) + c) & 0x3ffu;
    return ((u64)hi << 32) | (u32)acc;
}

// Radix-8 register rounds: each thread holds the 8 elements of its
// sub-transform that differ in three consecutive index bits, applies up to
// three butterfly stages in registers, and exchanges through LDS once per
// round (one barrier per three stages).  All index arithmetic is shifts and
// masks (sub-transform size and tile width are powers of two).  Within a
// stage the twiddle depends only on the held bits above the butterfly bit,
// so each distinct twiddle is loaded once per round.  The contiguous pass
// pads its LDS tile by one word per eight (u + u/8) so that the sixteen
// lanes serving one sub-transform hit distinct banks in every round.
//
// Rows of primes below 2^40 (SMALL, when both passes of the transform use
// these kernels) skip the per-stage reductions: forward values grow by 2q
// per stage from [0, q) (below 33q for N <= 2^16) and are reduced once at the
// end; inverse values double per stage (the difference term adds 2q 2^e at
// executed stage e so it stays non-negative) and the final product by N^-1
// reduces them.  Other rows keep the [0, 4q) / [0, 2q) invariants.
// Row access of a pass: load/store one word at global index g of the row, or
// two adjacent words (g even) on the contiguous 16-byte path.
struct RowIO {
    u64* __restrict__ a;
    __device__ __forceinline__ u64 load(int g) const { return a[g]; }
    __device__ __forceinline__ void store(int g, u64 v) const { a[g] = v; }
    __device__ __forceinline__ void load2(int g, u64& v0, u64& v1) const
    {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(a + g);
        v0 = v.x;
        v1 = v.y;
    }
    __device__ __forceinline__ void store2(int g, u64 v0, u64 v1) const
    {
        *reinterpret_cast<ulonglong2*>(a + g) = make_ulonglong2(v0, v1);
    }
};

// Arithmetic of a row (AR): 0 integer with [0, 4q) / [0, 2q) values, 1 the
// unreduced integer path of primes below 2^40, 2 binary64 for primes below
// 2^41 (the context's fp flag; tables twf / twfq, FpModulus).  In the binary64
// path the elements are integer-valued doubles: a forward (Cooley-Tukey)
// butterfly is (U + r, U - r) with r = fp_mulmod(V, w) in (-0.7 q, 0.7 q), so
// magnitudes grow by less than q per stage; an inverse (Gentleman-Sande)
// butterfly is (U + V, fp_mulmod(U - V, w)), at most doubling them, which a
// pass of at most 8 stages keeps below 2^49.  Every pass ends with canonical
// residues (the last inverse one after the product by N^-1).
// The twiddle pointers of the binary64 path are the twf / twfq tables passed
// through the same u64 parameters.
template <int AR>
struct ArithT { using V = u64; };
template <>
struct ArithT<2> { using V = double; };

// the arithmetic of a row of modulus q: binary64 when enabled and q < 2^41,
// else the unreduced integer path when allowed (lazy_small) and q < 2^40
__device__ __forceinline__ int row_arith(const DevCtx& ctx, u64 q, int lazy_small)
{
    if (ctx.fp && q < (1ull << 41)) return 2;
    return (lazy_small && q < (1ull << 40)) ? 1 : 0;
}

// An IO type with a nested Pre (operands of its store epilogue) has them
// loaded with the pass's input, so that their latency hides behind the
// butterflies: pre1 / pre2 fetch them for one word / two adjacent words, and
// store_pre / store2_pre complete the stores from them.
template <class IO, class = void>
struct IoPre {
    static constexpr bool on = false;
    struct type {};
};
template <class IO>
struct IoPre<IO, std::void_t<typename IO::Pre>> {
    static constexpr bool on = true;
    using type = typename IO::Pre;
};

template <int LOG_R, int TILE_LOG, bool STRIDED, bool INV, bool LAST, int AR, class IO>
__device__ __forceinline__ void ntt_r8_body(u64* __restrict__ s, const IO& io, const Modulus& M,
                                            const u64* __restrict__ tw, const u64* __restrict__ tw_sh, int log_n,
                                            int log_cols, int sigma0, const FpModulus* F = nullptr)
{
    constexpr bool SMALL = AR == 1;
    constexpr bool FP = AR == 2;
    using V = typename ArithT<AR>::V;
    constexpr int LOG_G = LOG_R - 3;  // threads per sub-transform: 2^LOG_G
    constexpr int ROUNDS = (LOG_R + 2) / 3;
    constexpr int R = 1 << LOG_R;
    constexpr int RP = R + R / 8;     // padded sub-transform stride (contiguous pass)
    const u64 q = M.q, q2 = 2 * q, nq = 0 - q;
    double fq = 0.0, fqinv = 0.0;
    if constexpr (FP) {
        fq = F->q;
        fqinv = F->qinv;
    }
    V* __restrict__ sv = reinterpret_cast<V*>(s);
    const double* __restrict__ twf = reinterpret_cast<const double*>(tw);
    const double* __restrict__ twfq = reinterpret_cast<const double*>(tw_sh);
    const int tid = threadIdx.x;
    const int cmask = (1 << log_cols) - 1;
    int c, g;
    if (STRIDED) { c = tid & cmask; g = tid >> log_cols; }
    else { g = tid & ((1 << LOG_G) - 1); c = tid >> LOG_G; }
    const int col = (blockIdx.x << log_cols) + c;
    const int log_stride = log_n - LOG_R;
    // local index u -> global index, LDS index
#define GIDX(u) (STRIDED ? col + ((u) << log_stride) : (col << LOG_R) + (u))
#define LIDX(u) (STRIDED ? ((u) << log_cols) + c : c * RP + (u) + ((u) >> 3))
    V x[8];
    typename IoPre<IO>::type pre;
#pragma clang loop unroll(full)
    for (int rho = 0; rho < ROUNDS; ++rho) {
        // bits held this round: [lo, lo + 3)
        const int lo = INV ? (3 * rho < LOG_R - 3 ? 3 * rho : LOG_R - 3)
                           : (LOG_R - 3 - 3 * rho > 0 ? LOG_R - 3 - 3 * rho : 0);
        const int umask = (1 << lo) - 1;
        const int ub = ((g >> lo) << (lo + 3)) | (g & umask);
        if (rho == 0) {
            u64 xi[8];
            if (!STRIDED && lo == 0) {
#pragma clang loop unroll(full)
                for (int h = 0; h < 4; ++h) io.load2(GIDX(ub) + 2 * h, xi[2 * h], xi[2 * h + 1]);
            } else {
#pragma clang loop unroll(full)
                for (int m = 0; m < 8; ++m) xi[m] = io.load(GIDX(ub | (m << lo)));
            }
            if constexpr (IoPre<IO>::on) {
                // the words this thread stores in the last round
                constexpr int rl = ROUNDS - 1;
                const int lo_l = INV ? (3 * rl < LOG_R - 3 ? 3 * rl : LOG_R - 3)
                                     : (LOG_R - 3 - 3 * rl > 0 ? LOG_R - 3 - 3 * rl : 0);
                const int ub_l = ((g >> lo_l) << (lo_l + 3)) | (g & ((1 << lo_l) - 1));
                if (!STRIDED && lo_l == 0) {
#pragma clang loop unroll(full)
                    for (int h = 0; h < 4; ++h) io.pre2(GIDX(ub_l) + 2 * h, pre, h);
                } else {
#pragma clang loop unroll(full)
                    for (int m = 0; m < 8; ++m) io.pre1(GIDX(ub_l | (m << lo_l)), pre, m);
                }
            }
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) {
                if constexpr (FP) x[m] = u2d(xi[m]);
                else x[m] = xi[m];
            }
        } else {
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) x[m] = sv[LIDX(ub | (m << lo))];
        }
#pragma clang loop unroll(full)
        for (int k = 0; k < 3; ++k) {
            int b, tau;
            if (!INV) { tau = 3 * rho + k; b = LOG_R - 1 - tau; }
            else { b = 3 * rho + k; tau = LOG_R - 1 - b; }
            if (tau < 0 || tau >= LOG_R || b < lo) continue;
            const int mb = b - lo;
            const int sigma = sigma0 + tau;
            const int shift = log_n - sigma;
            // inverse, SMALL: values entering this stage are below 2q 2^e,
            // e = stages already executed = log_n - 1 - sigma
            const u64 kdiff = (INV && SMALL) ? (q2 << (log_n - 1 - sigma)) : q2;
            // groups of held bits above mb share one twiddle
#pragma clang loop unroll(full)
            for (int hi = 0; hi < (4 >> mb); ++hi) {
                const int mbase = hi << (mb + 1);
                const int ti = (1 << sigma) + (GIDX(ub | (mbase << lo)) >> shift);
                if constexpr (FP) {
                    const double w = twf[ti], wq = twfq[ti];
#pragma clang loop unroll(full)
                    for (int low = 0; low < (1 << mb); ++low) {
                        const int m0 = mbase | low, m1 = m0 | (1 << mb);
                        if (!INV) {
                            const double r = fp_mulmod(x[m1], w, wq, fq);
                            const double U = x[m0];
                            x[m0] = U + r;
                            x[m1] = U - r;
                        } else {
                            const double U = x[m0], Vv = x[m1];
                            x[m0] = U + Vv;
                            x[m1] = fp_mulmod(U - Vv, w, wq, fq);
                        }
                    }
                } else {
                    const u64 w = tw[ti], wsh = tw_sh[ti];
#pragma clang loop unroll(full)
                    for (int low = 0; low < (1 << mb); ++low) {
                        const int m0 = mbase | low, m1 = m0 | (1 << mb);
                        if (!INV) {
                            u64 U = x[m0];
                            if (!SMALL) U = U >= q2 ? U - q2 : U;
                            const u64 Vv = SMALL ? mul_shoup_lazy_small(x[m1], w, wsh, nq)
                                                 : mul_shoup_lazy(x[m1], w, wsh, q);
                            x[m0] = U + Vv;
                            x[m1] = U - Vv + q2;
                        } else {
                            const u64 U = x[m0], Vv = x[m1];
                            const u64 sum = U + Vv;
                            x[m0] = SMALL ? sum : (sum >= q2 ? sum - q2 : sum);
                            x[m1] = SMALL ? mul_shoup_lazy_small(U - Vv + kdiff, w, wsh, nq)
                                          : mul_shoup_lazy(U - Vv + q2, w, wsh, q);
                        }
                    }
                }
            }
        }
        if (rho + 1 < ROUNDS) {
            if (rho > 0) __syncthreads();  // every thread has read this round's LDS values
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) sv[LIDX(ub | (m << lo))] = x[m];
            __syncthreads();
        } else {
            {
                u64 xo[8];
#pragma clang loop unroll(full)
                for (int m = 0; m < 8; ++m) {
                    if constexpr (FP) {
                        const double v = (INV && LAST) ? fp_mulmod(x[m], F->ninv, F->ninvq, fq) : x[m];
                        xo[m] = fp_canon(v, fq, fqinv);
                    } else {
                        u64 v = x[m];
                        if (LAST) {
                            if (INV) {
                                v = mul_shoup(v, M.n_inv, M.n_inv_sh, q);
                            } else if (SMALL) {
                                v = reduce64(v, q, M.ratio);
                            } else {
                                v = v >= q2 ? v - q2 : v;
                                v = v >= q ? v - q : v;
                            }
                        }
                        xo[m] = v;
                    }
                }
                if (!STRIDED && lo == 0) {
#pragma clang loop unroll(full)
                    for (int h = 0; h < 4; ++h) {
                        if constexpr (IoPre<IO>::on) io.store2_pre(GIDX(ub) + 2 * h, xo[2 * h], xo[2 * h + 1], pre, h);
                        else io.store2(GIDX(ub) + 2 * h, xo[2 * h], xo[2 * h + 1]);
                    }
                } else {
#pragma clang loop unroll(full)
                    for (int m = 0; m < 8; ++m) {
                        if constexpr (IoPre<IO>::on) io.store_pre(GIDX(ub | (m << lo)), xo[m], pre, m);
                        else io.store(GIDX(ub | (m << lo)), xo[m]);
                    }
                }
            }
        }
    }
#undef GIDX
#undef LIDX
}

// Runs the radix-8 body over a row of modulus index mi in its arithmetic
// (row_arith): binary64 tables and constants, or the integer tables.
template <int LOG_R, int TILE_LOG, bool STRIDED, bool INV, bool LAST, class IO>
__device__ __forceinline__ void ntt_r8_row(u64* __restrict__ s, const IO& io, const DevCtx& ctx, int mi,
                                           int log_cols, int sigma0, int lazy_small)
{
    const Modulus M = ctx.mod[mi];
    const int ar = row_arith(ctx, M.q, lazy_small);
    if (ar == 2) {
        const FpModulus F = ctx.fmod[mi];
        const double* tf = (INV ? ctx.itwf : ctx.twf) + (size_t)mi * ctx.n;
        const double* tq = (INV ? ctx.itwfq : ctx.twfq) + (size_t)mi * ctx.n;
        ntt_r8_body<LOG_R, TILE_LOG, STRIDED, INV, LAST, 2>(s, io, M, reinterpret_cast<const u64*>(tf),
                                                            reinterpret_cast<const u64*>(tq), ctx.log_n, log_cols,
                                                            sigma0, &F);
        return;
    }
    const u64* __restrict__ tw = (INV ? ctx.itw : ctx.tw) + (size_t)mi * ctx.n;
    const u64* __restrict__ tw_sh = (INV ? ctx.itw_sh : ctx.tw_sh) + (size_t)mi * ctx.n;
    if (ar == 1)
        ntt_r8_body<LOG_R, TILE_LOG, STRIDED, INV, LAST, 1>(s, io, M, tw, tw_sh, ctx.log_n, log_cols, sigma0);
    else
        ntt_r8_body<LOG_R, TILE_LOG, STRIDED, INV, LAST, 0>(s, io, M, tw, tw_sh, ctx.log_n, log_cols, sigma0);
}

template <int LOG_R, int TILE_LOG, bool STRIDED, bool INV, bool LAST>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_ntt_r8(u64* __restrict__ data, DevCtx ctx, RowMap map,
                                                                int log_cols, int sigma0, int lazy_small)
{
    constexpr int T = 1 << TILE_LOG;
    __shared__ u64 s[T + T / 8];
    const int row = blockIdx.y;
    const int mi = rowmap_mod(map, row);
    const RowIO io{data + (size_t)row * ctx.n};
    ntt_r8_row<LOG_R, TILE_LOG, STRIDED, INV, LAST>(s, io, ctx, mi, log_cols, sigma0, lazy_small);
}

// ---- forward NTT fused with the lift before it and the combine after it
// (ModDown, relinearisation, rescale).  Row r of the transform is limb
// i = r % nl of polynomial pg = r / nl; polynomial pg = e * polys + p belongs
// to element e of the group.
//   column pass: reads source row pg (coefficient form, modulus src_mod) and
//                lifts it to q_i (centered) on load, writes row r of R;
//   row pass:    reads R in place and, instead of storing the transform t,
//                stores out_e[p][i] = (x_e[p][i] - t) * inv_i (+ addend).
struct LiftIO {
    const u64* __restrict__ src;
    u64* __restrict__ a;
    u64 p_half, p_mod_q, q, ratio;
    __device__ __forceinline__ u64 load(int g) const { return centered_lift(src[g], p_half, p_mod_q, q, ratio); }
    __device__ __forceinline__ void store(int g, u64 v) const { a[g] = v; }
    __device__ __forceinline__ void load2(int g, u64& v0, u64& v1) const
    {
        v0 = load(g);
        v1 = load(g + 1);
    }
    __device__ __forceinline__ void store2(int g, u64 v0, u64 v1) const
    {
        *reinterpret_cast<ulonglong2*>(a + g) = make_ulonglong2(v0, v1);
    }
};

struct FinishIO {
    u64* __restrict__ a;                 // R row (read)
    const u64* __restrict__ x;           // minuend row
    const u64* __restrict__ add;         // addend row or null
    u64* __restrict__ out;               // destination row
    u64 q, inv, inv_sh;
    u32 perm;                            // Galois element for reading the addend (1: none)
    int log_n;
    __device__ __forceinline__ u64 load(int g) const { return a[g]; }
    __device__ __forceinline__ void load2(int g, u64& v0, u64& v1) const
    {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(a + g);
        v0 = v.x;
        v1 = v.y;
    }
    __device__ __forceinline__ u64 addend(int g) const
    {
        if (!add) return 0;
        if (perm == 1) return add[g];
        // NTT-form automorphism: entry g of tau(a) is entry pi(g) of a,
        // 2 brev(pi(g)) + 1 = perm (2 brev(g) + 1) mod 2N
        const u32 bits = (u32)log_n;
        const u32 bg = __brev((u32)g) >> (32 - bits);
        const u32 e = (u32)(((u64)perm * (2u * bg + 1u)) & ((2u << bits) - 1u));
        return add[__brev((e - 1u) >> 1) >> (32 - bits)];
    }
    __device__ __forceinline__ u64 finish(u64 t, u64 xv, u64 av) const
    {
        const u64 v = mul_shoup(sub_mod(xv, t, q), inv, inv_sh, q);
        return add_mod(v, av, q);
    }
    __device__ __forceinline__ void store(int g, u64 t) const { out[g] = finish(t, x[g], addend(g)); }
    __device__ __forceinline__ void store2(int g, u64 t0, u64 t1) const
    {
        const ulonglong2 xv = *reinterpret_cast<const ulonglong2*>(x + g);
        u64 a0 = 0, a1 = 0;
        if (add && perm == 1) {
            const ulonglong2 av = *reinterpret_cast<const ulonglong2*>(add + g);
            a0 = av.x;
            a1 = av.y;
        } else if (add) {
            a0 = addend(g);
            a1 = addend(g + 1);
        }
        *reinterpret_cast<ulonglong2*>(out + g) = make_ulonglong2(finish(t0, xv.x, a0), finish(t1, xv.y, a1));
    }
    // epilogue operands fetched with the input (IoPre)
    struct Pre {
        u64 x[8], a[8];
    };
    __device__ __forceinline__ void pre1(int g, Pre& p, int m) const
    {
        p.x[m] = x[g];
        p.a[m] = addend(g);
    }
    __device__ __forceinline__ void pre2(int g, Pre& p, int h) const
    {
        const ulonglong2 xv = *reinterpret_cast<const ulonglong2*>(x + g);
        p.x[2 * h] = xv.x;
        p.x[2 * h + 1] = xv.y;
        if (add && perm == 1) {
            const ulonglong2 av = *reinterpret_cast<const ulonglong2*>(add + g);
            p.a[2 * h] = av.x;
            p.a[2 * h + 1] = av.y;
        } else {
            p.a[2 * h] = addend(g);
            p.a[2 * h + 1] = addend(g + 1);
        }
    }
    __device__ __forceinline__ void store_pre(int g, u64 t, const Pre& p, int m) const
    {
        out[g] = finish(t, p.x[m], p.a[m]);
    }
    __device__ __forceinline__ void store2_pre(int g, u64 t0, u64 t1, const Pre& p, int h) const
    {
        *reinterpret_cast<ulonglong2*>(out + g) =
            make_ulonglong2(finish(t0, p.x[2 * h], p.a[2 * h]), finish(t1, p.x[2 * h + 1], p.a[2 * h + 1]));
    }
};

// TAG names the step the kernel serves (0 ModDown, 1 rescale, 2 ModUp), so
// that profiles can tell them apart.  ModUp: rows r = (pg * nl) + s hold
// digit j = pg % nl of source row pg, lifted to target t = s < j ? s : s + 1
// (t = nl: the special prime); the source modulus is q_j.  Otherwise the
// source modulus is fa.src_mod and the target is q_s.
template <int LOG_R, int TILE_LOG, int TAG>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_ntt_r8_lift(u64* __restrict__ R, DevCtx ctx, FuseArgs fa,
                                                                     const u64* __restrict__ qmod, int n_mod,
                                                                     int log_cols, int lazy_small)
{
    constexpr int T = 1 << TILE_LOG;
    __shared__ u64 s[T + T / 8];
    const int row = blockIdx.y;
    const int i = row % fa.nl, pg = row / fa.nl;
    constexpr bool MODUP = TAG == 2;
    int sm = fa.src_mod, mi = i;
    if (MODUP) {
        sm = pg % fa.nl;
        const int t = i < sm ? i : i + 1;
        mi = t == fa.nl ? ctx.p_index : t;
    }
    const Modulus M = ctx.mod[mi];
    const LiftIO io{fa.src + (size_t)pg * ctx.n, R + (size_t)row * ctx.n, ctx.mod[sm].half,
                    qmod[(size_t)sm * n_mod + mi], M.q, M.ratio};
    ntt_r8_row<LOG_R, TILE_LOG, true, false, false>(s, io, ctx, mi, log_cols, 0, lazy_small);
}

// First (row) pass of an inverse NTT that gathers its input: row
// r = (blk * B + b) * nl + j reads limb j of polynomial b of source block blk,
// through the automorphism of Galois element perm[blk] when it is not 1.
struct GatherIO {
    const u64* __restrict__ src;
    u64* __restrict__ a;
    u32 perm;
    int log_n;
    __device__ __forceinline__ u64 load(int g) const
    {
        if (perm == 1) return src[g];
        const u32 bits = (u32)log_n;
        const u32 bg = __brev((u32)g) >> (32 - bits);
        const u32 e = (u32)(((u64)perm * (2u * bg + 1u)) & ((2u << bits) - 1u));
        return src[__brev((e - 1u) >> 1) >> (32 - bits)];
    }
    __device__ __forceinline__ void load2(int g, u64& v0, u64& v1) const
    {
        if (perm == 1) {
            const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(src + g);
            v0 = v.x;
            v1 = v.y;
        } else {
            v0 = load(g);
            v1 = load(g + 1);
        }
    }
    __device__ __forceinline__ void store(int g, u64 v) const { a[g] = v; }
    __device__ __forceinline__ void store2(int g, u64 v0, u64 v1) const
    {
        *reinterpret_cast<ulonglong2*>(a + g) = make_ulonglong2(v0, v1);
    }
};

// Forward row pass (stages sigma0 .. log N - 1, contiguous sub-transforms of
// 2^LOG_R points) of binary64 elements, for the row-fused inner product: the
// same rounds and index maps as ntt_r8_body (contiguous, forward), with the
// workgroup's twiddle pairs (w, fl(w / q)) read from LDS (tws: stage tau's
// entries at ((2^tau - 1) << log_cols) + (c << tau) + (u >> (LOG_R - tau))).
// x holds round 0's elements on entry and the thread's eight consecutive
// outputs (unreduced) on exit.
template <int LOG_R>
__device__ __forceinline__ void ks_fp_row_pass(double* __restrict__ sv, const double* __restrict__ tws,
                                               double (&x)[8], int g, int c, int log_cols, double q)
{
    constexpr int ROUNDS = (LOG_R + 2) / 3;
    constexpr int R = 1 << LOG_R;
    constexpr int RP = R + R / 8;
#define LIDXF(u) (c * RP + (u) + ((u) >> 3))
#pragma clang loop unroll(full)
    for (int rho = 0; rho < ROUNDS; ++rho) {
        const int lo = LOG_R - 3 - 3 * rho > 0 ? LOG_R - 3 - 3 * rho : 0;
        const int umask = (1 << lo) - 1;
        const int ub = ((g >> lo) << (lo + 3)) | (g & umask);
        if (rho > 0) {
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) x[m] = sv[LIDXF(ub | (m << lo))];
        }
#pragma clang loop unroll(full)
        for (int k = 0; k < 3; ++k) {
            const int tau = 3 * rho + k, b = LOG_R - 1 - tau;
            if (tau >= LOG_R || b < lo) continue;
            const int mb = b - lo;
#pragma clang loop unroll(full)
            for (int hi = 0; hi < (4 >> mb); ++hi) {
                const int mbase = hi << (mb + 1);
                const int u = ub | (mbase << lo);
                const int ei = (((1 << tau) - 1) << log_cols) + (c << tau) + (u >> (LOG_R - tau));
                const double2 wp = *reinterpret_cast<const double2*>(tws + 2 * ei);
#pragma clang loop unroll(full)
                for (int low = 0; low < (1 << mb); ++low) {
                    const int m0 = mbase | low, m1 = m0 | (1 << mb);
                    const double rr = fp_mulmod(x[m1], wp.x, wp.y, q);
                    const double U = x[m0];
                    x[m0] = U + rr;
                    x[m1] = U - rr;
                }
            }
        }
        if (rho + 1 < ROUNDS) {
            if (rho > 0) __syncthreads();
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) sv[LIDXF(ub | (m << lo))] = x[m];
            __syncthreads();
        }
    }
#undef LIDXF
}

// The integer counterpart of ks_fp_row_pass for primes of any size below
// 2^61: Cooley-Tukey butterflies with Shoup products on values kept in
// [0, 4q) (the general path of ntt_r8_body), twiddle pairs (w, w') from LDS in
// the same layout; on exit the thread's eight outputs are canonical.
template <int LOG_R>
__device__ __forceinline__ void ks_int_row_pass(u64* __restrict__ sv, const u64* __restrict__ tws, u64 (&x)[8],
                                                int g, int c, int log_cols, u64 q)
{
    constexpr int ROUNDS = (LOG_R + 2) / 3;
    constexpr int R = 1 << LOG_R;
    constexpr int RP = R + R / 8;
    const u64 q2 = 2 * q;
#define LIDXI(u) (c * RP + (u) + ((u) >> 3))
#pragma clang loop unroll(full)
    for (int rho = 0; rho < ROUNDS; ++rho) {
        const int lo = LOG_R - 3 - 3 * rho > 0 ? LOG_R - 3 - 3 * rho : 0;
        const int umask = (1 << lo) - 1;
        const int ub = ((g >> lo) << (lo + 3)) | (g & umask);
        if (rho > 0) {
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) x[m] = sv[LIDXI(ub | (m << lo))];
        }
#pragma clang loop unroll(full)
        for (int k = 0; k < 3; ++k) {
            const int tau = 3 * rho + k, b = LOG_R - 1 - tau;
            if (tau >= LOG_R || b < lo) continue;
            const int mb = b - lo;
#pragma clang loop unroll(full)
            for (int hi = 0; hi < (4 >> mb); ++hi) {
                const int mbase = hi << (mb + 1);
                const int u = ub | (mbase << lo);
                const int ei = (((1 << tau) - 1) << log_cols) + (c << tau) + (u >> (LOG_R - tau));
                const ulonglong2 wp = *reinterpret_cast<const ulonglong2*>(tws + 2 * ei);
#pragma clang loop unroll(full)
                for (int low = 0; low < (1 << mb); ++low) {
                    const int m0 = mbase | low, m1 = m0 | (1 << mb);
                    u64 U = x[m0];
                    U = U >= q2 ? U - q2 : U;
                    const u64 Vv = mul_shoup_lazy(x[m1], wp.x, wp.y, q);
                    x[m0] = U + Vv;
                    x[m1] = U - Vv + q2;
                }
            }
        }
        if (rho + 1 < ROUNDS) {
            if (rho > 0) __syncthreads();
#pragma clang loop unroll(full)
            for (int m = 0; m < 8; ++m) sv[LIDXI(ub | (m << lo))] = x[m];
            __syncthreads();
        }
    }
#pragma clang loop unroll(full)
    for (int m = 0; m < 8; ++m) {
        u64 v = x[m];
        v = v >= q2 ? v - q2 : v;
        x[m] = v >= q ? v - q : v;
    }
#undef LIDXI
}

// The row pass of ModUp's forward NTT fused with the key-switch inner
// product of a group of rotations whose digits are those of tau(c1) itself
// (plain rotations).  Workgroup (tile, r = i E B + eb), eb = e B + b, owns the
// tile's slots of target limb t = tgt[i] (t = nl: P) of element e, batch
// entry b.  It starts its sums with the digit of limb t itself (limb t of
// tau(c1), read from dsrc through gdig), then for each digit j != t runs the
// row pass of modup row ((blk_e B + b) nl + j) nl + s (s: the target's place
// among digit j's targets; the column pass is done) in LDS and adds its
// outputs times element e's key rows (j, c, t).  The sums go to U (t < nl) /
// Up (t = nl), or with EXT to dst_e as (P tau(c0) + U_0, U_1).  The
// transformed digits never reach memory.  Needs nl >= 2 (at least one digit
// row per target).  Targets are split between two kernels: k_ks_rowfp for
// the binary64 rows (row_arith 2), k_ntt_r8_ksrow for the integer ones.
struct KsTargets {
    int nt;
    int tgt[UH_MAX_MODULI];
};
static_assert(sizeof(GroupArgs) + sizeof(KsTargets) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT,
              "row-fused inner-product arguments too large for the kernel-argument segment");

// output rows of target t and the stores of the thread's eight sums
__device__ __forceinline__ void ks_row_store(u64 (&a0)[8], u64 (&a1)[8], bool ext, const GroupArgs& ga,
                                             const DevCtx& ctx, u64* U, u64* Up, int e, int b, int eb, int t, int nl,
                                             int base, u64 q)
{
    const int n = ctx.n;
    u64 *o0, *o1;
    if (ext) {
        const size_t row = (size_t)b * 2 * (nl + 1) + t;
        o0 = ga.dst[e] + row * n;
        o1 = ga.dst[e] + (row + nl + 1) * n;
        if (t < nl) {
            const u64 pm = ctx.p_mod[2 * t], pm_sh = ctx.p_mod[2 * t + 1];
            const u64* __restrict__ c0 = ga.src[e] + ((size_t)b * 2 * nl + t) * n;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const u64 x = c0[auto_perm((u32)(base + m), ga.g[e], ctx.log_n)];
                a0[m] = add_mod(a0[m], mul_shoup(x, pm, pm_sh, q), q);
            }
        }
    } else if (t < nl) {
        o0 = U + (((size_t)eb * 2 + 0) * nl + t) * n;
        o1 = U + (((size_t)eb * 2 + 1) * nl + t) * n;
    } else {
        o0 = Up + ((size_t)eb * 2 + 0) * n;
        o1 = Up + ((size_t)eb * 2 + 1) * n;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        *reinterpret_cast<ulonglong2*>(o0 + base + 2 * h) = make_ulonglong2(a0[2 * h], a0[2 * h + 1]);
        *reinterpret_cast<ulonglong2*>(o1 + base + 2 * h) = make_ulonglong2(a1[2 * h], a1[2 * h + 1]);
    }
}

// Binary64 targets.  The workgroup's twiddle pairs of the row pass go to LDS
// once; each digit row's round-0 elements are loaded one row ahead and its
// key words before its transform, so their loads overlap the arithmetic of
// the row before; the sums stay unreduced doubles (at most n_data + 1 terms
// below 0.7 q) and carry the keys' Montgomery factor 2^64, removed once at
// the end.
template <int LOG_R, int TILE_LOG, bool EXT>
__device__ __forceinline__ void ks_fp_wg(double* __restrict__ s, u64* __restrict__ U, u64* __restrict__ Up,
                                         const u64* __restrict__ modup, const GroupArgs& ga, const DevCtx& ctx,
                                         const KsTargets& kt, int nl, int nd, int B, int log_cols, int sigma0)
{
    constexpr int T = 1 << TILE_LOG;
    const int n = ctx.n;
    const int r = blockIdx.y, EB = gridDim.y / kt.nt;
    const int t = kt.tgt[r / EB], eb = r % EB;
    const int e = eb / B, b = eb % B;
    const int tm = t == nl ? ctx.p_index : t;
    const int klimb = t == nl ? nd : t;
    const FpModulus F = ctx.fmod[tm];
    const int blk = ga.blk[e];
    const u64* __restrict__ key = ga.key[e];
    const int gth = threadIdx.x & ((1 << (LOG_R - 3)) - 1), cth = threadIdx.x >> (LOG_R - 3);
    const int rowbase = ((blockIdx.x << log_cols) + cth) << LOG_R;
    const int base = rowbase + (gth << 3);
    double* __restrict__ tws = s + T + T / 8;
    {
        const double* __restrict__ twf = ctx.twf + (size_t)tm * n;
        const double* __restrict__ twq = ctx.twfq + (size_t)tm * n;
        const int nthr = 1 << (LOG_R - 3 + log_cols);
#pragma unroll 1
        for (int tau = 0; tau < LOG_R; ++tau) {
            const int cnt = 1 << (log_cols + tau);
            const int off = ((1 << tau) - 1) << log_cols;
            const int t0 = (1 << (sigma0 + tau)) + (blockIdx.x << (log_cols + tau));
            for (int ei = threadIdx.x; ei < cnt; ei += nthr) {
                tws[2 * (off + ei)] = twf[t0 + ei];
                tws[2 * (off + ei) + 1] = twq[t0 + ei];
            }
        }
    }
    double f0[8], f1[8];
    if (t < nl) {
        const u64* __restrict__ dl = ga.dsrc[blk] + ((size_t)b * ga.dstride + t) * n;
        const u64* __restrict__ k0 = key + (((size_t)t * 2 + 0) * (nd + 1) + klimb) * n;
        const u64* __restrict__ k1 = key + (((size_t)t * 2 + 1) * (nd + 1) + klimb) * n;
        const u32 gd = ga.gdig[e];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const double d = u2d(dl[auto_perm((u32)(base + m), gd, ctx.log_n)]);
            f0[m] = fp_mulmod_var(d, u2d(k0[base + m]), F.qinv, F.q);
            f1[m] = fp_mulmod_var(d, u2d(k1[base + m]), F.qinv, F.q);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) f0[m] = f1[m] = 0.0;
    }
    constexpr int LO0 = LOG_R - 3;  // round 0 holds elements gth + m 2^LO0
    const size_t rstride = (size_t)nl * n;  // modup rows of consecutive digits j (same target place s)
    const u64* __restrict__ rows = modup + (((size_t)blk * B + b) * nl * nl) * n + rowbase;
    auto row_of = [&](int j) { return rows + (size_t)j * rstride + (size_t)(t < j ? t : t - 1) * n; };
    u64 xn[8];
    int j = t == 0 ? 1 : 0;  // first digit j != t
    {
        const u64* __restrict__ rp = row_of(j);
#pragma unroll
        for (int m = 0; m < 8; ++m) xn[m] = rp[gth | (m << LO0)];
    }
    __syncthreads();  // twiddle pairs written
#pragma unroll 1
    while (j < nl) {
        double x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = u2d(xn[m]);
        int jn = j + 1;
        if (jn == t) ++jn;
        if (jn < nl) {
            const u64* __restrict__ rp = row_of(jn);
#pragma unroll
            for (int m = 0; m < 8; ++m) xn[m] = rp[gth | (m << LO0)];
        }
        const u64* __restrict__ kr0 = key + (((size_t)j * 2 + 0) * (nd + 1) + klimb) * n + base;
        const u64* __restrict__ kr1 = key + (((size_t)j * 2 + 1) * (nd + 1) + klimb) * n + base;
        u64 kw0[8], kw1[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const ulonglong2 v0 = *reinterpret_cast<const ulonglong2*>(kr0 + 2 * h);
            const ulonglong2 v1 = *reinterpret_cast<const ulonglong2*>(kr1 + 2 * h);
            kw0[2 * h] = v0.x;
            kw0[2 * h + 1] = v0.y;
            kw1[2 * h] = v1.x;
            kw1[2 * h + 1] = v1.y;
        }
        ks_fp_row_pass<LOG_R>(s, tws, x, gth, cth, log_cols, F.q);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            f0[m] += fp_mulmod_var(x[m], u2d(kw0[m]), F.qinv, F.q);
            f1[m] += fp_mulmod_var(x[m], u2d(kw1[m]), F.qinv, F.q);
        }
        __syncthreads();  // the next row's first LDS writes must follow this row's last reads
        j = jn;
    }
    // the sums carry the keys' factor 2^64: times 2^-64 mod q, canonical
    u64 a0[8], a1[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        a0[m] = fp_canon(fp_mulmod(f0[m], F.rinv, F.rinvq, F.q), F.q, F.qinv);
        a1[m] = fp_canon(fp_mulmod(f1[m], F.rinv, F.rinvq, F.q), F.q, F.qinv);
    }
    ks_row_store(a0, a1, EXT, ga, ctx, U, Up, e, b, eb, t, nl, base, ctx.mod[tm].q);
}

// Integer targets (any prime below 2^61): the same structure as ks_fp_wg
// with Shoup products on [0, 4q) values (ks_int_row_pass) and Montgomery
// products with the key words, reduced per term.
template <int LOG_R, int TILE_LOG, bool EXT>
__device__ __forceinline__ void ks_int_wg(u64* __restrict__ s, u64* __restrict__ U, u64* __restrict__ Up,
                                          const u64* __restrict__ modup, const GroupArgs& ga, const DevCtx& ctx,
                                          const KsTargets& kt, int nl, int nd, int B, int log_cols, int sigma0)
{
    constexpr int T = 1 << TILE_LOG;
    const int n = ctx.n;
    const int r = blockIdx.y, EB = gridDim.y / kt.nt;
    const int t = kt.tgt[r / EB], eb = r % EB;
    const int e = eb / B, b = eb % B;
    const int tm = t == nl ? ctx.p_index : t;
    const int klimb = t == nl ? nd : t;
    const Modulus M = ctx.mod[tm];
    const int blk = ga.blk[e];
    const u64* __restrict__ key = ga.key[e];
    const int gth = threadIdx.x & ((1 << (LOG_R - 3)) - 1), cth = threadIdx.x >> (LOG_R - 3);
    const int rowbase = ((blockIdx.x << log_cols) + cth) << LOG_R;
    const int base = rowbase + (gth << 3);
    u64* __restrict__ tws = s + T + T / 8;
    {
        const u64* __restrict__ tw = ctx.tw + (size_t)tm * n;
        const u64* __restrict__ tws_g = ctx.tw_sh + (size_t)tm * n;
        const int nthr = 1 << (LOG_R - 3 + log_cols);
#pragma unroll 1
        for (int tau = 0; tau < LOG_R; ++tau) {
            const int cnt = 1 << (log_cols + tau);
            const int off = ((1 << tau) - 1) << log_cols;
            const int t0 = (1 << (sigma0 + tau)) + (blockIdx.x << (log_cols + tau));
            for (int ei = threadIdx.x; ei < cnt; ei += nthr) {
                tws[2 * (off + ei)] = tw[t0 + ei];
                tws[2 * (off + ei) + 1] = tws_g[t0 + ei];
            }
        }
    }
    u64 a0[8], a1[8];
    if (t < nl) {
        const u64* __restrict__ dl = ga.dsrc[blk] + ((size_t)b * ga.dstride + t) * n;
        const u64* __restrict__ k0 = key + (((size_t)t * 2 + 0) * (nd + 1) + klimb) * n;
        const u64* __restrict__ k1 = key + (((size_t)t * 2 + 1) * (nd + 1) + klimb) * n;
        const u32 gd = ga.gdig[e];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const u64 d = dl[auto_perm((u32)(base + m), gd, ctx.log_n)];
            a0[m] = mont_mul(d, k0[base + m], M.q, M.qinv_neg);
            a1[m] = mont_mul(d, k1[base + m], M.q, M.qinv_neg);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) a0[m] = a1[m] = 0;
    }
    constexpr int LO0 = LOG_R - 3;
    const size_t rstride = (size_t)nl * n;
    const u64* __restrict__ rows = modup + (((size_t)blk * B + b) * nl * nl) * n + rowbase;
    auto row_of = [&](int j) { return rows + (size_t)j * rstride + (size_t)(t < j ? t : t - 1) * n; };
    u64 xn[8];
    int j = t == 0 ? 1 : 0;
    {
        const u64* __restrict__ rp = row_of(j);
#pragma unroll
        for (int m = 0; m < 8; ++m) xn[m] = rp[gth | (m << LO0)];
    }
    __syncthreads();  // twiddle pairs written
#pragma unroll 1
    while (j < nl) {
        u64 x[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) x[m] = xn[m];
        int jn = j + 1;
        if (jn == t) ++jn;
        if (jn < nl) {
            const u64* __restrict__ rp = row_of(jn);
#pragma unroll
            for (int m = 0; m < 8; ++m) xn[m] = rp[gth | (m << LO0)];
        }
        const u64* __restrict__ kr0 = key + (((size_t)j * 2 + 0) * (nd + 1) + klimb) * n + base;
        const u64* __restrict__ kr1 = key + (((size_t)j * 2 + 1) * (nd + 1) + klimb) * n + base;
        u64 kw0[8], kw1[8];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const ulonglong2 v0 = *reinterpret_cast<const ulonglong2*>(kr0 + 2 * h);
            const ulonglong2 v1 = *reinterpret_cast<const ulonglong2*>(kr1 + 2 * h);
            kw0[2 * h] = v0.x;
            kw0[2 * h + 1] = v0.y;
            kw1[2 * h] = v1.x;
            kw1[2 * h + 1] = v1.y;
        }
        ks_int_row_pass<LOG_R>(s, tws, x, gth, cth, log_cols, M.q);
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            a0[m] = add_mod(a0[m], mont_mul(x[m], kw0[m], M.q, M.qinv_neg), M.q);
            a1[m] = add_mod(a1[m], mont_mul(x[m], kw1[m], M.q, M.qinv_neg), M.q);
        }
        __syncthreads();  // the next row's first LDS writes must follow this row's last reads
        j = jn;
    }
    ks_row_store(a0, a1, EXT, ga, ctx, U, Up, e, b, eb, t, nl, base, M.q);
}

// Kernels over a target list: the binary64 targets alone (k_ks_rowfp), the
// integer ones alone (k_ntt_r8_ksrow), or both in one grid (k_ks_rowmix, the
// target list ordered integer targets first so that their longer workgroups
// start first).
template <int LOG_R, int TILE_LOG, bool EXT>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_ks_rowfp(u64* __restrict__ U, u64* __restrict__ Up,
                                                                  const u64* __restrict__ modup, GroupArgs ga,
                                                                  DevCtx ctx, KsTargets kt, int nl, int nd, int B,
                                                                  int log_cols, int sigma0)
{
    constexpr int T = 1 << TILE_LOG;
    // exchange tile, then up to T twiddle pairs of the row pass
    __shared__ double s[T + T / 8 + 2 * T];
    ks_fp_wg<LOG_R, TILE_LOG, EXT>(s, U, Up, modup, ga, ctx, kt, nl, nd, B, log_cols, sigma0);
}

template <int LOG_R, int TILE_LOG, bool EXT>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_ntt_r8_ksrow(u64* __restrict__ U, u64* __restrict__ Up,
                                                                      const u64* __restrict__ modup, GroupArgs ga,
                                                                      DevCtx ctx, KsTargets kt, int nl, int nd, int B,
                                                                      int log_cols, int sigma0)
{
    constexpr int T = 1 << TILE_LOG;
    __shared__ u64 s[T + T / 8 + 2 * T];
    ks_int_wg<LOG_R, TILE_LOG, EXT>(s, U, Up, modup, ga, ctx, kt, nl, nd, B, log_cols, sigma0);
}

template <int LOG_R, int TILE_LOG, bool EXT>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_ks_rowmix(u64* __restrict__ U, u64* __restrict__ Up,
                                                                   const u64* __restrict__ modup, GroupArgs ga,
                                                                   DevCtx ctx, KsTargets kt, int nl, int nd, int B,
                                                                   int log_cols, int sigma0)
{
    constexpr int T = 1 << TILE_LOG;
    __shared__ double s[T + T / 8 + 2 * T];
    const int t = kt.tgt[blockIdx.y / (gridDim.y / kt.nt)];
    const u64 q = ctx.mod[t == nl ? ctx.p_index : t].q;
    if (row_arith(ctx, q, 1) == 2)
        ks_fp_wg<LOG_R, TILE_LOG, EXT>(s, U, Up, modup, ga, ctx, kt, nl, nd, B, log_cols, sigma0);
    else
        ks_int_wg<LOG_R, TILE_LOG, EXT>(reinterpret_cast<u64*>(s), U, Up, modup, ga, ctx, kt, nl, nd, B, log_cols,
                                        sigma0);
}

template <int LOG_R, int TILE_LOG>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_intt_r8_gather(u64* __restrict__ dcoef, DevCtx ctx,
                                                                        GatherArgs ga, int nl, int B, int log_cols,
                                                                        int sigma0, int lazy_small)
{
    constexpr int T = 1 << TILE_LOG;
    __shared__ u64 s[T + T / 8];
    const int row = blockIdx.y;
    const int j = row % nl, pb = row / nl;
    const int blk = pb / B, b = pb % B;
    const GatherIO io{ga.src[blk] + ((size_t)b * ga.stride + j) * ctx.n, dcoef + (size_t)row * ctx.n, ga.perm[blk],
                      ctx.log_n};
    ntt_r8_row<LOG_R, TILE_LOG, false, true, false>(s, io, ctx, ga.mod0 + j, log_cols, sigma0, lazy_small);
}

template <int LOG_R, int TILE_LOG, int TAG>
__global__ void __launch_bounds__((1 << TILE_LOG) / 8) k_ntt_r8_finish(u64* __restrict__ R, DevCtx ctx, FuseArgs fa,
                                                                       int log_cols, int sigma0, int lazy_small)
{
    constexpr int T = 1 << TILE_LOG;
    __shared__ u64 s[T + T / 8];
    const int row = blockIdx.y;
    const int i = row % fa.nl, pg = row / fa.nl;
    const int e = pg / fa.polys, p = pg % fa.polys, c = p & 1, b = p >> 1;
    const Modulus M = ctx.mod[i];
    const size_t n = (size_t)ctx.n;
    const u64* add = fa.add[e][c];
    const FinishIO io{R + (size_t)row * n,
                      fa.x[e] + ((size_t)p * fa.x_limbs + i) * n,
                      add ? add + ((size_t)b * fa.add_stride + i) * n : nullptr,
                      fa.out[e] + ((size_t)p * fa.nl + i) * n,
                      M.q, fa.inv[2 * i], fa.inv[2 * i + 1], fa.add_perm[e], ctx.log_n};
    ntt_r8_row<LOG_R, TILE_LOG, false, false, true>(s, io, ctx, i, log_cols, sigma0, lazy_small);
}

template <int LOG_R, int TILE_LOG>
void launch_r8(u64* data, const DevCtx& dev, const RowMap& map, int n_rows, int log_n, int sigma0, bool strided,
               bool inv, bool last, int lazy_small, hipStream_t st)
{
    const int avail_log = log_n - LOG_R;                 // log2 of sub-transforms per row
    int log_cols = TILE_LOG - LOG_R;                      // tile of 2^TILE_LOG words
    if (log_cols > avail_log) log_cols = avail_log;
    const int threads = 1 << (LOG_R - 3 + log_cols);
    dim3 grid(1 << (avail_log - log_cols), n_rows);
#define L8(S, I, Z) \
    k_ntt_r8<LOG_R, TILE_LOG, S, I, Z><<<grid, threads, 0, st>>>(data, dev, map, log_cols, sigma0, lazy_small)
    if (strided) {
        if (!inv) { if (last) L8(true, false, true); else L8(true, false, false); }
        else { if (last) L8(true, true, true); else L8(true, true, false); }
    } else {
        if (!inv) { if (last) L8(false, false, true); else L8(false, false, false); }
        else { if (last) L8(false, true, true); else L8(false, true, false); }
    }
#undef L8
}

// dispatch on the sub-transform size and tile; sizes below 8 points use the
// generic kernel
bool launch_pass_r8(u64* data, const DevCtx& dev, const RowMap& map, int n_rows, int log_n, int log_r, int sigma0,
                    bool strided, bool inv, bool last, int tile_log, int lazy_small, hipStream_t st)
{
#define LR(K)                                                                                      \
    case K:                                                                                        \
        if (tile_log == 12) launch_r8<K, 12>(data, dev, map, n_rows, log_n, sigma0, strided, inv, last, lazy_small, st); \
        else launch_r8<K, 11>(data, dev, map, n_rows, log_n, sigma0, strided, inv, last, lazy_small, st);      \
        return true;
    switch (log_r) {
    LR(3) LR(4) LR(5) LR(6) LR(7) LR(8)
    default: return false;
    }
#undef LR
}

void split(const unihenn_ctx* c, int* l1, int* l2)
{
    *l1 = c->ntt_split > 0 && c->ntt_split < c->log_n ? c->ntt_split : c->log_n / 2;
    *l2 = c->log_n - *l1;
}

int tile_cols(int log_r, int log_n)
{
    int r = 1 << log_r;
    int cols = TILE / r;
    int avail = 1 << (log_n - log_r);
    return cols < avail ? cols : avail;
}

}  // namespace

void launch_ntt_fwd(const unihenn_ctx* c, u64* data, int n_rows, const RowMap& map, hipStream_t st)
{
    if (n_rows <= 0) return;
    int l1, l2;
    split(c, &l1, &l2);
    // the unreduced small-prime path needs both passes in the radix-8 kernels
    const int lazy = (l1 >= 3 && l1 <= 8 && l2 >= 3 && l2 <= 8) ? 1 : 0;
    const double bytes = 16.0 * c->n * n_rows, half = 0.5 * c->n * n_rows;
    {
        LaunchTimer tm(KF_NTT_FWD_COL, bytes, st, half * l1);
        if (!launch_pass_r8(data, c->dev, map, n_rows, c->log_n, l1, 0, true, false, false, c->ntt_tile_log, lazy, st)) {
            int cols1 = tile_cols(l1, c->log_n);
            dim3 g1((1 << (c->log_n - l1)) / cols1, n_rows);
            k_ntt_fwd<true, false><<<g1, NTT_THREADS, 0, st>>>(data, c->dev, map, l1, cols1, 0);
        }
    }
    {
        LaunchTimer tm(KF_NTT_FWD_ROW, bytes, st, half * l2);
        if (!launch_pass_r8(data, c->dev, map, n_rows, c->log_n, l2, l1, false, false, true, c->ntt_tile_log, lazy, st)) {
            int cols2 = tile_cols(l2, c->log_n);
            dim3 g2((1 << (c->log_n - l2)) / cols2, n_rows);
            k_ntt_fwd<false, true><<<g2, NTT_THREADS, 0, st>>>(data, c->dev, map, l2, cols2, l1);
        }
    }
}

void launch_ntt_inv(const unihenn_ctx* c, u64* data, int n_rows, const RowMap& map, hipStream_t st)
{
    if (n_rows <= 0) return;
    int l1, l2;
    split(c, &l1, &l2);
    // the unreduced small-prime path needs both passes in the radix-8 kernels
    const int lazy = (l1 >= 3 && l1 <= 8 && l2 >= 3 && l2 <= 8) ? 1 : 0;
    const double bytes = 16.0 * c->n * n_rows, half = 0.5 * c->n * n_rows;
    {
        LaunchTimer tm(KF_NTT_INV_ROW, bytes, st, half * l2);
        if (!launch_pass_r8(data, c->dev, map, n_rows, c->log_n, l2, l1, false, true, false, c->ntt_tile_log, lazy, st)) {
            int cols2 = tile_cols(l2, c->log_n);
            dim3 g2((1 << (c->log_n - l2)) / cols2, n_rows);
            k_ntt_inv<false, false><<<g2, NTT_THREADS, 0, st>>>(data, c->dev, map, l2, cols2, l1);
        }
    }
    {
        LaunchTimer tm(KF_NTT_INV_COL, bytes, st, half * l1);
        if (!launch_pass_r8(data, c->dev, map, n_rows, c->log_n, l1, 0, true, true, true, c->ntt_tile_log, lazy, st)) {
            int cols1 = tile_cols(l1, c->log_n);
            dim3 g1((1 << (c->log_n - l1)) / cols1, n_rows);
            k_ntt_inv<true, true><<<g1, NTT_THREADS, 0, st>>>(data, c->dev, map, l1, cols1, 0);
        }
    }
}

// Lift + forward NTT + combine in two passes (both radix-8); false when the
// ring's split puts a pass outside the radix-8 kernels (the caller then runs
// the separate kernels).
bool launch_ntt_fwd_fused(const unihenn_ctx* c, u64* R, const FuseArgs& fa, int n_rows, KernelFamily fam,
                          hipStream_t st)
{
    int l1, l2;
    split(c, &l1, &l2);
    if (n_rows <= 0 || l1 < 3 || l1 > 8 || l2 < 3 || l2 > 8) return false;
    const int tile = c->ntt_tile_log == 12 ? 12 : 11;
    const double half = 0.5 * c->n * n_rows, rows = n_rows, polys = (double)n_rows / fa.nl;
    auto geom = [&](int log_r, int* log_cols, dim3* grid, int* threads) {
        const int avail_log = c->log_n - log_r;
        int lc = tile - log_r;
        if (lc > avail_log) lc = avail_log;
        *log_cols = lc;
        *threads = 1 << (log_r - 3 + lc);
        *grid = dim3(1 << (avail_log - lc), n_rows);
    };
    int lc, thr;
    dim3 grid;
    {
        // source rows once, R rows written
        LaunchTimer tm(fam, 8.0 * c->n * (polys + rows), st, half * l1);
        geom(l1, &lc, &grid, &thr);
#define LC(K, TL)                                                                                          \
    if (fam == KF_RESCALE)                                                                                 \
        k_ntt_r8_lift<K, TL, 1><<<grid, thr, 0, st>>>(R, c->dev, fa, c->d_qmod, (int)c->primes.size(), lc, 1); \
    else                                                                                                   \
        k_ntt_r8_lift<K, TL, 0><<<grid, thr, 0, st>>>(R, c->dev, fa, c->d_qmod, (int)c->primes.size(), lc, 1)
#define LCT(K) case K: if (tile == 12) { LC(K, 12); } else { LC(K, 11); } break;
        switch (l1) { LCT(3) LCT(4) LCT(5) LCT(6) LCT(7) LCT(8) }
#undef LCT
#undef LC
    }
    {
        // R rows read, minuend rows read, addend rows (c = 0 or both), outputs written
        LaunchTimer tm(fam, 8.0 * c->n * rows * 3.5, st, half * l2);
        geom(l2, &lc, &grid, &thr);
#define LF(K, TL)                                                                   \
    if (fam == KF_RESCALE) k_ntt_r8_finish<K, TL, 1><<<grid, thr, 0, st>>>(R, c->dev, fa, lc, l1, 1); \
    else k_ntt_r8_finish<K, TL, 0><<<grid, thr, 0, st>>>(R, c->dev, fa, lc, l1, 1)
#define LFT(K) case K: if (tile == 12) { LF(K, 12); } else { LF(K, 11); } break;
        switch (l2) { LFT(3) LFT(4) LFT(5) LFT(6) LFT(7) LFT(8) }
#undef LFT
#undef LF
    }
    return true;
}

// ModUp fused with its forward NTT: dcoef holds n_src coefficient-form rows
// (polynomial b, digit j) = row b * nl + j; modup receives rows
// ((b * nl + j) * nl + s), the digit lifted to target s < j ? s : s + 1 and
// transformed.  False when a pass is outside the radix-8 kernels.
bool launch_ntt_fwd_modup(const unihenn_ctx* c, u64* modup, const u64* dcoef, int n_src, int nl, hipStream_t st,
                          bool row_pass)
{
    int l1, l2;
    split(c, &l1, &l2);
    const int n_rows = n_src * nl;
    if (n_rows <= 0 || l1 < 3 || l1 > 8 || l2 < 3 || l2 > 8) return false;
    const int tile = c->ntt_tile_log == 12 ? 12 : 11;
    FuseArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.src = dcoef;
    fa.nl = nl;
    const double half = 0.5 * c->n * n_rows;
    {
        LaunchTimer tm(KF_MODUP, 8.0 * c->n * (n_src + n_rows), st, half * l1);
        const int avail_log = c->log_n - l1;
        int lc = tile - l1;
        if (lc > avail_log) lc = avail_log;
        const int thr = 1 << (l1 - 3 + lc);
        dim3 grid(1 << (avail_log - lc), n_rows);
#define LC(K, TL) \
    k_ntt_r8_lift<K, TL, 2><<<grid, thr, 0, st>>>(modup, c->dev, fa, c->d_qmod, (int)c->primes.size(), lc, 1)
#define LCT(K) case K: if (tile == 12) LC(K, 12); else LC(K, 11); break;
        switch (l1) { LCT(3) LCT(4) LCT(5) LCT(6) LCT(7) LCT(8) }
#undef LCT
#undef LC
    }
    if (row_pass) {
        LaunchTimer tm(KF_NTT_FWD_ROW, 16.0 * c->n * n_rows, st, half * l2);
        launch_pass_r8(modup, c->dev, rowmap_modup(nl, c->n_data), n_rows, c->log_n, l2, l1, false, false, true, tile,
                       1, st);
    }
    return true;
}

// LDS tile (log2 words) of the row-fused inner product: its own setting
// (ks_tile_log), at least one sub-transform of the row pass (2^l2 words)
static int ks_tile(const unihenn_ctx* c, int l2)
{
    int t = c->ks_tile_log ? c->ks_tile_log : (c->ntt_tile_log == 12 ? 12 : 11);
    if (t < 9) t = 9;
    if (t > 12) t = 12;
    return t < l2 ? l2 : t;
}

bool ks_rowfusable(const unihenn_ctx* c, int nl, int n_blocks)
{
    int l1, l2;
    split(c, &l1, &l2);
    // one grid row per (block, target limb)
    if (nl < 2 || l1 < 3 || l1 > 8 || l2 < 3 || l2 > 8 || (long)n_blocks * (nl + 1) > 65535) return false;
    // Each workgroup runs its n - 1 or n row passes one after another, so a
    // small group (few rotations at few limbs) is faster unfused, where the
    // row pass and the inner product each spread over many more workgroups:
    // fuse only with at least ks_fuse_min_wg workgroups (default 384, 1.5
    // per CU of a 256-CU device; measured on plain LeNet-1: 160 workgroups
    // 30 us fused against 19 us unfused, 432 workgroups 24 us against 28 us).
    const int tile = ks_tile(c, l2);
    const int avail_log = c->log_n - l2;
    const int lc = tile - l2 < avail_log ? tile - l2 : avail_log;
    // workgroups counted in units of 256 threads
    const long threads = (long)n_blocks * (nl + 1) * (1L << (avail_log - lc)) * (1L << (l2 - 3 + lc));
    return threads >= 256L * c->ks_fuse_min_wg;
}

void launch_ks_rowfused(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, const u64* modup, u64* U, u64* Up,
                        bool ext, hipStream_t st)
{
    int l1, l2;
    split(c, &l1, &l2);
    const int tile = ks_tile(c, l2);
    const int E = ga.E;
    // targets by arithmetic: binary64 rows (k_ks_rowfp) and integer rows (k_ntt_r8_ksrow)
    KsTargets tf, ti;
    memset(&tf, 0, sizeof(tf));
    memset(&ti, 0, sizeof(ti));
    for (int t = 0; t <= nl; ++t) {
        const u64 q = c->primes[t == nl ? c->n_data : t];
        if (c->dev.fp && q < (1ull << 41)) tf.tgt[tf.nt++] = t;
        else ti.tgt[ti.nt++] = t;
    }
    const int avail_log = c->log_n - l2;
    int lc = tile - l2;
    if (lc > avail_log) lc = avail_log;
    const int thr = 1 << (l2 - 3 + lc);
    // algorithmic bytes and butterfly-equivalents of a target list: per (e, b, t)
    // the digit rows after the column pass (n - 1, or n for P), the same-limb
    // digit (t < n), the outputs (2) and, extended, the c0 row (t < n); per
    // (e, t) the key rows (2 n); work: the row passes plus 2 n key products
    // per slot, a product counted as 52 / 38 butterflies
    auto accounting = [&](const KsTargets& k, double* bytes, double* ops) {
        double rows = 0, bf = 0, mac = 0;
        for (int i = 0; i < k.nt; ++i) {
            const int t = k.tgt[i];
            const double dig = t < nl ? nl - 1 : nl;
            rows += (double)E * B * (dig + (t < nl ? 1 : 0) + 2 + (ext && t < nl ? 1 : 0)) + (double)E * 2 * nl;
            bf += (double)E * B * dig * 0.5 * c->n * l2;
            mac += (double)E * B * 2.0 * nl * c->n;
        }
        *bytes = 8.0 * c->n * rows;
        *ops = bf + mac * 52.0 / 38.0;
    };
    if (!c->ks_split && tf.nt && ti.nt) {
        // one grid, integer targets first
        KsTargets all = ti;
        for (int i = 0; i < tf.nt; ++i) all.tgt[all.nt++] = tf.tgt[i];
        double by, op;
        accounting(all, &by, &op);
        LaunchTimer tm(KF_KS_ROWFUSED, by, st, op);
        dim3 grid(1 << (avail_log - lc), E * B * all.nt);
#define KM(K, TL)                                                                                             \
    if (ext) k_ks_rowmix<K, TL, true><<<grid, thr, 0, st>>>(U, Up, modup, ga, c->dev, all, nl, c->n_data, B, lc, l1); \
    else k_ks_rowmix<K, TL, false><<<grid, thr, 0, st>>>(U, Up, modup, ga, c->dev, all, nl, c->n_data, B, lc, l1)
#define KMT(K)                                     \
    case K:                                        \
        if (tile == 12) { KM(K, 12); }             \
        else if (tile == 11) { KM(K, 11); }        \
        else if (tile == 10) { KM(K, 10); }        \
        else { KM(K, 9); }                         \
        break;
        switch (l2) { KMT(3) KMT(4) KMT(5) KMT(6) KMT(7) KMT(8) }
#undef KMT
#undef KM
        return;
    }
    if (tf.nt) {
        double by, op;
        accounting(tf, &by, &op);
        LaunchTimer tm(KF_KS_ROWFUSED, by, st, op);
        dim3 grid(1 << (avail_log - lc), E * B * tf.nt);
#define KF(K, TL)                                                                                                 \
    if (ext) k_ks_rowfp<K, TL, true><<<grid, thr, 0, st>>>(U, Up, modup, ga, c->dev, tf, nl, c->n_data, B, lc, l1); \
    else k_ks_rowfp<K, TL, false><<<grid, thr, 0, st>>>(U, Up, modup, ga, c->dev, tf, nl, c->n_data, B, lc, l1)
#define KFT(K)                                     \
    case K:                                        \
        if (tile == 12) { KF(K, 12); }             \
        else if (tile == 11) { KF(K, 11); }        \
        else if (tile == 10) { KF(K, 10); }        \
        else { KF(K, 9); }                         \
        break;
        switch (l2) { KFT(3) KFT(4) KFT(5) KFT(6) KFT(7) KFT(8) }
#undef KFT
#undef KF
    }
    if (ti.nt) {
        double by, op;
        accounting(ti, &by, &op);
        LaunchTimer tm(KF_KS_INNER, by, st, op);
        dim3 grid(1 << (avail_log - lc), E * B * ti.nt);
#define KR(K, TL)                                                                                            \
    if (ext) k_ntt_r8_ksrow<K, TL, true><<<grid, thr, 0, st>>>(U, Up, modup, ga, c->dev, ti, nl, c->n_data, B, lc, l1); \
    else k_ntt_r8_ksrow<K, TL, false><<<grid, thr, 0, st>>>(U, Up, modup, ga, c->dev, ti, nl, c->n_data, B, lc, l1)
#define KRT(K)                                     \
    case K:                                        \
        if (tile == 12) { KR(K, 12); }             \
        else if (tile == 11) { KR(K, 11); }        \
        else if (tile == 10) { KR(K, 10); }        \
        else { KR(K, 9); }                         \
        break;
        switch (l2) { KRT(3) KRT(4) KRT(5) KRT(6) KRT(7) KRT(8) }
#undef KRT
#undef KR
    }
}

// Inverse NTT of gathered rows: dcoef row (blk * B + b) * nl + j is limb j
// of polynomial b of block blk (rows at ga.src[blk] + (b * ga.stride + j) * N,
// modulus index ga.mod0 + j), read through the automorphism ga.perm[blk]; the
// first pass loads them directly.  False when a pass is outside the radix-8
// kernels.
bool launch_ntt_inv_gather(const unihenn_ctx* c, u64* dcoef, const GatherArgs& ga, int D, int B, int nl,
                           hipStream_t st)
{
    int l1, l2;
    split(c, &l1, &l2);
    const int n_rows = D * B * nl;
    if (n_rows <= 0 || l1 < 3 || l1 > 8 || l2 < 3 || l2 > 8) return false;
    const int tile = c->ntt_tile_log == 12 ? 12 : 11;
    const double half = 0.5 * c->n * n_rows;
    {
        LaunchTimer tm(KF_NTT_INV_ROW, 16.0 * c->n * n_rows, st, half * l2);
        const int avail_log = c->log_n - l2;
        int lc = tile - l2;
        if (lc > avail_log) lc = avail_log;
        const int thr = 1 << (l2 - 3 + lc);
        dim3 grid(1 << (avail_log - lc), n_rows);
#define LG(K, TL) k_intt_r8_gather<K, TL><<<grid, thr, 0, st>>>(dcoef, c->dev, ga, nl, B, lc, l1, 1)
#define LGT(K) case K: if (tile == 12) LG(K, 12); else LG(K, 11); break;
        switch (l2) { LGT(3) LGT(4) LGT(5) LGT(6) LGT(7) LGT(8) }
#undef LGT
#undef LG
    }
    {
        LaunchTimer tm(KF_NTT_INV_COL, 16.0 * c->n * n_rows, st, half * l1);
        std::vector<int> mods(nl);
        for (int j = 0; j < nl; ++j) mods[j] = ga.mod0 + j;
        launch_pass_r8(dcoef, c->dev, ga.mod0 == 0 ? rowmap_ct(nl) : rowmap_list(mods), n_rows, c->log_n, l1, 0,
                       true, true, true, tile, 1, st);
    }
    return true;
}

// whether the fused transforms apply (both passes in the radix-8 kernels)
bool ntt_fusable(const unihenn_ctx* c)
{
    int l1, l2;
    split(c, &l1, &l2);
    return l1 >= 3 && l1 <= 8 && l2 >= 3 && l2 <= 8;
}
