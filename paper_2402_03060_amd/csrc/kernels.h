// Launchers of the elementwise kernels (kernels.hip) and the NTT (ntt.hip).
#pragma once
#include "internal.h"

// NTT-form automorphism: entry k of tau_g(a) is entry perm(k) of a, where
// 2 brev(perm(k)) + 1 = g (2 brev(k) + 1) mod 2N.
__device__ __forceinline__ u32 auto_perm(u32 k, u32 g, int log_n)
{
    const u32 bk = __brev(k) >> (32 - log_n);
    const u32 e = (u32)(((u64)g * (2u * bk + 1u)) & ((2u << log_n) - 1u));
    return __brev((e - 1u) >> 1) >> (32 - log_n);
}

#define UH_MAC_MAX_TERMS 128

// up to UH_MAC_MAX_TERMS (ciphertext batch, plaintext) pairs, passed by value
struct MacTerms {
    const u64* ct[UH_MAC_MAX_TERMS];  // [B][2][nl][N]
    const u64* pt[UH_MAC_MAX_TERMS];  // [nl][N], Montgomery form
};

void launch_automorphism(const unihenn_ctx* c, u64* out, const u64* in, int rows, u32 g, hipStream_t s);
void launch_modup(const unihenn_ctx* c, u64* out, const u64* dcoef, int batch, int nl, hipStream_t s);
void launch_ks_inner(const unihenn_ctx* c, u64* U, u64* Up, const u64* dntt, int d_stride, const u64* modup,
                     const u64* key, int nd, int batch, int nl, u32 g, hipStream_t s);
void launch_lift_last(const unihenn_ctx* c, u64* out, const u64* src, int n_src_rows, int nl, int src_mod,
                      KernelFamily fam, hipStream_t s);
void launch_sub_scale(const unihenn_ctx* c, u64* out, const u64* x, int x_limbs, const u64* r, const u64* inv,
                      int n_polys, int nl, const u64* add0, const u64* add1, int add_stride, KernelFamily fam,
                      hipStream_t s);
void launch_gather_rows(const unihenn_ctx* c, u64* dst, const u64* src, int rows, int per, int src_stride, int off,
                        hipStream_t s);
// pl (here and below): limb index taken modulo the special prime P (extended
// operands over {q_0..q_{nl-2}, P}, pl = nl - 1), or -1
void launch_mac(const unihenn_ctx* c, u64* acc, const MacTerms& terms, int n_terms, int nl, int batch, int accumulate,
                hipStream_t s, int pl = -1);
void launch_tensor_mul(const unihenn_ctx* c, u64* d0, u64* d1, u64* d2, const u64* a, const u64* b, int b_limbs,
                       int batch, int nl, hipStream_t s);
void launch_tensor_square(const unihenn_ctx* c, u64* d0, u64* d1, u64* d2, const u64* ct, int batch, int nl,
                          hipStream_t s);
void launch_add(const unihenn_ctx* c, u64* out, const u64* a, const u64* b, int rows, int nl, hipStream_t s);
void launch_add_plain(const unihenn_ctx* c, u64* out, const u64* a, const u64* pt, int batch, int nl, hipStream_t s);
void launch_mont_convert(const unihenn_ctx* c, u64* data, int rows, const RowMap& map, int to_mont, hipStream_t s);

// Galois element of a left rotation by `steps` slots: 5^(steps mod N/2) mod 2N
u32 galois_elt(const unihenn_ctx* c, long steps);

// ---- key switching core (evaluator.hip) ----
// Workspace rows (of N words) needed by the evaluator for `batch` ciphertexts at nl limbs.
size_t ks_ws_rows(int nl, int batch);
struct KsWs {
    u64* dcoef;   // [B][nl]       digits in coefficient form
    u64* modup;   // [B][nl][nl]   digits extended to the other moduli (NTT form)
    u64* U;       // [B][2][nl]    inner product, data limbs
    u64* Up;      // [B][2]        inner product, special-prime limb
    u64* R;       // [B][2][nl]    lifted special-prime limb
    u64* aux;     // [B][3][nl]    automorphism / tensor temporaries
};
KsWs ks_ws_carve(u64* base, int nl, int batch, int n);
// ModUp of d (NTT form, row (b, j) at d + (b * d_stride + j) * N)
void ks_modup(const unihenn_ctx* c, const u64* d, int d_stride, int batch, int nl, KsWs& ws, hipStream_t s);
// out[B][2][nl] = KS(tau_g(d)) after ks_modup(d), plus add0 on c = 0 and add1
// on c = 1 (rows (b, i) at add + (b * add_stride + i) * N)
void ks_finish(const unihenn_ctx* c, const u64* d, int d_stride, const u64* key, int nd, int batch, int nl, u32 g,
               u64* out, const u64* add0, const u64* add1, int add_stride, KsWs& ws, hipStream_t s);
void rescale_core(const unihenn_ctx* c, const u64* in, int batch, int nl, u64* out, KsWs& ws, hipStream_t s);

// ---- grouped rotations (several rotations per launch set) ----
#define UH_GROUP_MAX 64
struct GroupArgs {
    int E;                          // rotations in the group
    const u64* src[UH_GROUP_MAX];   // source ciphertexts [B][2][nl]
    u64* dst[UH_GROUP_MAX];         // destinations [B][2][nl]
    const u64* key[UH_GROUP_MAX];   // switching keys (device form)
    u32 g[UH_GROUP_MAX];            // Galois element of the rotation
    u32 gin[UH_GROUP_MAX];          // permutation applied when reading ModUp digits (hoisted: g, plain: 1)
    u32 gdig[UH_GROUP_MAX];         // permutation applied when reading the same-limb digit from dsrc
    int blk[UH_GROUP_MAX];          // ModUp block holding the element's digits
    const u64* dsrc[UH_GROUP_MAX];  // per ModUp block: NTT rows (b, j) at dsrc + (b * dstride + j) * N
    int dstride;
};
// ModUp of D polynomials (rows (b, j) at dsrc[d] + (b * dstride + j) * N, NTT
// form): dcoef [D][B][nl] and modup [D][B][nl][nl]
// perm (may be null): Galois element per block to read its rows through
// (honoured only where the fused transforms apply: ntt_fusable)
// row_pass = false asks to leave the digits after the column pass of their
// forward NTT; returns true when it did so (the fused transforms apply and
// ks_rowfusable holds), and then the inner product must run the row pass
// (group_switch / group_switch_ext with row_fused).
bool group_modup(const unihenn_ctx* c, int D, const u64* const* dsrc, int dstride, int B, int nl, u64* dcoef,
                 u64* modup, hipStream_t s, const u32* perm = nullptr, bool row_pass = true);
// inner product with each element's key, ModDown, and the c0 addend: aux holds
// tau_g(src) per element ([E][B][2][nl]); with c0_only the c0 rows of aux
// are computed here (hoisted), otherwise the caller filled aux.
// row_fused: modup holds the ModUp digits after the column pass of their
// forward NTT only (group_modup returned true); the row pass runs inside the
// inner product (launch_ks_rowfused).  Plain rotations only (gin = 1).
void group_switch(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, bool c0_only, const u64* modup, u64* aux,
                  u64* U, u64* Up, u64* R, hipStream_t s, bool row_fused = false);
// extended rotations (deferred ModDown): dst_e [B][2][nl+1] = (P tau(c0) +
// U_0, U_1) over {q_0..q_{nl-1}, P}, U the inner product of the digits in
// modup with element e's key; dst must not overlap any src
void group_switch_ext(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, const u64* modup, hipStream_t s,
                      bool row_fused = false);
// aux[e] = tau_{g_e}(src_e), both polynomials
void group_auto_both(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, u64* aux, hipStream_t s);

// ---- multiply-accumulate into several outputs at once (convolution) ----
#define UH_MACM_MAX_OUT 16
struct MacMulti {
    u64* acc[UH_MACM_MAX_OUT];          // outputs [B][2][nl]
    const u64* ct[UH_MAC_MAX_TERMS];    // terms [B][2][nl]
    const u64* pt_base;                 // plaintext (o, t) at pt_base + ((o * o_stride + t_off + t) * nl) * N
    int o_stride, t_off;
};
// acc[o] (+)= sum_t pt(o, t) (*) ct[t] for o < n_out, t < n_terms
void launch_mac_multi(const unihenn_ctx* c, const MacMulti& m, int n_out, int n_terms, int nl, int batch,
                      int accumulate, hipStream_t s, int pl = -1);

// ---- grouped elementwise steps (independent steps of one kind, one launch) ----
#define UH_EW_GROUP_MAX 32
struct EwGroup {
    int E;
    u64* out[UH_EW_GROUP_MAX];
    const u64* a[UH_EW_GROUP_MAX];
    const u64* b[UH_EW_GROUP_MAX];   // second operand (add) or plaintext (add_plain)
};
void launch_group_add(const unihenn_ctx* c, const EwGroup& g, int batch, int nl, bool plain, hipStream_t s,
                      int pl = -1);
// E independent sums of T ciphertext batches each (E * T <= UH_SUM_MAX_TERMS):
// out[e] (+)= sum_t in[e * T + t]
#define UH_SUM_MAX_TERMS 128
struct SumGroup {
    int E, T;
    u64* out[UH_EW_GROUP_MAX];
    const u64* in[UH_SUM_MAX_TERMS];
};
void launch_group_sum(const unihenn_ctx* c, const SumGroup& g, int batch, int nl, bool accumulate, hipStream_t s,
                      int pl = -1);
// out_e [B][2][nl+1] = P a_e ([B][2][nl]): limbs i < nl times P mod q_i, limb nl zero
void launch_group_to_ext(const unihenn_ctx* c, const EwGroup& g, int batch, int nl, hipStream_t s);
// ModDown of E extended ciphertext batches [B][2][nl+1] -> [B][2][nl]; ws
// holds E * B * 2 * (nl + 1) rows
void group_moddown(const unihenn_ctx* c, int E, const u64* const* in, u64* const* out, int batch, int nl, u64* ws,
                   hipStream_t s);
// rescale of E ciphertext batches [B][2][nl] -> [B][2][nl-1]; ws holds
// E * B * 2 * nl rows
void group_rescale(const unihenn_ctx* c, int E, const u64* const* in, u64* const* out, int batch, int nl, u64* ws,
                   hipStream_t s);
// square + relinearise + rescale of E ciphertext batches at nl limbs
// ([B][2][nl] -> [B][2][nl-1]); ws holds group_square_ws_rows rows
size_t group_square_ws_rows(int E, int nl, int batch);
// with in2: the product in[e] x in2[e] instead of the square (in2 rows have
// in2_limbs limbs per polynomial, the first nl used)
void group_square(const unihenn_ctx* c, int E, const u64* const* in, u64* const* out, const u64* rlk, int batch, int nl,
                  u64* ws, hipStream_t s, const u64* const* in2 = nullptr, int in2_limbs = 0);
// E single-output multiply-accumulates with T terms each (E * T <= 64)
#define UH_MACG_MAX 64
struct MacGroup {
    int E, T;
    u64* acc[UH_EW_GROUP_MAX];
    const u64* ct[UH_MACG_MAX];
    const u64* pt[UH_MACG_MAX];
};
void launch_mac_group(const unihenn_ctx* c, const MacGroup& m, int nl, int batch, hipStream_t s, int pl = -1);

// Launch descriptors travel by value in the kernel-argument segment, beside
// the DevCtx and a few scalars: each must stay below 4 KiB with that
// headroom.  group_switch fills FuseArgs and GatherArgs entries per group
// element, so a group may not be larger than those descriptors.
constexpr size_t UH_KERNARG_LIMIT = 4096;
constexpr size_t UH_KERNARG_HEADROOM = sizeof(DevCtx) + 128;
static_assert(sizeof(GroupArgs) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "GroupArgs too large for kernel arguments");
static_assert(sizeof(FuseArgs) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "FuseArgs too large for kernel arguments");
static_assert(sizeof(GatherArgs) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "GatherArgs too large for kernel arguments");
static_assert(sizeof(MacTerms) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "MacTerms too large for kernel arguments");
static_assert(sizeof(MacMulti) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "MacMulti too large for kernel arguments");
static_assert(sizeof(MacGroup) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "MacGroup too large for kernel arguments");
static_assert(sizeof(SumGroup) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "SumGroup too large for kernel arguments");
static_assert(sizeof(EwGroup) + UH_KERNARG_HEADROOM <= UH_KERNARG_LIMIT, "EwGroup too large for kernel arguments");
static_assert(UH_GROUP_MAX <= UH_FUSE_MAX, "a rotation group indexes FuseArgs / GatherArgs by element");
