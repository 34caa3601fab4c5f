// Internal structures shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/unihenn.h"
#include "modarith.h"

#define UH_MAX_MODULI 24

// Device-side view of the context, passed by value to kernels.
struct DevCtx {
    int log_n;
    int n;                 // ring degree N
    int n_data;            // data primes q_0..q_{L}
    int p_index;           // index of the special prime P (= n_data)
    const Modulus* mod;    // [n_data + 1]
    const u64* tw;         // forward twiddles  [n_mod][N]: psi^brev(k)
    const u64* tw_sh;      // Shoup companions
    const u64* itw;        // inverse twiddles  [n_mod][N]: psi^-brev(k)
    const u64* itw_sh;
    const u64* p_mod;      // [i][2]: P mod q_i and its Shoup companion, i < n_data
    // binary64 arithmetic for primes below 2^41 (FpModulus; other moduli hold zeros)
    const FpModulus* fmod; // [n_mod]
    const double* twf;     // [n_mod][N]: forward twiddles as doubles
    const double* twfq;    // fl(twiddle / q)
    const double* itwf;    // inverse twiddles
    const double* itwfq;
    int fp;                // 1: transforms of primes below 2^41 use the binary64 path
};

struct unihenn_ctx {
    int log_n = 0;
    int n = 0;
    int n_data = 0;
    double scale = 0;
    std::vector<u64> primes;          // data primes then P
    std::vector<Modulus> host_mod;
    // small constant tables on the host (read by launchers)
    std::vector<u64> q_mod;           // [a][b] = q_a mod q_b   (n_mod x n_mod)
    std::vector<u64> inv_last;        // [l][i] = q_l^-1 mod q_i (Shoup pair interleaved)
    std::vector<u64> p_inv;           // [i] = P^-1 mod q_i (value, shoup)
    std::vector<u64> p_mod;           // [i] = P mod q_i (value, shoup)
    // device memory
    Modulus* d_mod = nullptr;
    u64* d_tw = nullptr;              // 4 tables of n_mod * N
    u64* d_qmod = nullptr;            // q_mod on device
    u64* d_inv_last = nullptr;
    u64* d_p_inv = nullptr;
    u64* d_p_mod = nullptr;
    uint32_t* d_galois_e = nullptr;   // 5^k mod 2N, k < N/2
    double* d_cos = nullptr;          // cos(pi t / N) as double-double, t < 2N: [2N][2]
    FpModulus* d_fmod = nullptr;      // binary64 constants per modulus
    double* d_twf = nullptr;          // 4 tables of n_mod * N doubles (twf, twfq, itwf, itwfq)
    int device = 0;
    DevCtx dev;
    // launch parameters (defaults, or chosen by unihenn_autotune); every
    // choice gives the same results bit for bit
    int ntt_split = 0;                // stages in the column pass (0: log_n / 2)
    int ntt_tile_log = 11;            // LDS tile of the radix-8 passes: 2^11 or 2^12 words
    int mac_min_wg = 2048;            // workgroups a multi-output MAC launch aims for
    int ks_min_wg = 2048;             // workgroups a key-switch inner product aims for
    int ks_order = 0;                 // workgroup order of the grouped inner product (0, 1), 2: row-fused
    int ks_tile_log = 9;              // LDS tile of the row-fused inner product, 9..12 (2^9 words: one wave per workgroup)
    int ks_split = 0;                 // row-fused inner product: binary64 and integer targets in two launches
    int ks_fuse_min_wg = 384;         // order 2 fuses only launches of at least this many workgroups
                                      // (environment UNIHENN_KS_FUSE_MIN_WG at context creation)
};

// error reporting (thread-local message)
int uh_fail(int code, const std::string& msg);
#define UH_CHECK_HIP(expr)                                                                \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess) return uh_fail(UNIHENN_EDEVICE, std::string(#expr) + ": " + \
                                             hipGetErrorString(_e));                     \
    } while (0)

// -------------------------------------------------------------------------
// row -> modulus mapping for batched transforms and elementwise kernels
// -------------------------------------------------------------------------
// Rows are N-word polynomials laid out back to back.  Row r uses modulus
//   PERIODIC: mods[r % period]
//   MODUP:    r = j * n + s (digit j, slot s < n): target t = s < j ? s : s+1,
//             and t == n means the special prime (mods[n]); mods[] lists the
//             moduli of q_0..q_{n-1}, P.
struct RowMap {
    int kind;          // 0 periodic, 1 modup
    int period;        // periodic: period; modup: n
    int mods[UH_MAX_MODULI];
};

__host__ __device__ __forceinline__ int rowmap_mod(const RowMap& m, int r)
{
    if (m.kind == 0) return m.mods[r % m.period];
    int n = m.period;
    int j = (r / n) % n, s = r % n;
    int t = s < j ? s : s + 1;
    return m.mods[t];
}

RowMap rowmap_ct(int n_limbs);                       // rows [..][n_limbs]: mod = limb
RowMap rowmap_list(const std::vector<int>& mods);    // periodic over a list
RowMap rowmap_modup(int n_limbs, int p_index);

// -------------------------------------------------------------------------
// launchers (all asynchronous on `stream`)
// -------------------------------------------------------------------------
void launch_ntt_fwd(const unihenn_ctx* c, u64* data, int n_rows, const RowMap& map, hipStream_t s);
void launch_ntt_inv(const unihenn_ctx* c, u64* data, int n_rows, const RowMap& map, hipStream_t s);

// Lift + forward NTT + combine (ModDown, relinearisation, rescale) over the
// rows r = (e * polys + p) * nl + i of R:
//   R[r] = NTT(centered lift of src[e * polys + p] (modulus src_mod) to q_i)
//   out[e][p][i] = (x[e][(p * x_limbs + i)] - R[r]) * inv_i
//                  + add[e][p & 1][((p >> 1) * add_stride + i)] (read through
//                  the automorphism of Galois element add_perm[e] when != 1)
#define UH_FUSE_MAX 64
struct FuseArgs {
    const u64* src;
    int src_mod;
    int nl;                          // limbs of R and of the outputs
    int polys;                       // polynomials per element
    const u64* x[UH_FUSE_MAX];
    int x_limbs;
    const u64* add[UH_FUSE_MAX][2];
    int add_stride;
    u32 add_perm[UH_FUSE_MAX];
    u64* out[UH_FUSE_MAX];
    const u64* inv;                  // [i][2] value, Shoup companion
};
enum KernelFamily : int;
bool launch_ntt_fwd_fused(const unihenn_ctx* c, u64* R, const FuseArgs& fa, int n_rows, KernelFamily fam,
                          hipStream_t st);
// sources of a gathering inverse NTT (up to UH_FUSE_MAX blocks)
struct GatherArgs {
    const u64* src[UH_FUSE_MAX];
    u32 perm[UH_FUSE_MAX];
    int stride;                      // rows per polynomial in the sources
    int mod0;                        // modulus index of gathered limb j: mod0 + j
};
bool launch_ntt_inv_gather(const unihenn_ctx* c, u64* dcoef, const GatherArgs& ga, int D, int B, int nl,
                           hipStream_t st);
bool ntt_fusable(const unihenn_ctx* c);
// ModUp (centered lift of each digit to every other target) fused with the
// forward NTT of the lifted rows; false when not applicable
bool launch_ntt_fwd_modup(const unihenn_ctx* c, u64* modup, const u64* dcoef, int n_src, int nl, hipStream_t st,
                          bool row_pass = true);
// ModUp row pass fused with the inner product of plain rotations
// (k_ntt_r8_ksrow) over n_blocks = E B (element, batch entry) pairs; false
// when the ring's transform split or the grid does not allow it
bool ks_rowfusable(const unihenn_ctx* c, int nl, int n_blocks);
struct GroupArgs;
// requires ks_rowfusable(c, nl, ga.E * B)
void launch_ks_rowfused(const unihenn_ctx* c, const GroupArgs& ga, int B, int nl, const u64* modup, u64* U, u64* Up,
                        bool ext, hipStream_t st);

// kernel timing hooks (per kernel family), see unihenn_stats_*
enum KernelFamily : int {
    KF_NTT_FWD_COL = 0, KF_NTT_FWD_ROW, KF_NTT_INV_ROW, KF_NTT_INV_COL, KF_MODUP, KF_KS_INNER, KF_MODDOWN,
    KF_RESCALE, KF_MAC, KF_AUTO, KF_TENSOR, KF_ADD, KF_ENCODE, KF_OTHER, KF_KS_ROWFUSED, KF_COUNT
};
// Times one launch (or a group of launches) on its stream with HIP events when
// timing is on; `bytes` is the algorithmic traffic, `ops` the algorithmic
// operation count (NTT butterflies) of what it brackets.
struct LaunchTimer {
    LaunchTimer(KernelFamily f, double bytes, hipStream_t s, double ops = 0.0);
    ~LaunchTimer();
    KernelFamily fam;
    double bytes;
    double ops;
    hipStream_t stream;
    hipEvent_t ev0, ev1;
    bool on;
};
void stats_collect();
bool stats_enabled();

// network hooks for the tuner (network.hip)
struct unihenn_net;
int net_ks_group(const unihenn_net* net);
int net_ks_group_cap(const unihenn_ctx* c, const unihenn_net* net);
int net_set_ks_group(const unihenn_ctx* c, unihenn_net* net, int e);
void net_drop_graphs(unihenn_net* net);
int net_max_batch(const unihenn_net* net);
int net_in_limbs(const unihenn_net* net);
int net_n_out(const unihenn_net* net);
int net_n_inputs(const unihenn_net* net);
int net_mode(const unihenn_net* net);
void net_set_mode_raw(unihenn_net* net, int mode);
uint64_t net_fingerprint(const unihenn_net* net);
