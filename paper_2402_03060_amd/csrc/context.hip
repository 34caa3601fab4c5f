// Context: ring degree, modulus chain, NTT tables and per-prime constants,
// built on the host and uploaded once; plus error reporting and the
// per-kernel-family launch timers.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "dd.h"
#include "internal.h"

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

int uh_fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

extern "C" const char* unihenn_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- number theory (host)
static u64 h_mulmod(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
static u64 h_powmod(u64 b, u64 e, u64 m)
{
    u64 r = 1;
    b %= m;
    for (; e; e >>= 1) {
        if (e & 1) r = h_mulmod(r, b, m);
        b = h_mulmod(b, b, m);
    }
    return r;
}
static u64 h_inv(u64 a, u64 m) { return h_powmod(a % m, m - 2, m); }

// Miller-Rabin with the first twelve primes as bases (deterministic below 2^64)
static bool h_is_prime(u64 n)
{
    const u64 w[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (u64 p : w)
        if (n % p == 0) return n == p;
    u64 d = n - 1;
    int r = 0;
    while (!(d & 1)) { d >>= 1; ++r; }
    for (u64 a : w) {
        u64 x = h_powmod(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int i = 1; i < r && witness; ++i) {
            x = h_mulmod(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

// Largest unused prime below 2^bits, of that bit length, = 1 mod 2N.
static bool pick_prime(int bits, int log_n, const std::vector<u64>& used, u64* out)
{
    const u64 step = (u64)2 << log_n;
    const u64 floor_v = (u64)1 << (bits - 1);
    for (u64 p = ((u64)1 << bits) + 1 - step; p > floor_v; p -= step) {
        if (std::find(used.begin(), used.end(), p) != used.end()) continue;
        if (h_is_prime(p)) { *out = p; return true; }
    }
    return false;
}

// The numerically smallest primitive 2N-th root of unity mod q.
static u64 smallest_psi(u64 q, int n)
{
    u64 order = 2 * (u64)n, cof = (q - 1) / order, root = 0;
    for (u64 g = 2; g < q; ++g) {
        u64 c = h_powmod(g, cof, q);
        if (h_powmod(c, order / 2, q) == q - 1) { root = c; break; }
    }
    // all primitive roots are root^k, k odd; keep the smallest
    u64 best = root, sq = h_mulmod(root, root, q), cur = root;
    for (u64 k = 1; k < order; k += 2) {
        if (cur < best) best = cur;
        cur = h_mulmod(cur, sq, q);
    }
    return best;
}

static u64 shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

static u32 bitrev(u32 x, int bits)
{
    u32 r = 0;
    for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
    return r;
}

static Modulus make_modulus(u64 q, int n)
{
    Modulus m;
    memset(&m, 0, sizeof(m));
    m.q = q;
    m.ratio = (u64)(~(u64)0) / q;  // q odd: floor((2^64-1)/q) = floor(2^64/q)
    u64 inv = q;                    // q q = 1 mod 8
    for (int i = 0; i < 6; ++i) inv *= 2 - q * inv;
    m.qinv_neg = (u64)0 - inv;
    u64 r1 = (u64)(((u128)1 << 64) % q);
    m.r2 = h_mulmod(r1, r1, q);
    m.half = (q - 1) / 2;
    m.n_inv = h_inv((u64)n, q);
    m.n_inv_sh = shoup(m.n_inv, q);
    return m;
}

// cos(pi t / N) for t < 2N in double-double: symmetry down to [0, pi/4],
// then Taylor series of cos or sin in double-double.
static const dd DD_PI = {3.141592653589793116e+00, 1.224646799147353207e-16};

static dd dd_cos_sin_small(dd x, bool want_sin)
{
    // sum_k (-1)^k x^(2k + s) / (2k + s)!, s = 1 for sin
    dd x2 = dd_mul(x, x);
    dd term = want_sin ? x : dd_make(1.0, 0.0);
    dd sum = term;
    int k0 = want_sin ? 1 : 0;
    for (int k = 1; k < 40; ++k) {
        int a = 2 * k + k0 - 1, b = 2 * k + k0;
        term = dd_div_d(dd_mul(term, x2), (double)a * (double)b);
        term = dd_neg(term);
        sum = dd_add(sum, term);
        if (fabs(term.hi) < 1e-40) break;
    }
    return sum;
}

static dd dd_cos_pi_frac(long t, long n)  // cos(pi t / n), n a power of two
{
    long a = ((t % (2 * n)) + 2 * n) % (2 * n);
    if (a > n) a = 2 * n - a;   // cos(2 pi - x) = cos x
    bool neg = false;
    if (a > n / 2) { a = n - a; neg = true; }  // cos(pi - x) = -cos x
    dd r;
    if (4 * a <= n) {
        r = dd_cos_sin_small(dd_mul_d(DD_PI, (double)a / (double)n), false);
    } else {
        long b = n / 2 - a;  // cos x = sin(pi/2 - x)
        r = dd_cos_sin_small(dd_mul_d(DD_PI, (double)b / (double)n), true);
    }
    return neg ? dd_neg(r) : r;
}

extern "C" int unihenn_debug_cos_table(uint32_t log_n, double* out /* [2N][2] host */)
{
    long n = 1L << log_n;
    for (long t = 0; t < 2 * n; ++t) {
        dd v = dd_cos_pi_frac(t, n);
        out[2 * t] = v.hi;
        out[2 * t + 1] = v.lo;
    }
    return 0;
}

// ---------------------------------------------------------------- row maps
RowMap rowmap_ct(int n_limbs)
{
    RowMap m;
    memset(&m, 0, sizeof(m));
    m.kind = 0;
    m.period = n_limbs;
    for (int i = 0; i < n_limbs; ++i) m.mods[i] = i;
    return m;
}
RowMap rowmap_list(const std::vector<int>& mods)
{
    RowMap m;
    memset(&m, 0, sizeof(m));
    m.kind = 0;
    m.period = (int)mods.size();
    for (size_t i = 0; i < mods.size(); ++i) m.mods[i] = mods[i];
    return m;
}
RowMap rowmap_modup(int n_limbs, int p_index)
{
    RowMap m;
    memset(&m, 0, sizeof(m));
    m.kind = 1;
    m.period = n_limbs;
    for (int i = 0; i < n_limbs; ++i) m.mods[i] = i;
    m.mods[n_limbs] = p_index;
    return m;
}

// ---------------------------------------------------------------- context
extern "C" int unihenn_ctx_create(uint32_t log_n, const uint32_t* prime_bits, uint32_t n_data,
                                  uint32_t special_bits, double scale, unihenn_ctx** out)
{
    if (!out || !prime_bits) return uh_fail(UNIHENN_EINVAL, "null argument");
    if (log_n < 4 || log_n > 16) return uh_fail(UNIHENN_EINVAL, "log_n must be in 4..16");
    if (n_data < 1 || n_data + 1 > UH_MAX_MODULI - 1) return uh_fail(UNIHENN_EINVAL, "too many primes");
    std::vector<u64> primes;
    for (uint32_t i = 0; i <= n_data; ++i) {
        int b = (int)(i < n_data ? prime_bits[i] : special_bits);
        if (b < (int)log_n + 2 || b > 61) return uh_fail(UNIHENN_EINVAL, "prime size must be in log_n+2..61 bits");
        u64 p;
        if (!pick_prime(b, (int)log_n, primes, &p)) return uh_fail(UNIHENN_EINVAL, "no prime of that size");
        primes.push_back(p);
    }
    unihenn_ctx* c = new unihenn_ctx();
    c->log_n = (int)log_n;
    if (const char* v = getenv("UNIHENN_KS_FUSE_MIN_WG")) c->ks_fuse_min_wg = atoi(v);
    if (const char* v = getenv("UNIHENN_KSROW_TILE")) c->ks_tile_log = atoi(v);
    if (const char* v = getenv("UNIHENN_KSROW_SPLIT")) c->ks_split = atoi(v) != 0;
    c->n = 1 << log_n;
    c->n_data = (int)n_data;
    c->scale = scale;
    c->primes = primes;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return uh_fail(UNIHENN_EDEVICE, "no current HIP device");
    }
    const int n = c->n, nm = (int)primes.size();

    std::vector<u64> tw((size_t)4 * nm * n);
    for (int mi = 0; mi < nm; ++mi) {
        u64 q = primes[mi];
        c->host_mod.push_back(make_modulus(q, n));
        u64 psi = smallest_psi(q, n), psi_inv = h_inv(psi, q);
        std::vector<u64> pw(n), ipw(n);
        u64 a = 1, b = 1;
        for (int k = 0; k < n; ++k) { pw[k] = a; ipw[k] = b; a = h_mulmod(a, psi, q); b = h_mulmod(b, psi_inv, q); }
        for (int k = 0; k < n; ++k) {
            u32 r = bitrev((u32)k, c->log_n);
            size_t o = (size_t)mi * n + k;
            tw[o] = pw[r];
            tw[(size_t)nm * n + o] = shoup(pw[r], q);
            tw[(size_t)2 * nm * n + o] = ipw[r];
            tw[(size_t)3 * nm * n + o] = shoup(ipw[r], q);
        }
    }
    // binary64 tables for primes below 2^41: twiddles and twiddle / q
    std::vector<double> twf((size_t)4 * nm * n, 0.0);
    std::vector<FpModulus> fm(nm);
    memset(fm.data(), 0, sizeof(FpModulus) * nm);
    for (int mi = 0; mi < nm; ++mi) {
        const u64 q = primes[mi];
        if (q >= (1ull << 41)) continue;
        const double qd = (double)q;
        for (int k = 0; k < n; ++k) {
            const size_t o = (size_t)mi * n + k;
            twf[o] = (double)tw[o];
            twf[(size_t)nm * n + o] = (double)tw[o] / qd;
            twf[(size_t)2 * nm * n + o] = (double)tw[(size_t)2 * nm * n + o];
            twf[(size_t)3 * nm * n + o] = (double)tw[(size_t)2 * nm * n + o] / qd;
        }
        const u64 r64 = (u64)(((unsigned __int128)1 << 64) % q);
        const u64 rinv = h_inv(r64, q);
        fm[mi].q = qd;
        fm[mi].qinv = 1.0 / qd;
        fm[mi].ninv = (double)c->host_mod[mi].n_inv;
        fm[mi].ninvq = fm[mi].ninv / qd;
        fm[mi].rinv = (double)rinv;
        fm[mi].rinvq = (double)rinv / qd;
    }
    c->q_mod.resize((size_t)nm * nm);
    for (int a = 0; a < nm; ++a)
        for (int b = 0; b < nm; ++b) c->q_mod[(size_t)a * nm + b] = primes[a] % primes[b];
    // q_l^-1 mod q_i, i < l < n_data, as (value, shoup) pairs: [l][i][2]
    c->inv_last.assign((size_t)nm * nm * 2, 0);
    for (int l = 1; l < (int)n_data; ++l)
        for (int i = 0; i < l; ++i) {
            u64 v = h_inv(primes[l] % primes[i], primes[i]);
            c->inv_last[((size_t)l * nm + i) * 2] = v;
            c->inv_last[((size_t)l * nm + i) * 2 + 1] = shoup(v, primes[i]);
        }
    u64 P = primes[n_data];
    c->p_inv.assign((size_t)nm * 2, 0);
    c->p_mod.assign((size_t)nm * 2, 0);
    for (int i = 0; i < (int)n_data; ++i) {
        u64 v = h_inv(P % primes[i], primes[i]);
        c->p_inv[2 * i] = v;
        c->p_inv[2 * i + 1] = shoup(v, primes[i]);
        c->p_mod[2 * i] = P % primes[i];
        c->p_mod[2 * i + 1] = shoup(P % primes[i], primes[i]);
    }
    std::vector<uint32_t> ge(n / 2);
    u64 e = 1;
    for (int k = 0; k < n / 2; ++k) { ge[k] = (uint32_t)e; e = e * 5 % (2 * (u64)n); }
    std::vector<double> cs((size_t)4 * n);
    unihenn_debug_cos_table(log_n, cs.data());

    auto fail = [&](const char* what) {
        unihenn_ctx_destroy(c);
        return uh_fail(UNIHENN_ENOMEM, what);
    };
    if (hipMalloc(&c->d_mod, sizeof(Modulus) * nm) != hipSuccess) return fail("hipMalloc moduli");
    if (hipMalloc(&c->d_tw, sizeof(u64) * tw.size()) != hipSuccess) return fail("hipMalloc twiddles");
    if (hipMalloc(&c->d_qmod, sizeof(u64) * c->q_mod.size()) != hipSuccess) return fail("hipMalloc qmod");
    if (hipMalloc(&c->d_inv_last, sizeof(u64) * c->inv_last.size()) != hipSuccess) return fail("hipMalloc inv");
    if (hipMalloc(&c->d_p_inv, sizeof(u64) * c->p_inv.size()) != hipSuccess) return fail("hipMalloc pinv");
    if (hipMalloc(&c->d_p_mod, sizeof(u64) * c->p_mod.size()) != hipSuccess) return fail("hipMalloc pmod");
    if (hipMalloc(&c->d_galois_e, sizeof(uint32_t) * ge.size()) != hipSuccess) return fail("hipMalloc galois");
    if (hipMalloc(&c->d_cos, sizeof(double) * cs.size()) != hipSuccess) return fail("hipMalloc cos");
    if (hipMalloc(&c->d_fmod, sizeof(FpModulus) * nm) != hipSuccess) return fail("hipMalloc fp moduli");
    if (hipMalloc(&c->d_twf, sizeof(double) * twf.size()) != hipSuccess) return fail("hipMalloc fp twiddles");
    hipError_t up = hipMemcpy(c->d_mod, c->host_mod.data(), sizeof(Modulus) * nm, hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_tw, tw.data(), sizeof(u64) * tw.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_qmod, c->q_mod.data(), sizeof(u64) * c->q_mod.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess)
        up = hipMemcpy(c->d_inv_last, c->inv_last.data(), sizeof(u64) * c->inv_last.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_p_inv, c->p_inv.data(), sizeof(u64) * c->p_inv.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_p_mod, c->p_mod.data(), sizeof(u64) * c->p_mod.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_galois_e, ge.data(), sizeof(uint32_t) * ge.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_cos, cs.data(), sizeof(double) * cs.size(), hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_fmod, fm.data(), sizeof(FpModulus) * nm, hipMemcpyHostToDevice);
    if (up == hipSuccess) up = hipMemcpy(c->d_twf, twf.data(), sizeof(double) * twf.size(), hipMemcpyHostToDevice);
    if (up != hipSuccess) {
        unihenn_ctx_destroy(c);
        return uh_fail(UNIHENN_EDEVICE, std::string("constant upload: ") + hipGetErrorString(up));
    }

    c->dev.log_n = c->log_n;
    c->dev.n = n;
    c->dev.n_data = c->n_data;
    c->dev.p_index = c->n_data;
    c->dev.mod = c->d_mod;
    c->dev.tw = c->d_tw;
    c->dev.tw_sh = c->d_tw + (size_t)nm * n;
    c->dev.itw = c->d_tw + (size_t)2 * nm * n;
    c->dev.itw_sh = c->d_tw + (size_t)3 * nm * n;
    c->dev.p_mod = c->d_p_mod;
    c->dev.fmod = c->d_fmod;
    c->dev.twf = c->d_twf;
    c->dev.twfq = c->d_twf + (size_t)nm * n;
    c->dev.itwf = c->d_twf + (size_t)2 * nm * n;
    c->dev.itwfq = c->d_twf + (size_t)3 * nm * n;
    c->dev.fp = 1;
    if (const char* v = getenv("UNIHENN_NTT_FP")) c->dev.fp = atoi(v) != 0;
    *out = c;
    return UNIHENN_OK;
}

extern "C" int unihenn_ctx_destroy(unihenn_ctx* c)
{
    if (!c) return UNIHENN_OK;
    (void)hipFree(c->d_mod);
    (void)hipFree(c->d_tw);
    (void)hipFree(c->d_qmod);
    (void)hipFree(c->d_inv_last);
    (void)hipFree(c->d_p_inv);
    (void)hipFree(c->d_p_mod);
    (void)hipFree(c->d_galois_e);
    (void)hipFree(c->d_cos);
    (void)hipFree(c->d_fmod);
    (void)hipFree(c->d_twf);
    delete c;
    return UNIHENN_OK;
}

extern "C" int unihenn_ctx_primes(const unihenn_ctx* c, uint64_t* out)
{
    if (!c || !out) return uh_fail(UNIHENN_EINVAL, "null argument");
    for (size_t i = 0; i < c->primes.size(); ++i) out[i] = c->primes[i];
    return UNIHENN_OK;
}

// ---------------------------------------------------------------- launch timing
namespace {
struct Pending {
    int fam;
    double bytes, ops;
    hipEvent_t a, b;
};
std::mutex g_stats_mu;
bool g_stats_on = false;
std::vector<Pending> g_pending;
uint64_t g_launches[KF_COUNT];
double g_ms[KF_COUNT];
double g_bytes[KF_COUNT];
double g_ops[KF_COUNT];
const char* g_names[KF_COUNT] = {"ntt_fwd_col", "ntt_fwd_row", "ntt_inv_row", "ntt_inv_col", "modup", "ks_inner",
                                 "moddown", "rescale", "mac", "automorphism", "tensor", "add", "encode", "other",
                                 "ks_rowfused"};
}  // namespace

// fold finished timer pairs into the per-family totals (g_stats_mu held)
static void drain_pending_locked()
{
    for (auto& p : g_pending) {
        float ms = 0;
        if (hipEventSynchronize(p.b) != hipSuccess || hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) ms = 0;
        g_launches[p.fam]++;
        g_ms[p.fam] += ms;
        g_bytes[p.fam] += p.bytes;
        g_ops[p.fam] += p.ops;
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}

LaunchTimer::LaunchTimer(KernelFamily f, double b, hipStream_t s, double o)
    : fam(f), bytes(b), ops(o), stream(s), on(false)
{
    if (!g_stats_on) return;
    on = hipEventCreate(&ev0) == hipSuccess;
    if (on && hipEventCreate(&ev1) != hipSuccess) {
        (void)hipEventDestroy(ev0);
        on = false;
    }
    if (on) (void)hipEventRecord(ev0, s);
}

LaunchTimer::~LaunchTimer()
{
    if (!on) return;
    (void)hipEventRecord(ev1, stream);
    std::lock_guard<std::mutex> g(g_stats_mu);
    g_pending.push_back({(int)fam, bytes, ops, ev0, ev1});
    if (g_pending.size() > 8192) drain_pending_locked();  // bound the number of live events
}

void stats_collect()
{
    std::lock_guard<std::mutex> g(g_stats_mu);
    drain_pending_locked();
}

bool stats_enabled() { return g_stats_on; }

extern "C" int unihenn_stats_enable(int on)
{
    stats_collect();
    g_stats_on = on != 0;
    return UNIHENN_OK;
}

extern "C" int unihenn_stats_reset(void)
{
    stats_collect();
    for (int i = 0; i < KF_COUNT; ++i) { g_launches[i] = 0; g_ms[i] = 0; g_bytes[i] = 0; g_ops[i] = 0; }
    return UNIHENN_OK;
}

extern "C" int unihenn_stats_get(int family, uint64_t* launches, double* total_ms, double* bytes, double* ops)
{
    if (family < 0 || family >= KF_COUNT) return uh_fail(UNIHENN_EINVAL, "bad kernel family");
    stats_collect();
    if (launches) *launches = g_launches[family];
    if (total_ms) *total_ms = g_ms[family];
    if (bytes) *bytes = g_bytes[family];
    if (ops) *ops = g_ops[family];
    return UNIHENN_OK;
}

extern "C" const char* unihenn_kernel_family_name(int family)
{
    if (family < 0 || family >= KF_COUNT) return "";
    return g_names[family];
}
