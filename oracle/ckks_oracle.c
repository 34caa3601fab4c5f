/*
 * ckks_oracle.c -- plain, slow CPU reference of the CKKS arithmetic that the
 * UniHENN hot path is built from (UniHENN, Section II-B: Add, Mul(P), Mul(C),
 * Rot on CKKS ciphertexts in R_q^2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file.  It is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * Style: every operation is written the way its definition reads, with
 * "(unsigned __int128) a * b % q" for modular products, in coefficient form at
 * every entry point.  Polynomial products in Z_q[X]/(X^N+1) are computed by
 * twisting with a primitive 2N-th root psi and a textbook cyclic radix-2 DFT
 * (the twist turns the negacyclic product into a cyclic one); tests pin this
 * against a schoolbook product.
 *
 * Readings of the paper that this file fixes (the paper runs SEAL and does not
 * state them):
 *   - prime chain: for each requested bit size, in order, the largest unused
 *     prime p < 2^b with p = 1 (mod 2N) and bit length b;
 *   - slot k <-> root psi^(5^k mod 2N); left rotation by r <-> X -> X^(5^r);
 *   - encode rounds the exact real value half away from zero (computed in
 *     binary128) and reduces it modulo every prime;
 *   - key switching: one digit per data prime, digit lifted to the centered
 *     range, one special prime P, ModDown by exact rounding division by P;
 *   - rescale: exact rounding division by the last prime.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;
typedef __int128 i128;

/* ------------------------------------------------------------------------ */
/* modular arithmetic                                                        */
/* ------------------------------------------------------------------------ */
static u64 mul_mod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 add_mod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }
static u64 pow_mod(u64 b, u64 e, u64 q)
{
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mul_mod(r, b, q);
        b = mul_mod(b, b, q);
        e >>= 1;
    }
    return r;
}
static u64 inv_mod(u64 a, u64 q) { return pow_mod(a, q - 2, q); } /* q prime */
static u64 reduce_i128(i128 x, u64 q)
{
    i128 r = x % (i128)q;
    if (r < 0) r += (i128)q;
    return (u64)r;
}
/* representative of x mod q in (-q/2, q/2]; q is odd so the range is
 * symmetric: (-(q-1)/2 .. (q-1)/2) */
static i64 centered(u64 x, u64 q) { return x > (q - 1) / 2 ? (i64)x - (i64)q : (i64)x; }

/* ------------------------------------------------------------------------ */
/* primes                                                                    */
/* ------------------------------------------------------------------------ */
static int is_prime(u64 n)
{
    static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = pow_mod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) {
            x = mul_mod(x, x, n);
            if (x == n - 1) { comp = 0; break; }
        }
        if (comp) return 0;
    }
    return 1;
}

/* For each bit size bits[i] in order: the largest prime p < 2^b, p of bit
 * length b, p = 1 mod 2N, not chosen before.  Returns 0 or -1. */
int or_gen_primes(int log_n, const int *bits, int count, u64 *out)
{
    u64 two_n = (u64)2 << log_n;
    for (int i = 0; i < count; i++) {
        int b = bits[i];
        if (b < log_n + 2 || b > 61) return -1;
        u64 lo = (u64)1 << (b - 1);
        u64 p = ((u64)1 << b) - two_n + 1;
        int found = 0;
        for (; p > lo; p -= two_n) {
            if (!is_prime(p)) continue;
            int used = 0;
            for (int k = 0; k < i; k++) used |= (out[k] == p);
            if (used) continue;
            out[i] = p;
            found = 1;
            break;
        }
        if (!found) return -1;
    }
    return 0;
}

int or_is_prime(u64 n) { return is_prime(n); }

/* ------------------------------------------------------------------------ */
/* PRNG: xoshiro256** seeded through SplitMix64 (Blackman & Vigna).  A      */
/* research generator, not a cryptographic one.                              */
/* ------------------------------------------------------------------------ */
typedef struct { u64 s[4]; } prng_t;
static u64 splitmix64(u64 *x)
{
    u64 z = (*x += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
static u64 rotl(u64 x, int k) { return (x << k) | (x >> (64 - k)); }
static u64 prng_next(prng_t *p)
{
    u64 *s = p->s;
    u64 result = rotl(s[1] * 5, 7) * 9;
    u64 t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}
void *or_prng_new(u64 seed)
{
    prng_t *p = (prng_t *)malloc(sizeof(prng_t));
    u64 x = seed;
    for (int i = 0; i < 4; i++) p->s[i] = splitmix64(&x);
    return p;
}
void or_prng_free(void *p) { free(p); }

/* uniform ternary {-1,0,1}: two bits, rejecting the fourth value */
static int sample_ternary(prng_t *p)
{
    for (;;) {
        u64 r = prng_next(p) >> 62;
        if (r < 3) return (int)r - 1;
    }
}
/* one rounded-Gaussian candidate (Box-Muller, sigma = 3.2) from u1 in (0,1]
   and u2 in [0,1): returns 1 and stores it in *e when |e| <= 19 (accepted),
   0 when it must be redrawn */
int or_gauss_candidate(double u1, double u2, int *e)
{
    double z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    double r = nearbyint(3.2 * z);
    if (fabs(r) > 19.0) return 0;
    *e = (int)r;
    return 1;
}
static int sample_gauss(prng_t *p)
{
    for (;;) {
        double u1 = ((prng_next(p) >> 11) + 1) * 0x1p-53; /* (0,1] */
        double u2 = (prng_next(p) >> 11) * 0x1p-53;       /* [0,1) */
        int e;
        if (or_gauss_candidate(u1, u2, &e)) return e;
    }
}
/* uniform in [0,q) by rejection on the top bits */
static u64 sample_uniform(prng_t *p, u64 q)
{
    int bits = 64 - __builtin_clzll(q);
    for (;;) {
        u64 r = prng_next(p) >> (64 - bits);
        if (r < q) return r;
    }
}

/* n draws of one sampler (test hook): kind 0 ternary, 1 rounded Gaussian,
   2 uniform in [0, q) */
void or_sample(void *pv, int kind, u64 q, int n, int64_t *out)
{
    prng_t *p = (prng_t *)pv;
    for (int i = 0; i < n; i++)
        out[i] = kind == 0 ? sample_ternary(p) : kind == 1 ? sample_gauss(p) : (int64_t)sample_uniform(p, q);
}

/* ------------------------------------------------------------------------ */
/* context: N, moduli q_0..q_L and P, per-modulus transform tables           */
/* ------------------------------------------------------------------------ */
typedef struct {
    u64 q;
    u64 psi, psi_inv, n_inv;
    u64 *psi_pow;     /* psi^j, j < N      */
    u64 *psi_inv_pow; /* psi^-j, j < N     */
    u64 *w_fwd;       /* omega^j, j < N/2, omega = psi^2 */
    u64 *w_inv;       /* omega^-j          */
} modulus_t;

typedef struct {
    int log_n, n;
    int n_mod;        /* L+2: data primes then P */
    modulus_t *mod;
    u64 *galois_e;    /* e_k = 5^k mod 2N, k < N/2 */
    __float128 *cos_tab; /* cos(pi t / N), t < 2N */
    int *bitrev;
} ctx_t;

static u64 find_psi(u64 q, int n)
{
    u64 e = (q - 1) / (2 * (u64)n);
    for (u64 x = 2;; x++) {
        u64 g = pow_mod(x, e, q);
        if (pow_mod(g, (u64)n, q) == q - 1) return g; /* order exactly 2N */
    }
}

void *or_ctx_new(int log_n, const u64 *moduli, int n_mod)
{
    ctx_t *c = (ctx_t *)calloc(1, sizeof(ctx_t));
    c->log_n = log_n;
    c->n = 1 << log_n;
    c->n_mod = n_mod;
    int n = c->n;
    c->mod = (modulus_t *)calloc(n_mod, sizeof(modulus_t));
    for (int i = 0; i < n_mod; i++) {
        modulus_t *m = &c->mod[i];
        m->q = moduli[i];
        m->psi = find_psi(m->q, n);
        m->psi_inv = inv_mod(m->psi, m->q);
        m->n_inv = inv_mod((u64)n, m->q);
        m->psi_pow = (u64 *)malloc(sizeof(u64) * n);
        m->psi_inv_pow = (u64 *)malloc(sizeof(u64) * n);
        m->w_fwd = (u64 *)malloc(sizeof(u64) * (n / 2 + 1));
        m->w_inv = (u64 *)malloc(sizeof(u64) * (n / 2 + 1));
        u64 a = 1, b = 1;
        for (int j = 0; j < n; j++) {
            m->psi_pow[j] = a;
            m->psi_inv_pow[j] = b;
            a = mul_mod(a, m->psi, m->q);
            b = mul_mod(b, m->psi_inv, m->q);
        }
        u64 w = mul_mod(m->psi, m->psi, m->q), wi = mul_mod(m->psi_inv, m->psi_inv, m->q);
        a = 1; b = 1;
        for (int j = 0; j <= n / 2; j++) {
            m->w_fwd[j] = a;
            m->w_inv[j] = b;
            a = mul_mod(a, w, m->q);
            b = mul_mod(b, wi, m->q);
        }
    }
    c->bitrev = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; i++) {
        int r = 0;
        for (int b = 0; b < log_n; b++)
            if (i & (1 << b)) r |= 1 << (log_n - 1 - b);
        c->bitrev[i] = r;
    }
    c->galois_e = (u64 *)malloc(sizeof(u64) * (n / 2));
    u64 e = 1;
    for (int k = 0; k < n / 2; k++) {
        c->galois_e[k] = e;
        e = (e * 5) % (2 * (u64)n);
    }
    c->cos_tab = NULL; /* built on first encode */
    return c;
}

void or_ctx_free(void *vc)
{
    ctx_t *c = (ctx_t *)vc;
    for (int i = 0; i < c->n_mod; i++) {
        free(c->mod[i].psi_pow); free(c->mod[i].psi_inv_pow);
        free(c->mod[i].w_fwd); free(c->mod[i].w_inv);
    }
    free(c->mod); free(c->galois_e); free(c->cos_tab); free(c->bitrev);
    free(c);
}

u64 or_ctx_psi(void *vc, int mod_index) { return ((ctx_t *)vc)->mod[mod_index].psi; }

/* ------------------------------------------------------------------------ */
/* negacyclic products                                                       */
/* ------------------------------------------------------------------------ */
/* textbook cyclic DFT X_k = sum_j x_j w^{jk} (bit-reversal + iterative
 * radix-2 Cooley-Tukey); wtab holds w^j for j <= N/2 */
static void dft(const ctx_t *c, u64 *a, const u64 *wtab, u64 q)
{
    int n = c->n;
    for (int i = 0; i < n; i++) {
        int r = c->bitrev[i];
        if (i < r) { u64 t = a[i]; a[i] = a[r]; a[r] = t; }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int half = len / 2, step = n / len;
        for (int i = 0; i < n; i += len) {
            for (int j = 0; j < half; j++) {
                u64 u = a[i + j];
                u64 v = mul_mod(a[i + j + half], wtab[j * step], q);
                a[i + j] = add_mod(u, v, q);
                a[i + j + half] = sub_mod(u, v, q);
            }
        }
    }
}
/* a -> DFT(a_j psi^j): the negacyclic evaluation of a at the odd powers of psi */
static void to_eval(const ctx_t *c, int mi, const u64 *a, u64 *out)
{
    const modulus_t *m = &c->mod[mi];
    for (int j = 0; j < c->n; j++) out[j] = mul_mod(a[j], m->psi_pow[j], m->q);
    dft(c, out, m->w_fwd, m->q);
}
/* inverse of to_eval */
static void from_eval(const ctx_t *c, int mi, u64 *a)
{
    const modulus_t *m = &c->mod[mi];
    dft(c, a, m->w_inv, m->q);
    for (int j = 0; j < c->n; j++)
        a[j] = mul_mod(mul_mod(a[j], m->n_inv, m->q), m->psi_inv_pow[j], m->q);
}

/* out = a * b in Z_q[X]/(X^N+1), q = moduli[mi] */
void or_poly_mul(void *vc, int mi, const u64 *a, const u64 *b, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    u64 *ta = (u64 *)malloc(sizeof(u64) * n), *tb = (u64 *)malloc(sizeof(u64) * n);
    to_eval(c, mi, a, ta);
    to_eval(c, mi, b, tb);
    for (int j = 0; j < n; j++) ta[j] = mul_mod(ta[j], tb[j], c->mod[mi].q);
    from_eval(c, mi, ta);
    memcpy(out, ta, sizeof(u64) * n);
    free(ta); free(tb);
}

/* ------------------------------------------------------------------------ */
/* encode (Section II-B, III-A): real slot vector z, k < N/2, to the integer  */
/* plaintext round(scale * m_j) with m_j = (2/N) sum_k z_k cos(pi e_k j / N)  */
/* ------------------------------------------------------------------------ */
static void ensure_cos(ctx_t *c)
{
    if (c->cos_tab) return;
    int n = c->n;
    c->cos_tab = (__float128 *)malloc(sizeof(__float128) * 2 * n);
    for (int t = 0; t < 2 * n; t++) c->cos_tab[t] = cosq(M_PIq * (__float128)t / (__float128)n);
}

/* m_j of z in binary128, j < N (zero slots contribute nothing and are skipped) */
static void real_transform(ctx_t *c, const double *z, int n_slots, __float128 *m)
{
    int n = c->n;
    u64 two_n = 2 * (u64)n;
    ensure_cos(c);
    for (int j = 0; j < n; j++) m[j] = 0;
    for (int k = 0; k < n_slots; k++) {
        if (z[k] == 0.0) continue;
        __float128 zk = z[k];
        u64 ek = c->galois_e[k];
        for (int j = 0; j < n; j++) m[j] += zk * c->cos_tab[(ek * (u64)j) & (two_n - 1)];
    }
    __float128 f = 2.0Q / (__float128)n;
    for (int j = 0; j < n; j++) m[j] *= f;
}

/* limb i < n_limbs of coefficient j: the rounded value mod q_i; with ext
 * (n_limbs = nl + 1) the last limb is taken mod P */
static void round_reduce(const ctx_t *c, __float128 v, int n_limbs, u64 *out, int j, int ext)
{
    __float128 r = roundq(v); /* half away from zero */
    i128 iv = (i128)r;
    for (int i = 0; i < n_limbs; i++) {
        int mi = (ext && i == n_limbs - 1) ? c->n_mod - 1 : i;
        out[(size_t)i * c->n + j] = reduce_i128(iv, c->mod[mi].q);
    }
}

/* pt[i][j] for i < n_limbs.  Returns -1 if a coefficient does not fit. */
int or_encode(void *vc, const double *z, int n_slots, double scale, int n_limbs, u64 *pt)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    if (n_slots > n / 2) return -1;
    __float128 *m = (__float128 *)malloc(sizeof(__float128) * n);
    real_transform(c, z, n_slots, m);
    int rc = 0;
    for (int j = 0; j < n; j++) {
        __float128 v = (__float128)scale * m[j];
        if (fabsq(v) > 0x1p100Q) { rc = -1; break; }
        round_reduce(c, v, n_limbs, pt, j, 0);
    }
    free(m);
    return rc;
}

/* Encode(w_t * z) for several scalars w_t at once.  By linearity of the
 * exact transform, m(w z) = w m(z); the product scale * w is exact in
 * binary128, so only the final product with m_j is rounded before the
 * rounding to an integer.  out: [n_w][n_limbs][N]. */
static int encode_scaled(ctx_t *c, const double *z, int n_slots, const double *w, int n_w, double scale,
                         int n_limbs, int ext, u64 *out)
{
    int n = c->n;
    if (n_slots > n / 2) return -1;
    __float128 *m = (__float128 *)malloc(sizeof(__float128) * n);
    real_transform(c, z, n_slots, m);
    int rc = 0;
    for (int t = 0; t < n_w && rc == 0; t++) {
        __float128 sw = (__float128)scale * (__float128)w[t];
        u64 *pt = out + (size_t)t * n_limbs * n;
        for (int j = 0; j < n; j++) {
            __float128 v = sw * m[j];
            if (fabsq(v) > 0x1p100Q) { rc = -1; break; }
            round_reduce(c, v, n_limbs, pt, j, ext);
        }
    }
    free(m);
    return rc;
}

int or_encode_scaled(void *vc, const double *z, int n_slots, const double *w, int n_w, double scale,
                     int n_limbs, u64 *out)
{
    return encode_scaled((ctx_t *)vc, z, n_slots, w, n_w, scale, n_limbs, 0, out);
}

/* the same with the residue mod P as limb nl: out [n_w][nl+1][N], the
 * plaintexts of products with extended ciphertexts */
int or_encode_scaled_ext(void *vc, const double *z, int n_slots, const double *w, int n_w, double scale, int nl,
                         u64 *out)
{
    return encode_scaled((ctx_t *)vc, z, n_slots, w, n_w, scale, nl + 1, 1, out);
}

/* exact real transform, exported as hi/lo doubles for tests */
void or_real_transform(void *vc, const double *z, int n_slots, double *hi, double *lo)
{
    ctx_t *c = (ctx_t *)vc;
    __float128 *m = (__float128 *)malloc(sizeof(__float128) * c->n);
    real_transform(c, z, n_slots, m);
    for (int j = 0; j < c->n; j++) {
        hi[j] = (double)m[j];
        lo[j] = (double)(m[j] - (__float128)hi[j]);
    }
    free(m);
}

/* ------------------------------------------------------------------------ */
/* automorphism tau_g: a(X) -> a(X^g), g odd, in coefficient form           */
/* ------------------------------------------------------------------------ */
static void automorphism(const ctx_t *c, u64 q, const u64 *a, u64 g, u64 *out)
{
    int n = c->n;
    u64 two_n = 2 * (u64)n;
    for (int j = 0; j < n; j++) {
        u64 e = ((u64)j * g) % two_n; /* X^j -> X^(jg) = +-X^(jg mod N) */
        if (e < (u64)n) out[e] = a[j];
        else out[e - n] = a[j] ? q - a[j] : 0;
    }
}

/* Galois element of a left rotation by r slots: 5^(r mod N/2) mod 2N */
u64 or_galois_elt(void *vc, i64 r)
{
    ctx_t *c = (ctx_t *)vc;
    i64 h = c->n / 2;
    i64 rr = ((r % h) + h) % h;
    return c->galois_e[rr];
}

void or_automorphism(void *vc, const u64 *poly, int n_limbs, u64 g, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    for (int i = 0; i < n_limbs; i++)
        automorphism(c, c->mod[i].q, poly + (size_t)i * c->n, g, out + (size_t)i * c->n);
}

/* ------------------------------------------------------------------------ */
/* keys and encryption (client side)                                        */
/* ------------------------------------------------------------------------ */
/* secret key: ternary coefficients */
void or_gen_secret(void *vc, void *vp, int8_t *s)
{
    ctx_t *c = (ctx_t *)vc;
    for (int j = 0; j < c->n; j++) s[j] = (int8_t)sample_ternary((prng_t *)vp);
}

/* residues of a small signed polynomial modulo moduli[mi] */
static void small_to_mod(const ctx_t *c, const i64 *x, int mi, u64 *out)
{
    for (int j = 0; j < c->n; j++) out[j] = reduce_i128(x[j], c->mod[mi].q);
}

/* public key over the data primes q_0..q_L: (-a s + e, a).  pk: [2][L+1][N] */
void or_gen_pk(void *vc, void *vp, const int8_t *s, int n_data, u64 *pk)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    i64 *e = (i64 *)malloc(sizeof(i64) * n), *si = (i64 *)malloc(sizeof(i64) * n);
    u64 *sm = (u64 *)malloc(sizeof(u64) * n), *as = (u64 *)malloc(sizeof(u64) * n);
    for (int j = 0; j < n; j++) { e[j] = sample_gauss((prng_t *)vp); si[j] = s[j]; }
    for (int i = 0; i < n_data; i++) {
        u64 q = c->mod[i].q;
        u64 *p0 = pk + (size_t)i * n, *p1 = pk + ((size_t)n_data + i) * n;
        for (int j = 0; j < n; j++) p1[j] = sample_uniform((prng_t *)vp, q);
        small_to_mod(c, si, i, sm);
        or_poly_mul(c, i, p1, sm, as);
        for (int j = 0; j < n; j++) p0[j] = sub_mod(reduce_i128(e[j], q), as[j], q);
    }
    free(e); free(si); free(sm); free(as);
}

/* Switching key for target polynomial t (small signed coefficients), over
 * the basis {q_0..q_L, P} (n_data = L+1 data primes, P = moduli[n_data]):
 *   evk_j = (-a_j s + e_j + [i == j] (P mod q_i) t, a_j)   for j <= L.
 * key: [L+1][2][L+2][N]. */
/* Switching key for target t (C3): digit d, basis limb i (q_0..q_{n_data-1},
 * then P) holds (-a s + e + [i = d] (P mod q_i) t, a).  With levels < n_data
 * only the rows a ciphertext of `levels` limbs reads are formed (digits below
 * `levels`, limbs below `levels` and P); the others stay zero.  Every random
 * draw is still made, so the formed rows equal those of the whole key. */
static void gen_switch_key_rows(ctx_t *c, prng_t *p, const int8_t *s, const i64 *t, int n_data, int levels,
                                u64 *key)
{
    int n = c->n, nb = n_data + 1;
    i64 *e = (i64 *)malloc(sizeof(i64) * n), *si = (i64 *)malloc(sizeof(i64) * n);
    u64 *sm = (u64 *)malloc(sizeof(u64) * n), *as = (u64 *)malloc(sizeof(u64) * n);
    u64 P = c->mod[n_data].q;
    for (int j = 0; j < n; j++) si[j] = s[j];
    for (int d = 0; d < n_data; d++) {
        for (int k = 0; k < n; k++) e[k] = sample_gauss(p);
        for (int i = 0; i < nb; i++) {
            u64 q = c->mod[i].q;
            u64 *k0 = key + (((size_t)d * 2 + 0) * nb + i) * n;
            u64 *k1 = key + (((size_t)d * 2 + 1) * nb + i) * n;
            for (int k = 0; k < n; k++) k1[k] = sample_uniform(p, q);
            if (d >= levels || (i >= levels && i != n_data)) {
                memset(k0, 0, sizeof(u64) * n);
                memset(k1, 0, sizeof(u64) * n);
                continue;
            }
            small_to_mod(c, si, i, sm);
            or_poly_mul(c, i, k1, sm, as);
            u64 pmod = P % q;
            for (int k = 0; k < n; k++) {
                u64 v = sub_mod(reduce_i128(e[k], q), as[k], q);
                if (i == d) v = add_mod(v, mul_mod(pmod, reduce_i128(t[k], q), q), q);
                k0[k] = v;
            }
        }
    }
    free(e); free(si); free(sm); free(as);
}

/* rotation key for a left rotation by r: target tau_g(s), g = 5^r mod 2N;
 * or_gen_rotation_key_rows forms only the rows of `levels` limbs */
void or_gen_rotation_key_rows(void *vc, void *vp, const int8_t *s, int n_data, i64 r, int levels, u64 *key);
void or_gen_rotation_key(void *vc, void *vp, const int8_t *s, int n_data, i64 r, u64 *key)
{
    or_gen_rotation_key_rows(vc, vp, s, n_data, r, n_data, key);
}
void or_gen_rotation_key_rows(void *vc, void *vp, const int8_t *s, int n_data, i64 r, int levels, u64 *key)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    u64 g = or_galois_elt(vc, r);
    i64 *t = (i64 *)malloc(sizeof(i64) * n);
    u64 two_n = 2 * (u64)n;
    for (int j = 0; j < n; j++) {
        u64 e = ((u64)j * g) % two_n;
        if (e < (u64)n) t[e] = s[j];
        else t[e - n] = -(i64)s[j];
    }
    gen_switch_key_rows(c, (prng_t *)vp, s, t, n_data, levels, key);
    free(t);
}

/* relinearisation key: target s^2 (product over the integers, |coef| <= N) */
void or_gen_relin_key_rows(void *vc, void *vp, const int8_t *s, int n_data, int levels, u64 *key);
void or_gen_relin_key(void *vc, void *vp, const int8_t *s, int n_data, u64 *key)
{
    or_gen_relin_key_rows(vc, vp, s, n_data, n_data, key);
}
void or_gen_relin_key_rows(void *vc, void *vp, const int8_t *s, int n_data, int levels, u64 *key)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    i64 *t = (i64 *)calloc(n, sizeof(i64));
    for (int a = 0; a < n; a++) {
        if (!s[a]) continue;
        for (int b = 0; b < n; b++) {
            if (!s[b]) continue;
            int k = a + b;
            i64 v = (i64)s[a] * s[b];
            if (k < n) t[k] += v;
            else t[k - n] -= v; /* X^N = -1 */
        }
    }
    gen_switch_key_rows(c, (prng_t *)vp, s, t, n_data, levels, key);
    free(t);
}

/* public-key encryption: (v pk0 + e0 + m, v pk1 + e1) over n_data primes.
 * pt, ct in coefficient form; pt: [n_data][N], ct: [2][n_data][N]. */
void or_encrypt_pk(void *vc, void *vp, const u64 *pk, const u64 *pt, int n_data, u64 *ct)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    prng_t *p = (prng_t *)vp;
    i64 *v = (i64 *)malloc(sizeof(i64) * n), *e0 = (i64 *)malloc(sizeof(i64) * n),
        *e1 = (i64 *)malloc(sizeof(i64) * n);
    u64 *vm = (u64 *)malloc(sizeof(u64) * n), *tmp = (u64 *)malloc(sizeof(u64) * n);
    for (int j = 0; j < n; j++) v[j] = sample_ternary(p);
    for (int j = 0; j < n; j++) e0[j] = sample_gauss(p);
    for (int j = 0; j < n; j++) e1[j] = sample_gauss(p);
    for (int i = 0; i < n_data; i++) {
        u64 q = c->mod[i].q;
        small_to_mod(c, v, i, vm);
        u64 *c0 = ct + (size_t)i * n, *c1 = ct + ((size_t)n_data + i) * n;
        or_poly_mul(c, i, vm, pk + (size_t)i * n, tmp);
        for (int j = 0; j < n; j++)
            c0[j] = add_mod(add_mod(tmp[j], reduce_i128(e0[j], q), q), pt[(size_t)i * n + j], q);
        or_poly_mul(c, i, vm, pk + ((size_t)n_data + i) * n, tmp);
        for (int j = 0; j < n; j++) c1[j] = add_mod(tmp[j], reduce_i128(e1[j], q), q);
    }
    free(v); free(e0); free(e1); free(vm); free(tmp);
}

/* decryption residues m = c0 + c1 s, per limb, coefficient form */
void or_decrypt(void *vc, const int8_t *s, const u64 *ct, int n_limbs, u64 *m)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    i64 *si = (i64 *)malloc(sizeof(i64) * n);
    u64 *sm = (u64 *)malloc(sizeof(u64) * n), *tmp = (u64 *)malloc(sizeof(u64) * n);
    for (int j = 0; j < n; j++) si[j] = s[j];
    for (int i = 0; i < n_limbs; i++) {
        u64 q = c->mod[i].q;
        small_to_mod(c, si, i, sm);
        or_poly_mul(c, i, ct + ((size_t)n_limbs + i) * n, sm, tmp);
        for (int j = 0; j < n; j++) m[(size_t)i * n + j] = add_mod(ct[(size_t)i * n + j], tmp[j], q);
    }
    free(si); free(sm); free(tmp);
}

/* ------------------------------------------------------------------------ */
/* key switching (hybrid, one digit per data prime, one special prime)       */
/* ------------------------------------------------------------------------ */
/* A loaded switching key keeps the evaluations (to_eval) of its limbs, so
 * repeated switching does not re-transform it.  The key is made at level L
 * (n_data = L+1) and used at any level l <= L through digits j <= l and limbs
 * {q_0..q_l, P}. */
typedef struct { int n_data; u64 *ev; } swkey_t;

void *or_key_load(void *vc, const u64 *key, int n_data)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n, nb = n_data + 1;
    swkey_t *k = (swkey_t *)malloc(sizeof(swkey_t));
    k->n_data = n_data;
    size_t cnt = (size_t)n_data * 2 * nb;
    k->ev = (u64 *)malloc(sizeof(u64) * cnt * n);
    for (int d = 0; d < n_data; d++)
        for (int cc = 0; cc < 2; cc++)
            for (int i = 0; i < nb; i++) {
                size_t off = (((size_t)d * 2 + cc) * nb + i) * n;
                to_eval(c, i, key + off, k->ev + off);
            }
    return k;
}
void or_key_free(void *vk) { swkey_t *k = (swkey_t *)vk; free(k->ev); free(k); }

/* target basis index b (0..nl-1 data limbs, nl -> P) to moduli index */
static int basis_mod(const swkey_t *k, int nl, int b) { return b < nl ? b : k->n_data; }

/* U_c = sum_j d_j evk_{j,c} for the centered digits dig[j][coef] (j < nl),
 * over the basis {q_0..q_{nl-1}, P}: acc [2][nl+1][N], coefficient form. */
static void ks_accumulate(ctx_t *c, const swkey_t *k, const i64 *dig, int nl, u64 *acc)
{
    int n = c->n, nbk = k->n_data + 1, nb = nl + 1;
    memset(acc, 0, sizeof(u64) * (size_t)2 * nb * n);
    u64 *ev = (u64 *)malloc(sizeof(u64) * n), *dm = (u64 *)malloc(sizeof(u64) * n);
    for (int b = 0; b < nb; b++) {
        int mi = basis_mod(k, nl, b);
        u64 q = c->mod[mi].q;
        for (int j = 0; j < nl; j++) {
            /* digit j reduced mod the target modulus, then evaluated */
            for (int t = 0; t < n; t++) dm[t] = reduce_i128(dig[(size_t)j * n + t], q);
            to_eval(c, mi, dm, ev);
            for (int cc = 0; cc < 2; cc++) {
                const u64 *kev = k->ev + (((size_t)j * 2 + cc) * nbk + mi) * n;
                u64 *a = acc + ((size_t)cc * nb + b) * n;
                for (int t = 0; t < n; t++) a[t] = add_mod(a[t], mul_mod(ev[t], kev[t], q), q);
            }
        }
        for (int cc = 0; cc < 2; cc++) from_eval(c, mi, acc + ((size_t)cc * nb + b) * n);
    }
    free(ev); free(dm);
}

/* ModDown: out_p[i] = (E_p[i] - centered(E_p[P])) * P^-1 mod q_i, the exact
 * rounding division by P of each of n_polys polynomials over
 * {q_0..q_{nl-1}, P} (in: [n_polys][nl+1][N], out: [n_polys][nl][N]) */
static void moddown(const ctx_t *c, const u64 *in, int nl, int n_polys, u64 *out)
{
    int n = c->n;
    u64 P = c->mod[c->n_mod - 1].q;
    for (int p = 0; p < n_polys; p++) {
        const u64 *up = in + ((size_t)p * (nl + 1) + nl) * n;
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q, pinv = inv_mod(P % q, q);
            const u64 *ui = in + ((size_t)p * (nl + 1) + i) * n;
            u64 *o = out + ((size_t)p * nl + i) * n;
            for (int t = 0; t < n; t++) {
                u64 r = reduce_i128(centered(up[t], P), q);
                o[t] = mul_mod(sub_mod(ui[t], r, q), pinv, q);
            }
        }
    }
}

/* Given the centered digits dig[j][coef] (j < nl), compute
 * out_c[i] = round((sum_j d_j evk_{j,c}) / P) mod q_i, i < nl. */
static void ks_from_digits(ctx_t *c, const swkey_t *k, const i64 *dig, int nl, u64 *out)
{
    u64 *acc = (u64 *)malloc(sizeof(u64) * (size_t)2 * (nl + 1) * c->n);
    ks_accumulate(c, k, dig, nl, acc);
    moddown(c, acc, nl, 2, out);
    free(acc);
}

/* digits of d (coefficient form, nl limbs): centered residues, as integers */
static void centered_digits(const ctx_t *c, const u64 *d, int nl, i64 *dig)
{
    int n = c->n;
    for (int j = 0; j < nl; j++)
        for (int t = 0; t < n; t++) dig[(size_t)j * n + t] = centered(d[(size_t)j * n + t], c->mod[j].q);
}

/* KS(d): out [2][nl][N] with out_0 + out_1 s ~= d t */
int or_keyswitch(void *vc, const u64 *d, int nl, void *vk, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    swkey_t *k = (swkey_t *)vk;
    if (nl > k->n_data) return -1;
    i64 *dig = (i64 *)malloc(sizeof(i64) * (size_t)nl * c->n);
    centered_digits(c, d, nl, dig);
    ks_from_digits(c, k, dig, nl, out);
    free(dig);
    return 0;
}

/* Rot(ct, r) = (tau_g(c0) + KS_0(tau_g(c1)), KS_1(tau_g(c1))), g = 5^r */
int or_rotate(void *vc, const u64 *ct, int nl, i64 r, void *vk, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    size_t lsz = (size_t)nl * n;
    u64 g = or_galois_elt(vc, r);
    u64 *t0 = (u64 *)malloc(sizeof(u64) * lsz), *t1 = (u64 *)malloc(sizeof(u64) * lsz);
    u64 *ks = (u64 *)malloc(sizeof(u64) * 2 * lsz);
    or_automorphism(vc, ct, nl, g, t0);
    or_automorphism(vc, ct + lsz, nl, g, t1);
    int rc = or_keyswitch(vc, t1, nl, vk, ks);
    if (rc == 0) {
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q;
            for (int t = 0; t < n; t++) {
                size_t o = (size_t)i * n + t;
                out[o] = add_mod(t0[o], ks[o], q);
                out[lsz + o] = ks[lsz + o];
            }
        }
    }
    free(t0); free(t1); free(ks);
    return rc;
}

/* Hoisted rotations: the digits of c1 are lifted once; for each rotation the
 * automorphism is applied to the lifted integer digits (a signed coefficient
 * permutation, which commutes with the centered lift). outs: [nr][2][nl][N] */
int or_rotate_hoisted(void *vc, const u64 *ct, int nl, const i64 *rs, int nr, void **keys, u64 *outs)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    size_t lsz = (size_t)nl * n;
    u64 two_n = 2 * (u64)n;
    i64 *dig = (i64 *)malloc(sizeof(i64) * lsz), *rdig = (i64 *)malloc(sizeof(i64) * lsz);
    u64 *t0 = (u64 *)malloc(sizeof(u64) * lsz);
    centered_digits(c, ct + lsz, nl, dig);
    int rc = 0;
    for (int w = 0; w < nr && rc == 0; w++) {
        swkey_t *k = (swkey_t *)keys[w];
        if (nl > k->n_data) { rc = -1; break; }
        u64 g = or_galois_elt(vc, rs[w]);
        for (int j = 0; j < nl; j++)
            for (int t = 0; t < n; t++) {
                u64 e = ((u64)t * g) % two_n;
                i64 v = dig[(size_t)j * n + t];
                if (e < (u64)n) rdig[(size_t)j * n + e] = v;
                else rdig[(size_t)j * n + e - n] = -v;
            }
        u64 *out = outs + (size_t)w * 2 * lsz;
        ks_from_digits(c, k, rdig, nl, out);
        or_automorphism(vc, ct, nl, g, t0);
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q;
            for (int t = 0; t < n; t++) {
                size_t o = (size_t)i * n + t;
                out[o] = add_mod(out[o], t0[o], q);
            }
        }
    }
    free(dig); free(rdig); free(t0);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* deferred ModDown: ciphertexts over the extended basis {q_0..q_{nl-1}, P}  */
/* ------------------------------------------------------------------------ */
/* An extended ciphertext E = (E_0, E_1) over Q_l P stands for the ciphertext
 * ModDown(E) over Q_l (the exact rounding division by P above).  A rotation
 * kept in this form skips the ModDown of its key switch:
 *     E = (P tau_g(c0) + U_0, U_1),   U = sum_j d_j evk_j  (d: digits of tau_g(c1)),
 * and ModDown(E) is exactly Rot(ct, r): P tau_g(c0) has residue 0 mod P and
 * divides exactly.  A ciphertext enters the form as P ct (residue 0 mod P).
 * Sums and plaintext products (with the plaintext's residue mod P as the
 * last limb) act limb by limb, so one ModDown of a sum of such terms
 * replaces one per rotation; it rounds once, where the sum of rotated
 * ciphertexts rounds once per term, so the two differ in the last bits. */

/* out [2][nl+1][N]: (P tau_g(c0) + U_0, U_1) for the left rotation by r */
int or_rotate_ext(void *vc, const u64 *ct, int nl, i64 r, void *vk, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    swkey_t *k = (swkey_t *)vk;
    int n = c->n;
    if (nl > k->n_data) return -1;
    size_t lsz = (size_t)nl * n;
    u64 g = or_galois_elt(vc, r);
    u64 P = c->mod[c->n_mod - 1].q;
    u64 *t0 = (u64 *)malloc(sizeof(u64) * lsz), *t1 = (u64 *)malloc(sizeof(u64) * lsz);
    i64 *dig = (i64 *)malloc(sizeof(i64) * lsz);
    or_automorphism(vc, ct, nl, g, t0);
    or_automorphism(vc, ct + lsz, nl, g, t1);
    centered_digits(c, t1, nl, dig);
    ks_accumulate(c, k, dig, nl, out);
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i].q, pm = P % q;
        for (int t = 0; t < n; t++) {
            size_t o = (size_t)i * n + t;
            out[o] = add_mod(out[o], mul_mod(pm, t0[o], q), q);
        }
    }
    free(t0); free(t1); free(dig);
    return 0;
}

/* out [n_polys][nl+1][N] = P in [n_polys][nl][N]: limbs i < nl scaled by
 * P mod q_i, limb nl zero */
void or_to_ext(void *vc, const u64 *in, int nl, int n_polys, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    u64 P = c->mod[c->n_mod - 1].q;
    for (int p = 0; p < n_polys; p++) {
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q, pm = P % q;
            const u64 *x = in + ((size_t)p * nl + i) * n;
            u64 *y = out + ((size_t)p * (nl + 1) + i) * n;
            for (int t = 0; t < n; t++) y[t] = mul_mod(pm, x[t], q);
        }
        memset(out + ((size_t)p * (nl + 1) + nl) * n, 0, sizeof(u64) * n);
    }
}

/* ModDown of n_polys extended polynomials: [n_polys][nl+1][N] -> [n_polys][nl][N] */
void or_moddown(void *vc, const u64 *in, int nl, int n_polys, u64 *out)
{
    moddown((const ctx_t *)vc, in, nl, n_polys, out);
}

/* out = a + b over extended operands (n_polys polynomials of nl+1 limbs) */
void or_add_ext(void *vc, const u64 *a, const u64 *b, int nl, int n_polys, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    for (int p = 0; p < n_polys; p++)
        for (int i = 0; i <= nl; i++) {
            u64 q = c->mod[i < nl ? i : c->n_mod - 1].q;
            size_t off = ((size_t)p * (nl + 1) + i) * n;
            for (int j = 0; j < n; j++) out[off + j] = add_mod(a[off + j], b[off + j], q);
        }
}

/* ------------------------------------------------------------------------ */
/* plaintext multiply-accumulate, add, square + relinearise, rescale        */
/* ------------------------------------------------------------------------ */
/* acc[o] = sum_t pts[o*n_ct + t] * cts[t], for o < n_out.  Each ciphertext is
 * evaluated once and shared by every output (Algorithm 1 reuses each rotated
 * ciphertext for all output channels).  A NULL plaintext is a zero term.
 * Limb i of every operand is taken modulo c->mod[mods[i]].
 * cts[t]: [2][nb][N]; pts: [nb][N]; acc[o]: [2][nb][N]. */
static void mac_matrix(ctx_t *c, const int *mods, int nb, int n_ct, const u64 **cts, int n_out, const u64 **pts,
                       u64 **acc)
{
    int n = c->n;
    size_t lsz = (size_t)nb * n;
    u64 *ev = (u64 *)malloc(sizeof(u64) * (size_t)n_ct * 2 * lsz);
    for (int t = 0; t < n_ct; t++)
        for (int cc = 0; cc < 2; cc++)
            for (int i = 0; i < nb; i++)
                to_eval(c, mods[i], cts[t] + (size_t)cc * lsz + (size_t)i * n,
                        ev + ((size_t)t * 2 + cc) * lsz + (size_t)i * n);
    u64 *pev = (u64 *)malloc(sizeof(u64) * n);
    u64 *a = (u64 *)malloc(sizeof(u64) * 2 * lsz);
    for (int o = 0; o < n_out; o++) {
        memset(a, 0, sizeof(u64) * 2 * lsz);
        for (int t = 0; t < n_ct; t++) {
            const u64 *pt = pts[(size_t)o * n_ct + t];
            if (!pt) continue;
            for (int i = 0; i < nb; i++) {
                u64 q = c->mod[mods[i]].q;
                to_eval(c, mods[i], pt + (size_t)i * n, pev);
                for (int cc = 0; cc < 2; cc++) {
                    const u64 *x = ev + ((size_t)t * 2 + cc) * lsz + (size_t)i * n;
                    u64 *y = a + (size_t)cc * lsz + (size_t)i * n;
                    for (int j = 0; j < n; j++) y[j] = add_mod(y[j], mul_mod(pev[j], x[j], q), q);
                }
            }
        }
        for (int cc = 0; cc < 2; cc++)
            for (int i = 0; i < nb; i++) from_eval(c, mods[i], a + (size_t)cc * lsz + (size_t)i * n);
        memcpy(acc[o], a, sizeof(u64) * 2 * lsz);
    }
    free(ev); free(pev); free(a);
}

/* moduli of the limbs of an extended operand: q_0..q_{nl-1}, then P */
static int *limb_mods(const ctx_t *c, int nl)
{
    int *m = (int *)malloc(sizeof(int) * (nl + 1));
    for (int i = 0; i < nl; i++) m[i] = i;
    m[nl] = c->n_mod - 1;
    return m;
}

void or_mac_matrix(void *vc, int nl, int n_ct, const u64 **cts, int n_out, const u64 **pts, u64 **acc)
{
    ctx_t *c = (ctx_t *)vc;
    int *m = limb_mods(c, nl);
    mac_matrix(c, m, nl, n_ct, cts, n_out, pts, acc);
    free(m);
}

/* the same over extended operands (nl data limbs and P): cts[t], acc[o]
 * [2][nl+1][N], pts [nl+1][N] */
void or_mac_matrix_ext(void *vc, int nl, int n_ct, const u64 **cts, int n_out, const u64 **pts, u64 **acc)
{
    ctx_t *c = (ctx_t *)vc;
    int *m = limb_mods(c, nl);
    mac_matrix(c, m, nl + 1, n_ct, cts, n_out, pts, acc);
    free(m);
}

/* out = a + b (n_polys polynomials of nl limbs each) */
void or_add(void *vc, const u64 *a, const u64 *b, int nl, int n_polys, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    for (int p = 0; p < n_polys; p++)
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q;
            size_t off = ((size_t)p * nl + i) * n;
            for (int j = 0; j < n; j++) out[off + j] = add_mod(a[off + j], b[off + j], q);
        }
}

/* (c0, c1)^2 -> (c0^2, 2 c0 c1, c1^2), then relinearise c1^2 with the key */
int or_square_relin(void *vc, const u64 *ct, int nl, void *vk, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    size_t lsz = (size_t)nl * n;
    u64 *d0 = (u64 *)malloc(sizeof(u64) * lsz), *d1 = (u64 *)malloc(sizeof(u64) * lsz),
        *d2 = (u64 *)malloc(sizeof(u64) * lsz), *ks = (u64 *)malloc(sizeof(u64) * 2 * lsz);
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i].q;
        const u64 *c0 = ct + (size_t)i * n, *c1 = ct + lsz + (size_t)i * n;
        or_poly_mul(vc, i, c0, c0, d0 + (size_t)i * n);
        or_poly_mul(vc, i, c0, c1, d1 + (size_t)i * n);
        or_poly_mul(vc, i, c1, c1, d2 + (size_t)i * n);
        for (int j = 0; j < n; j++) d1[(size_t)i * n + j] = add_mod(d1[(size_t)i * n + j], d1[(size_t)i * n + j], q);
    }
    int rc = or_keyswitch(vc, d2, nl, vk, ks);
    if (rc == 0) {
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q;
            for (int j = 0; j < n; j++) {
                size_t o = (size_t)i * n + j;
                out[o] = add_mod(d0[o], ks[o], q);
                out[lsz + o] = add_mod(d1[o], ks[lsz + o], q);
            }
        }
    }
    free(d0); free(d1); free(d2); free(ks);
    return rc;
}

/* Mul(C) of Section II-B with relinearisation: the tensor product
 * (a0 b0, a0 b1 + a1 b0, a1 b1) of two ciphertexts at nl limbs, then the
 * key switch of the last part with the key of s^2 added in.  out: [2][nl][N]. */
int or_mul_relin(void *vc, const u64 *a, const u64 *b, int nl, void *vk, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n;
    size_t lsz = (size_t)nl * n;
    u64 *d0 = (u64 *)malloc(sizeof(u64) * lsz), *d1 = (u64 *)malloc(sizeof(u64) * lsz),
        *d2 = (u64 *)malloc(sizeof(u64) * lsz), *t = (u64 *)malloc(sizeof(u64) * n),
        *ks = (u64 *)malloc(sizeof(u64) * 2 * lsz);
    for (int i = 0; i < nl; i++) {
        u64 q = c->mod[i].q;
        const u64 *a0 = a + (size_t)i * n, *a1 = a + lsz + (size_t)i * n;
        const u64 *b0 = b + (size_t)i * n, *b1 = b + lsz + (size_t)i * n;
        or_poly_mul(vc, i, a0, b0, d0 + (size_t)i * n);
        or_poly_mul(vc, i, a0, b1, d1 + (size_t)i * n);
        or_poly_mul(vc, i, a1, b0, t);
        for (int j = 0; j < n; j++) d1[(size_t)i * n + j] = add_mod(d1[(size_t)i * n + j], t[j], q);
        or_poly_mul(vc, i, a1, b1, d2 + (size_t)i * n);
    }
    int rc = or_keyswitch(vc, d2, nl, vk, ks);
    if (rc == 0) {
        for (int i = 0; i < nl; i++) {
            u64 q = c->mod[i].q;
            for (int j = 0; j < n; j++) {
                size_t o = (size_t)i * n + j;
                out[o] = add_mod(d0[o], ks[o], q);
                out[lsz + o] = add_mod(d1[o], ks[lsz + o], q);
            }
        }
    }
    free(d0); free(d1); free(d2); free(t); free(ks);
    return rc;
}

/* Rescale by the last prime q_l (l = nl-1): exact rounding division,
 * c'[i] = (c[i] - centered([c]_{q_l})) q_l^-1 mod q_i.  n_polys polynomials;
 * in: [n_polys][nl][N], out: [n_polys][nl-1][N]. */
void or_rescale(void *vc, const u64 *in, int nl, int n_polys, u64 *out)
{
    ctx_t *c = (ctx_t *)vc;
    int n = c->n, l = nl - 1;
    u64 ql = c->mod[l].q;
    for (int p = 0; p < n_polys; p++) {
        const u64 *last = in + ((size_t)p * nl + l) * n;
        for (int i = 0; i < l; i++) {
            u64 q = c->mod[i].q, inv = inv_mod(ql % q, q);
            const u64 *x = in + ((size_t)p * nl + i) * n;
            u64 *y = out + ((size_t)p * l + i) * n;
            for (int j = 0; j < n; j++) {
                u64 r = reduce_i128(centered(last[j], ql), q);
                y[j] = mul_mod(sub_mod(x[j], r, q), inv, q);
            }
        }
    }
}
