/*
 * tjgen.c - seeded synthetic inputs for the equi-join / sort workloads.
 *
 * This file generates input columns only. It contains none of the join or
 * sort arithmetic: both the CPU oracle and the GPU path consume the arrays it
 * writes. Every generator is counter based (value i depends only on the seed
 * and i), so the OpenMP thread count never changes the output.
 *
 * Primitives (all published, written here from their definitions):
 *   - SplitMix64 (Steele, Lea, Flood 2014): a Weyl sequence seed + (i+1)*gamma
 *     passed through the 64-bit finalizer with shifts 30/27/31.
 *   - bij40: a bijection on [0, 2^40) composed of odd multiplications modulo
 *     2^40 and xor-shifts (each step invertible), used to spread key indices
 *     uniformly over the 40-bit key domain without collisions.
 *   - cycle-walking permutation of [0, n): a bijection on [0, 2^k) applied
 *     repeatedly until the value falls below n (Black & Rogaway 2002).
 *   - Zipf(theta, D) by rejection-inversion (Hoermann & Derflinger 1996).
 */
#include <stdint.h>
#include <math.h>
#include <stddef.h>
#include <stdlib.h>

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* i-th output of the SplitMix64 stream started at `seed` (i = 0, 1, ...). */
uint64_t tjgen_splitmix64(uint64_t seed, uint64_t i)
{
    return sm64_mix(seed + (i + 1) * GOLDEN_GAMMA);
}

/* Derive an independent stream seed from a base seed and a tag. */
uint64_t tjgen_stream(uint64_t base_seed, uint64_t tag)
{
    return tjgen_splitmix64(base_seed ^ 0xD1B54A32D192ED03ull, tag);
}

/* ---------------------------------------------------------------------------
 * Bijection on [0, 2^k), 2 <= k <= 64, parameterised by a seed.
 * ------------------------------------------------------------------------- */
typedef struct {
    uint64_t mask, a, b, x;
    unsigned s1, s2;
} bij_t;

static bij_t bij_make(unsigned k, uint64_t seed)
{
    bij_t f;
    f.mask = (k >= 64) ? ~0ull : ((1ull << k) - 1ull);
    f.a = (tjgen_splitmix64(seed, 0) | 1ull) & f.mask;
    f.b = (tjgen_splitmix64(seed, 1) | 1ull) & f.mask;
    f.x = tjgen_splitmix64(seed, 2) & f.mask;
    if (f.a == 0) f.a = 1;
    if (f.b == 0) f.b = 1;
    f.s1 = k / 2 ? k / 2 : 1;
    f.s2 = (k * 3) / 7 ? (k * 3) / 7 : 1;
    return f;
}

static inline uint64_t bij_apply(const bij_t *f, uint64_t v)
{
    v = (v * f->a) & f->mask;
    v ^= v >> f->s1;
    v = (v * f->b) & f->mask;
    v ^= v >> f->s2;
    v ^= f->x;
    return v & f->mask;
}

/* Exposed for the bijection tests: y = f_k,seed(x). */
uint64_t tjgen_bij(unsigned k, uint64_t seed, uint64_t x)
{
    bij_t f = bij_make(k, seed);
    return bij_apply(&f, x & f.mask);
}

static unsigned ceil_log2(uint64_t n)
{
    unsigned k = 0;
    while (k < 64 && (1ull << k) < n) k++;
    return k < 2 ? 2 : k;
}

/* Permutation of [0, n) by cycle walking a bijection on [0, 2^ceil(log2 n)). */
typedef struct { bij_t f; uint64_t n; } perm_t;

static perm_t perm_make(uint64_t n, uint64_t seed)
{
    perm_t p;
    p.f = bij_make(ceil_log2(n), seed);
    p.n = n;
    return p;
}

static inline uint64_t perm_apply(const perm_t *p, uint64_t i)
{
    uint64_t v = bij_apply(&p->f, i);
    while (v >= p->n) v = bij_apply(&p->f, v);
    return v;
}

uint64_t tjgen_perm_at(uint64_t n, uint64_t seed, uint64_t i)
{
    perm_t p = perm_make(n, seed);
    return perm_apply(&p, i);
}

/* ---------------------------------------------------------------------------
 * Zipf(theta) over ranks 1..D by rejection-inversion.
 *
 * h(x) = x^-theta is the unnormalised mass; Hint(x) = (x^(1-theta) - 1)/(1-theta)
 * (log x when theta = 1) is its antiderivative. A uniform u in
 * [Hint(D + 1/2), Hint(3/2) - 1] is inverted through Hint; the rounded value k
 * is accepted when it lies close enough to the inverse (the squeeze k - x <= s)
 * or when u lies above Hint(k + 1/2) - h(k). Each candidate consumes one
 * uniform drawn from the sample's own counter stream.
 * ------------------------------------------------------------------------- */
typedef struct {
    double theta, hx1, hn, s;
    uint64_t d;
} zipf_t;

/* (exp(y) - 1) / y, continuous at 0 */
static double expm1_over(double y)
{
    return fabs(y) > 1e-8 ? expm1(y) / y : 1.0 + y * 0.5 * (1.0 + y / 3.0);
}

/* log1p(y) / y, continuous at 0 */
static double log1p_over(double y)
{
    return fabs(y) > 1e-8 ? log1p(y) / y : 1.0 - y * (0.5 - y / 3.0);
}

static double zipf_hint(const zipf_t *z, double x)
{
    double lx = log(x);
    return expm1_over((1.0 - z->theta) * lx) * lx;
}

static double zipf_h(const zipf_t *z, double x)
{
    return exp(-z->theta * log(x));
}

static double zipf_hint_inv(const zipf_t *z, double y)
{
    double t = y * (1.0 - z->theta);
    if (t < -1.0) t = -1.0;
    return exp(log1p_over(t) * y);
}

static zipf_t zipf_make(double theta, uint64_t d)
{
    zipf_t z;
    z.theta = theta;
    z.d = d;
    z.hx1 = zipf_hint(&z, 1.5) - 1.0;
    z.hn = zipf_hint(&z, (double)d + 0.5);
    z.s = 2.0 - zipf_hint_inv(&z, zipf_hint(&z, 2.5) - zipf_h(&z, 2.0));
    return z;
}

static inline double u01(uint64_t r)
{
    return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

/* rank in [0, D): 0 is the most frequent. `stream` is the sample's own seed. */
static uint64_t zipf_sample(const zipf_t *z, uint64_t stream)
{
    for (uint64_t j = 0;; j++) {
        double u = z->hn + u01(tjgen_splitmix64(stream, j)) * (z->hx1 - z->hn);
        double x = zipf_hint_inv(z, u);
        double kf = floor(x + 0.5);
        if (kf < 1.0) kf = 1.0;
        if (kf > (double)z->d) kf = (double)z->d;
        uint64_t k = (uint64_t)kf;
        if (kf - x <= z->s || u >= zipf_hint(z, kf + 0.5) - zipf_h(z, kf))
            return k - 1;
    }
}

/* Uniform integer in [0, d) from a 64-bit random value (multiply-shift). */
static inline uint64_t below(uint64_t r, uint64_t d)
{
    return (uint64_t)(((unsigned __int128)r * d) >> 64);
}

/* Exposed for the sampler tests. theta == 0 gives the uniform distribution. */
void tjgen_zipf_ranks(uint64_t *out, uint64_t m, double theta, uint64_t d, uint64_t seed)
{
    zipf_t z = zipf_make(theta, d);
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)m; i++) {
        uint64_t st = tjgen_splitmix64(seed, (uint64_t)i);
        out[i] = theta == 0.0 ? below(st, d) : zipf_sample(&z, st);
    }
}

/* ---------------------------------------------------------------------------
 * Column generators.
 * ------------------------------------------------------------------------- */

/* keys_i = low `bits` bits of SplitMix64(seed, i), as int32. */
void tjgen_uniform_i32(int32_t *out, uint64_t n, uint64_t seed, unsigned bits)
{
    uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++)
        out[i] = (int32_t)(uint32_t)(tjgen_splitmix64(seed, (uint64_t)i) & mask);
}

/* keys_i = low `bits` bits of SplitMix64(seed, i), as int64 (bits = 64: full range). */
void tjgen_uniform_i64(int64_t *out, uint64_t n, uint64_t seed, unsigned bits)
{
    uint64_t mask = bits >= 64 ? ~0ull : ((1ull << bits) - 1ull);
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++)
        out[i] = (int64_t)(tjgen_splitmix64(seed, (uint64_t)i) & mask);
}

/* out_i = perm(i): a seeded permutation of [0, n) (used as row ids). */
void tjgen_perm_i32(int32_t *out, uint64_t n, uint64_t seed)
{
    perm_t p = perm_make(n ? n : 1, seed);
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++)
        out[i] = (int32_t)perm_apply(&p, (uint64_t)i);
}

/* out_i = i */
void tjgen_iota_i32(int32_t *out, uint64_t n)
{
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++) out[i] = (int32_t)i;
}

/*
 * Build relation R of n_r rows over the 40-bit key domain.
 *
 * Distinct key d (0 <= d < D) is bij40(d). The first `hot` distinct keys occur
 * `mult` times, the others once, so D = n_r - hot*(mult-1). Rows are shuffled:
 * row i takes slot perm(i); slot s < hot*mult holds distinct key s / mult,
 * a later slot s holds distinct key s - hot*(mult-1).
 */
void tjgen_r_keys40(int64_t *out, uint64_t n_r, uint64_t hot, uint64_t mult,
                    uint64_t key_seed, uint64_t perm_seed)
{
    bij_t f = bij_make(40, key_seed);
    perm_t p = perm_make(n_r ? n_r : 1, perm_seed);
    uint64_t hot_slots = hot * mult;
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n_r; i++) {
        uint64_t s = perm_apply(&p, (uint64_t)i);
        uint64_t d = s < hot_slots ? s / mult : s - hot * (mult - 1);
        out[i] = (int64_t)bij_apply(&f, d);
    }
}

/*
 * Build relation S of n_s rows, foreign-key style against R from
 * tjgen_r_keys40 (same key_seed, same hot/mult, D distinct R keys).
 *
 * Slot s = perm(i) decides row i: the first m = n_matched slots draw a
 * distinct-key rank z ~ Zipf(theta, D) (theta = 0: uniform) and take key
 * bij40(z); the remaining slots take fresh keys bij40(D + (s - m)), which no R
 * row holds. Returns sum over matched rows of the R multiplicity of their key,
 * i.e. the exact equi-join size |R join S| implied by the construction.
 */
uint64_t tjgen_s_keys40(int64_t *out, uint64_t n_s, uint64_t n_matched, uint64_t d_keys,
                        uint64_t hot, uint64_t mult, double theta,
                        uint64_t key_seed, uint64_t perm_seed, uint64_t zipf_seed)
{
    bij_t f = bij_make(40, key_seed);
    perm_t p = perm_make(n_s ? n_s : 1, perm_seed);
    zipf_t z = zipf_make(theta == 0.0 ? 0.5 : theta, d_keys ? d_keys : 1);
    uint64_t total = 0;
    long long i;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (i = 0; i < (long long)n_s; i++) {
        uint64_t s = perm_apply(&p, (uint64_t)i);
        uint64_t d;
        if (s < n_matched) {
            uint64_t st = tjgen_splitmix64(zipf_seed, s);
            uint64_t r = theta == 0.0 ? below(st, d_keys) : zipf_sample(&z, st);
            d = r;
            total += r < hot ? mult : 1;
        } else {
            d = d_keys + (s - n_matched);
        }
        out[i] = (int64_t)bij_apply(&f, d);
    }
    return total;
}

/* ---------------------------------------------------------------------------
 * Learned-partitioner workloads: int64 keys with non-uniform distributions.
 * Every value i draws from its own SplitMix64 counters (seed, 2i), (seed, 2i+1).
 * ------------------------------------------------------------------------- */

/* uniform in (0, 1]: never 0, so its logarithm is finite */
static inline double u01_open(uint64_t r)
{
    return ((double)(r >> 11) + 1.0) * (1.0 / 9007199254740992.0);
}

static inline int64_t clamp_key(double v)
{
    if (!(v >= 0.0)) return 0;
    if (v >= 9223372036854775807.0) return INT64_MAX;
    return (int64_t)v;
}

/* keys_i = floor(exp(mu + sigma * z_i)), z_i standard normal (Box-Muller with
 * two uniforms of the row's own counters), clamped to [0, INT64_MAX]. */
void tjgen_lognormal_i64(int64_t *out, uint64_t n, uint64_t seed, double mu, double sigma)
{
    const double two_pi = 6.283185307179586476925286766559;
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++) {
        double u1 = u01_open(tjgen_splitmix64(seed, 2 * (uint64_t)i));
        double u2 = u01(tjgen_splitmix64(seed, 2 * (uint64_t)i + 1));
        double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
        out[i] = clamp_key(floor(exp(mu + sigma * z)));
    }
}

/* Mixture of `ncomp` (<= 64) uniform intervals. Component c starts at a
 * uniform point of [0, 2^62), has width 2^(wlo + (whi - wlo) u) and weight
 * proportional to -log(u) (Dirichlet(1, ..., 1) weights); all drawn from
 * `seed` before any row. Row i picks a component by the weights and a uniform
 * offset inside it. lo/width/weight of the components are written to comp[3*ncomp]
 * (as doubles) when comp is not NULL. */
void tjgen_mixture_i64(int64_t *out, uint64_t n, uint64_t seed, unsigned ncomp, double wlo, double whi,
                       double *comp)
{
    uint64_t lo[64];
    double width[64], cum[64], tot = 0.0;
    unsigned c;
    if (ncomp == 0 || ncomp > 64) return;
    for (c = 0; c < ncomp; c++) {
        uint64_t r0 = tjgen_splitmix64(seed, 3 * (uint64_t)c);
        lo[c] = r0 >> 2;
        width[c] = exp2(wlo + (whi - wlo) * u01(tjgen_splitmix64(seed, 3 * (uint64_t)c + 1)));
        double w = -log(u01_open(tjgen_splitmix64(seed, 3 * (uint64_t)c + 2)));
        tot += w;
        cum[c] = tot;
        if (comp) {
            comp[3 * c] = (double)lo[c];
            comp[3 * c + 1] = width[c];
            comp[3 * c + 2] = w;
        }
    }
    const uint64_t rs = tjgen_splitmix64(seed, 1000003);
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++) {
        double u = u01(tjgen_splitmix64(rs, 2 * (uint64_t)i)) * tot;
        unsigned k = 0;
        while (k + 1 < ncomp && u >= cum[k]) k++;
        uint64_t off = (uint64_t)(u01(tjgen_splitmix64(rs, 2 * (uint64_t)i + 1)) * width[k]);
        uint64_t v = lo[k] + off;
        out[i] = v > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)v;
    }
}

/* Sequential keys with random gaps, shuffled: the j-th smallest key is
 * k_j = j + sum_{t <= j} g_t with g_t ~ Geometric(p) on {0, 1, ...} (so
 * consecutive keys differ by 1 + g); row i holds k_{perm(i)}. The gaps come
 * from a counter-based stream, the prefix sum runs in blocks. */
void tjgen_seqgap_i64(int64_t *out, uint64_t n, uint64_t seed, double p)
{
    if (n == 0) return;
    int64_t *seq = out;  /* the ordered keys are built in place, then shuffled below */
    const double lq = log1p(-p);
    const uint64_t gs = tjgen_splitmix64(seed, 7);
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++) {
        double u = u01_open(tjgen_splitmix64(gs, (uint64_t)i));
        seq[i] = 1 + (int64_t)floor(log(u) / lq);  /* 1 + Geometric(p) */
    }
    /* inclusive prefix sum, two-level */
    const uint64_t B = 1u << 16;
    const uint64_t nb = (n + B - 1) / B;
    int64_t *bsum = (int64_t *)malloc(nb * sizeof(int64_t));
    long long b;
#pragma omp parallel for schedule(static)
    for (b = 0; b < (long long)nb; b++) {
        uint64_t e = ((uint64_t)b + 1) * B < n ? ((uint64_t)b + 1) * B : n;
        int64_t s = 0;
        for (uint64_t j = (uint64_t)b * B; j < e; j++) { s += seq[j]; seq[j] = s; }
        bsum[b] = s;
    }
    int64_t run = 0;
    for (uint64_t j = 0; j < nb; j++) { int64_t t = bsum[j]; bsum[j] = run; run += t; }
#pragma omp parallel for schedule(static)
    for (b = 0; b < (long long)nb; b++) {
        uint64_t e = ((uint64_t)b + 1) * B < n ? ((uint64_t)b + 1) * B : n;
        for (uint64_t j = (uint64_t)b * B; j < e; j++) seq[j] += bsum[b];
    }
    free(bsum);
    /* shuffle: cycle-walk permutation, applied out of place through a copy */
    int64_t *tmp = (int64_t *)malloc(n * sizeof(int64_t));
    perm_t pm = perm_make(n, tjgen_splitmix64(seed, 11));
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++) tmp[i] = seq[perm_apply(&pm, (uint64_t)i)];
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n; i++) out[i] = tmp[i];
    free(tmp);
}

/* S of a foreign-key pair: the first n_matched rows copy the key of a uniform
 * random R row, the rest come from fresh[] (draws of R's distribution with
 * another seed); then rows are shuffled by a seeded permutation. */
void tjgen_fk_from(int64_t *out, uint64_t n_s, uint64_t n_matched, const int64_t *r, uint64_t n_r,
                   const int64_t *fresh, uint64_t seed)
{
    if (n_s == 0) return;
    int64_t *tmp = (int64_t *)malloc(n_s * sizeof(int64_t));
    long long i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n_s; i++)
        tmp[i] = (uint64_t)i < n_matched ? r[below(tjgen_splitmix64(seed, (uint64_t)i), n_r)]
                                         : fresh[(uint64_t)i - n_matched];
    perm_t pm = perm_make(n_s, tjgen_splitmix64(seed, ~0ull));
#pragma omp parallel for schedule(static)
    for (i = 0; i < (long long)n_s; i++) out[i] = tmp[perm_apply(&pm, (uint64_t)i)];
    free(tmp);
}
