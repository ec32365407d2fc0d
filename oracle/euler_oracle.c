/*
 * euler_oracle.c -- reference (oracle) implementation of the Euler-approximation
 * schemes for Markovian queueing networks (Hong, Song & Wang, "Fast Discrete-Event
 * Simulation of Markovian Queueing Networks through Euler Approximation").
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * The product path never links, loads or calls it, and it shares no code with the
 * HIP library: the two sides implement the same written contract (random-number
 * layout, sampler algorithms and their floating-point operation order) separately.
 *
 * Style: plain, slow, obviously correct loops.  Every floating-point operation that
 * decides an integer (a sampler branch, a rejection test, an inversion comparison)
 * is an IEEE fp32 basic operation (+ - * / sqrt), an explicit fmaf, an int<->float
 * conversion, floorf or rintf.  No transcendental from libm reaches a sampler;
 * log/exp/expm1/log1p below are written from their defining series.  Host-side
 * table precompute (routing conditionals, departure probabilities, rate integrals)
 * is done in fp64 with libm and rounded once to fp32.
 * Compile with:  gcc -O2 -ffp-contract=off -fno-fast-math -fPIC -shared -pthread
 *
 * Where the paper is silent (random-number layout, sampler algorithms and thresholds,
 * statistics definitions), the reading taken is stated in the comment of the function that
 * implements it.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOTDAG -2
#define ORC_ENOMEM -3
#define ORC_EOVERFLOW -5

#define SCHEME_BACKWARD 0
#define SCHEME_FORWARD 1
#define DEP_EXACT 0
#define DEP_NAIVE 1

#define SUB_ARRIVAL 0u
#define SUB_DEPART 1u
#define SUB_ROUTE 2u
#define SUB_SOJOURN 3u

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC 2011): 10 rounds of two 32x32->64 multiplies with the   */
/* published multipliers and Weyl key increments.                              */
/* ------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------- */
/* Event counters (instrumentation only: they change no result).  Every thread */
/* counts the algorithm's events in its own array; a run adds the arrays of its */
/* worker threads into the totals that orc_op_counts reads.                     */
/* ------------------------------------------------------------------------- */
enum {
    EV_STATION_STEP,   /* (replication, station, step) updates */
    EV_PHILOX,         /* Philox4x32-10 blocks generated */
    EV_UNIFORM,        /* uniforms used */
    EV_POIS_INV,       /* Poisson draws by inversion (lam < 10) */
    EV_POIS_INV_STEP,  /*   their search steps */
    EV_PTRS,           /* Poisson draws by PTRS */
    EV_PTRS_TRY,       /*   attempts */
    EV_PTRS_SLOW,      /*   attempts that reach the logarithmic test */
    EV_BIN_INV,        /* binomial draws by inversion (n p < 80) */
    EV_BIN_INV_STEP,   /*   their search steps */
    EV_BTRS,           /* binomial draws by BTRS */
    EV_BTRS_TRY,       /*   attempts */
    EV_BTRS_SLOW,      /*   attempts that reach the logarithmic test */
    EV_BIN_PREP,       /* binomials whose probability is computed in the step (x > m branch) */
    EV_GAMMA,          /* gamma (Erlang) draws */
    EV_GAMMA_POLAR,    /*   polar-method tries (pairs of uniforms) */
    EV_GAMMA_TRY,      /*   attempts with a normal */
    EV_GAMMA_SLOW,     /*   attempts that reach the logarithmic test */
    EV_EXPM1,          /* 1 - e^{-mu (h - T)} of the T <= h branch */
    EV_DEPART,         /* departure draws (x > 0) */
    EV_EDGE,           /* routing edges drawn */
    EV_PUSH,           /* routed counts pushed (nonzero) */
    EV_COUNT
};
static _Thread_local int64_t tl_ev[EV_COUNT];
static int64_t g_ev[EV_COUNT];
static pthread_mutex_t g_ev_lock = PTHREAD_MUTEX_INITIALIZER;
#define EV(e) (tl_ev[e] += 1)

static void ev_flush(void)
{
    pthread_mutex_lock(&g_ev_lock);
    for (int e = 0; e < EV_COUNT; ++e) g_ev[e] += tl_ev[e];
    pthread_mutex_unlock(&g_ev_lock);
    memset(tl_ev, 0, sizeof tl_ev);
}

/* Event totals of the runs since the last reset (out[EV_COUNT]); reset clears them. */
int orc_op_counts(int64_t *out, int reset)
{
    pthread_mutex_lock(&g_ev_lock);
    if (out) memcpy(out, g_ev, sizeof g_ev);
    if (reset) memset(g_ev, 0, sizeof g_ev);
    pthread_mutex_unlock(&g_ev_lock);
    return EV_COUNT;
}

/* One uniform stream per (replication, station, step, substream).  The Philox   */
/* key is (low 32 bits of seed, high 32 bits of seed XOR network id); the        */
/* counter is (rep, station, step-1, substream<<24 | block).  Words are consumed */
/* in order x0..x3, then the block index advances.                               */
#define BLOCK_LIMIT (1u << 24)

typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t sub, block;
    uint32_t buf[4];
    int idx;
    int *overflow;
} ustream;

static void us_init(ustream *s, uint64_t seed, uint32_t net_id, uint32_t rep,
                    uint32_t station, uint32_t step0, uint32_t sub, int *overflow)
{
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32) ^ net_id;
    s->ctr[0] = rep;
    s->ctr[1] = station;
    s->ctr[2] = step0;
    s->sub = sub;
    s->block = 0;
    s->idx = 4;
    s->overflow = overflow;
}

static uint32_t us_next_u32(ustream *s)
{
    if (s->idx == 4) {
        if (s->block >= BLOCK_LIMIT) {
            if (s->overflow) *s->overflow = 1;
            s->block = 0;
        }
        s->ctr[3] = (s->sub << 24) | s->block;
        orc_philox4x32_10(s->ctr, s->key, s->buf);
        EV(EV_PHILOX);
        s->block += 1;
        s->idx = 0;
    }
    return s->buf[s->idx++];
}

/* u = (2*(x>>9) + 1) * 2^-24: exactly representable, in [2^-24, 1-2^-24]. */
float orc_u01(uint32_t x)
{
    uint32_t j = ((x >> 9) << 1) | 1u;
    return (float)j * 0x1p-24f;
}

static float us_u01(ustream *s) { EV(EV_UNIFORM); return orc_u01(us_next_u32(s)); }

/* ------------------------------------------------------------------------- */
/* fp32 elementary functions from their series (no libm in the samplers).      */
/* ------------------------------------------------------------------------- */
static const float LN2_HI = 0x1.62ep-1f;        /* ln 2 rounded to 12 significant bits */
static const float LN2_LO = 0x1.0bfbe8p-15f;    /* fp32(ln 2 - LN2_HI) */
static const float INV_LN2 = 0x1.715476p+0f;    /* fp32(1/ln 2) */
static const float HALF_LN2 = 0x1.62e43p-2f;    /* fp32(ln 2 / 2) */
static const float HALF_LOG_2PI = 0x1.d67f1cp-1f; /* fp32(0.5 ln(2 pi)) */

static inline float f_from_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static inline uint32_t bits_from_f(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/* R(z) = 2z/3 + 2z^2/5 + ... + 2z^5/11, so that 2 atanh(s) = 2s + s R(s^2). */
static float atanh_tail(float z)
{
    float p = 0x1.745d18p-3f;          /* 2/11 */
    p = fmaf(p, z, 0x1.c71c72p-3f);    /* 2/9 */
    p = fmaf(p, z, 0x1.24924ap-2f);    /* 2/7 */
    p = fmaf(p, z, 0x1.99999ap-2f);    /* 2/5 */
    p = fmaf(p, z, 0x1.555556p-1f);    /* 2/3 */
    return z * p;
}

/* ln(1+f) for |f| small, via s = f/(2+f): ln(1+f) = 2 atanh(s) = 2s + s R and        */
/* 2s = f - s f, with s f = h - s h for h = f^2/2, giving f - (h - s (h + R)).         */
/* `lo` is a small extra term added at the innermost level (e ln2_lo for the log).    */
static float log1p_core(float f, float lo)
{
    float s = f / (2.0f + f);
    float z = s * s;
    float R = atanh_tail(z);
    float hfsq = (0.5f * f) * f;
    return f - (hfsq - fmaf(s, hfsq + R, lo));
}

/* ln(u) + corr for positive normal u, |corr| << ulp(ln u): u = 2^e (1+f) with 1+f in */
/* (sqrt(2)/2, sqrt(2)], ln u = e ln2 + ln(1+f), ln 2 split in a 12-bit head and a     */
/* tail (Cody-Waite), corr added with the tail.                                          */
static float log_corr(float u, float corr)
{
    uint32_t b = bits_from_f(u);
    int e = (int)(b >> 23) - 127;
    uint32_t mb = (b & 0x007FFFFFu) | 0x3F800000u;
    if (mb > 0x3FB504F3u) {            /* mantissa > sqrt(2): use half of it, e+1 */
        mb -= 0x00800000u;
        e += 1;
    }
    float f = f_from_bits(mb) - 1.0f;  /* exact */
    float ef = (float)e;
    return fmaf(ef, LN2_HI, log1p_core(f, fmaf(ef, LN2_LO, corr)));
}

float orc_logf(float x) { return log_corr(x, 0.0f); }

/* log(1+x) for x > -1.  For |x| >= 1/4, u = fl(1+x) loses the rounding error           */
/* c = (1+x) - u, recovered exactly (Sterbenz) and added back as c/u.                    */
float orc_log1pf(float x)
{
    if (fabsf(x) < 0.25f) return log1p_core(x, 0.0f);
    float u = 1.0f + x;
    float c = (x < 1.0f) ? x - (u - 1.0f) : 1.0f - (u - x);
    return log_corr(u, c / u);
}

/* exp(r) for |r| <= ln2/2: Taylor polynomial through r^7/7!. */
static float exp_poly(float r)
{
    float p = 0x1.a01a02p-13f;         /* 1/7! */
    p = fmaf(p, r, 0x1.6c16c2p-10f);   /* 1/6! */
    p = fmaf(p, r, 0x1.111112p-7f);    /* 1/5! */
    p = fmaf(p, r, 0x1.555556p-5f);    /* 1/4! */
    p = fmaf(p, r, 0x1.555556p-3f);    /* 1/3! */
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return p;
}

/* exp(x): x = k ln2 + r, exp(x) = 2^k exp(r).  Results below ~e^-86 are */
/* returned as 0 (never needed: only probabilities far from underflow).   */
float orc_expf(float x)
{
    if (x < -86.0f) return 0.0f;
    if (x > 88.0f) return INFINITY;
    float k = rintf(x * INV_LN2);
    float r = fmaf(-k, LN2_HI, x);
    r = fmaf(-k, LN2_LO, r);
    float p = exp_poly(r);
    int ki = (int)k;
    return p * f_from_bits((uint32_t)(ki + 127) << 23);
}

/* exp(r)-1 for |r| <= ln2/2: r + r^2 (1/2 + r/3! + ... + r^6/8!). */
static float expm1_poly(float r)
{
    float p = 0x1.a01a02p-16f;         /* 1/8! */
    p = fmaf(p, r, 0x1.a01a02p-13f);   /* 1/7! */
    p = fmaf(p, r, 0x1.6c16c2p-10f);   /* 1/6! */
    p = fmaf(p, r, 0x1.111112p-7f);    /* 1/5! */
    p = fmaf(p, r, 0x1.555556p-5f);    /* 1/4! */
    p = fmaf(p, r, 0x1.555556p-3f);    /* 1/3! */
    p = fmaf(p, r, 0.5f);
    return fmaf(r * r, p, r);
}

/* exp(x)-1: for |x| < ln2/2 the series directly; otherwise x = k ln2 + r and      */
/* exp(x)-1 = 2^k (exp(r)-1) + (2^k - 1), exact 2^k - 1 for |k| <= 24.              */
float orc_expm1f(float x)
{
    if (fabsf(x) < HALF_LN2) return expm1_poly(x);
    if (x < -16.0f || x > 16.0f) return orc_expf(x) - 1.0f;
    float k = rintf(x * INV_LN2);
    float r = fmaf(-k, LN2_HI, x);
    r = fmaf(-k, LN2_LO, r);
    float two_k = f_from_bits((uint32_t)((int)k + 127) << 23);
    return fmaf(two_k, expm1_poly(r), two_k - 1.0f);
}

/* ------------------------------------------------------------------------- */
/* Tables shared by the samplers: fp32(1/k) and the Stirling-series remainder  */
/* fc(j) = ln j! - [(j+1/2) ln(j+1) - (j+1) + ln(2 pi)/2].                      */
/* ------------------------------------------------------------------------- */
#define INV_TAB 256
#define POIS_INV_MAX 63          /* Poisson inversion (lam < 10) stops at k = 63 */
#define BINOM_INV_MAX 255        /* binomial inversion (n p < 80) stops at k = 255 */
#define BINOM_INV_NP 80.0f       /* n p below this: inversion, else BTRS */
static float INV[INV_TAB];
static float FC_TAB[10];
static pthread_once_t tab_once = PTHREAD_ONCE_INIT;

static void init_tables(void)
{
    INV[0] = 0.0f;
    for (int k = 1; k < INV_TAB; ++k) INV[k] = 1.0f / (float)k;
    for (int j = 0; j < 10; ++j) {
        double jd = (double)j;
        double lf = lgamma(jd + 1.0);
        double st = (jd + 0.5) * log(jd + 1.0) - (jd + 1.0) + 0.5 * log(2.0 * M_PI);
        FC_TAB[j] = (float)(lf - st);
    }
}

void orc_get_tables(float *inv256, float *fc10)
{
    pthread_once(&tab_once, init_tables);
    if (inv256) memcpy(inv256, INV, sizeof INV);
    if (fc10) memcpy(fc10, FC_TAB, sizeof FC_TAB);
}

/* Stirling-series remainder: table for j < 10, else 1/12a - 1/360a^3 + 1/1260a^5, a=j+1. */
float orc_stirling_fc(int32_t j)
{
    if (j < 10) return FC_TAB[j];
    float a = (float)j + 1.0f;
    float ia = 1.0f / a;
    float ia2 = ia * ia;
    float t = 0x1.a01a02p-11f;                     /* 1/1260 */
    t = 0x1.6c16c2p-9f - ia2 * t;                  /* 1/360 - ... */
    t = 0x1.555556p-4f - ia2 * t;                  /* 1/12 - ... */
    return ia * t;
}

/* ------------------------------------------------------------------------- */
/* Samplers.  Each consumes uniforms from one stream in a fixed order.          */
/* ------------------------------------------------------------------------- */
#define REJECT_CAP 100000

/* ln f(k) = k ln lam - lam - ln k! of Poisson(lam), with ln k! by the Stirling series:   */
/*   (k+1-lam) - (k+1/2) log1p((k+1-lam)/lam) - ln(lam)/2 - ln(2pi)/2 - fc(k).               */
/* loglam = ln(lam) as the caller made it.  PTRS's acceptance test compares against this. */
static float ptrs_log_pmf(float lam, float loglam, float kf)
{
    float t = (kf + 1.0f) - lam;
    return t - (kf + 0.5f) * orc_log1pf(t / lam) - 0.5f * loglam - HALF_LOG_2PI - orc_stirling_fc((int32_t)kf);
}

/* The same, exported for its pin against lgamma. */
float orc_ptrs_log_pmf(float lam, int32_t k)
{
    pthread_once(&tab_once, init_tables);
    return ptrs_log_pmf(lam, orc_logf(lam), (float)k);
}

/* Poisson(lam).  lam < 10: sequential-search inversion from k = 0 (one uniform). */
/* lam >= 10: PTRS transformed rejection with squeeze (Hormann 1993).             */
int32_t orc_poisson(float lam, ustream *S)
{
    if (!(lam > 0.0f)) return 0;
    if (lam < 10.0f) {
        EV(EV_POIS_INV);
        float p = orc_expf(-lam);
        float F = p;
        float u = us_u01(S);
        int32_t k = 0;
        while (u > F && k < POIS_INV_MAX) {
            EV(EV_POIS_INV_STEP);
            k += 1;
            p = p * (lam * INV[k]);
            float Fn = F + p;
            if (Fn == F) break;
            F = Fn;
        }
        return k;
    }
    /* a mean of 2^24 or more: fp32 cannot represent the values exactly (overflow flag) */
    if (lam >= 0x1p24f && S->overflow) *S->overflow = 1;
    float slam = sqrtf(lam);
    float loglam = orc_logf(lam);
    float b = 0.931f + 2.53f * slam;
    float a = -0.059f + 0.02483f * b;
    float two_a = 2.0f * a;
    float invalpha = 1.1239f + 1.1328f / (b - 3.4f);
    float vr = 0.9277f - 3.6224f / (b - 2.0f);
    EV(EV_PTRS);
    for (int it = 0; it < REJECT_CAP; ++it) {
        EV(EV_PTRS_TRY);
        float U = us_u01(S) - 0.5f;
        float V = us_u01(S);
        float us = 0.5f - fabsf(U);
        float kf = floorf((two_a / us + b) * U + (lam + 0.43f));
        if (us >= 0.07f && V <= vr) return (int32_t)kf;
        if (kf < 0.0f || (us < 0.013f && V > us)) continue;
        EV(EV_PTRS_SLOW);
        float lhs = orc_logf(V * invalpha / (a / (us * us) + b));
        if (lhs <= ptrs_log_pmf(lam, loglam, kf)) return (int32_t)kf;
    }
    if (S->overflow) *S->overflow = 1;
    return (int32_t)floorf(lam);
}

/* Binomial(n, p) for n*p < 80, 0 < p <= 1/2: inversion from k = 0 (one uniform),  */
/* at most BINOM_INV_MAX steps (P(X > 255) < 1e-40 there).                           */
/* P(X = 0) = q^n = e^x, x = n ln q >= -2 ln 2 n p > -111, is formed as the          */
/* exponential forms it, exp(r) 2^e with x = e ln 2 + r, but with the binary exponent */
/* raised by sc = -120 - e when e < -120 (q^n below the normal fp32 range), and the  */
/* uniform raised by the same 2^sc.  Scaling by a power of two is exact, so every    */
/* step and comparison is the one an fp32 without the lower exponent limit makes;    */
/* sc = 0 for n p < 56, where q^n >= e^-78 is a normal number anyway.  The factor   */
/* of the pmf recurrence, (n+1) r / k - r, is one fma of g = (n+1) r and fp32 1/k.  */
static int32_t binom_inversion(int32_t n, float p, ustream *S)
{
    float q = 1.0f - p;
    float r = p / q;
    float g = r * ((float)n + 1.0f);
    float x = (float)n * orc_log1pf(-p);
    float ek = rintf(x * INV_LN2);
    float rr = fmaf(-ek, LN2_HI, x);
    rr = fmaf(-ek, LN2_LO, rr);
    int32_t e = (int32_t)ek;
    int32_t sc = e < -120 ? -120 - e : 0;
    float f = exp_poly(rr) * f_from_bits((uint32_t)(e + sc + 127) << 23);   /* P(X = 0) 2^sc */
    float F = f;
    float u = us_u01(S) * f_from_bits((uint32_t)(sc + 127) << 23);
    int32_t k = 0;
    EV(EV_BIN_INV);
    while (u > F && k < n && k < BINOM_INV_MAX) {
        EV(EV_BIN_INV_STEP);
        k += 1;
        f = f * fmaf(g, INV[k], -r);                  /* f_k = f_{k-1} (n-k+1)/k p/q */
        float Fn = F + f;
        if (Fn == F) break;
        F = Fn;
    }
    return k;
}

/* ln f(k)/f(m) of Binomial(n, p), r = p/q, m = mf = floor((n+1) p), by the Stirling series:  */
/*   hm + (n+1) ln(nm/nk) + (k+1/2) ln(nk r/(k+1)) - fc(k) - fc(n-k),  nm = n-m+1, nk = n-k+1, */
/*   hm = (m+1/2) ln((m+1)/(r nm)) + fc(m) + fc(n-m),                                           */
/* with ln(nm/nk) = log1p((k-m)/nk).  ln((m+1)/(r nm)) is log1p((m + 1 - r nm) / (r nm)): for */
/* a large mode the ratio is near 1, and rounding it before the log, times m + 1/2, would    */
/* swamp the log-ratio; so the difference is one fp64 fma of exact integers (n - m + 1 and   */
/* m + 1 below 2^28, times the fp32 r: an exact product), rounded once (likewise ln(nk r/(k+1))). */
static float btrs_hm(int32_t n, float nf, int32_t m, float mf, float r)
{
    float nm = nf - mf + 1.0f;
    float rnm = r * nm;
    float dm = (float)fma(-(double)r, (double)(n - m + 1), (double)(m + 1));
    return (mf + 0.5f) * orc_log1pf(dm / rnm) + orc_stirling_fc(m) + orc_stirling_fc(n - m);
}

static float btrs_log_ratio(float hm, int32_t n, float nf, float mf, float r, int32_t k, float kf)
{
    float nk = nf - kf + 1.0f;
    return hm + (nf + 1.0f) * orc_log1pf((kf - mf) / nk)
           + (kf + 0.5f) * orc_log1pf((float)fma((double)r, (double)(n - k + 1), -(double)(k + 1)) / (kf + 1.0f))
           - orc_stirling_fc(k) - orc_stirling_fc(n - k);
}

/* The same for 0 < p <= 1/2, exported for its pin against lgamma. */
float orc_btrs_log_ratio(int32_t n, float p, int32_t k)
{
    pthread_once(&tab_once, init_tables);
    float nf = (float)n;
    float r = p / (1.0f - p);
    float mf = floorf((nf + 1.0f) * p);
    int32_t m = (int32_t)mf;
    return btrs_log_ratio(btrs_hm(n, nf, m, mf, r), n, nf, mf, r, k, (float)k);
}

/* Binomial(n, p) for n*p >= 80, p <= 1/2: transformed rejection with squeeze */
/* (BTRS of Hormann 1993).  Acceptance compares against ln f(k)/f(m), m the mode. */
static int32_t binom_btrs(int32_t n, float p, ustream *S)
{
    float nf = (float)n;
    float q = 1.0f - p;
    float spq = sqrtf(nf * p * q);
    float b = 1.15f + 2.53f * spq;
    float a = -0.0873f + 0.0248f * b + 0.01f * p;
    float two_a = 2.0f * a;
    float c = nf * p + 0.5f;
    float alpha = (2.83f + 5.1f / b) * spq;
    float vr = 0.92f - 4.2f / b;
    float r = p / q;
    float mf = floorf((nf + 1.0f) * p);
    int32_t m = (int32_t)mf;
    float hm = btrs_hm(n, nf, m, mf, r);
    /* a mode of 2^24 or more: fp32 cannot represent the values exactly (overflow flag) */
    if (m >= (1 << 24) && S->overflow) *S->overflow = 1;
    EV(EV_BTRS);
    for (int it = 0; it < REJECT_CAP; ++it) {
        EV(EV_BTRS_TRY);
        float u = us_u01(S) - 0.5f;
        float v = us_u01(S);
        float us = 0.5f - fabsf(u);
        float kf = floorf((two_a / us + b) * u + c);
        if (us >= 0.07f && v <= vr) return (int32_t)kf;
        if (kf < 0.0f || kf > nf) continue;
        int32_t k = (int32_t)kf;
        if (k > n) continue;               /* nf may round n up when n >= 2^24 */
        EV(EV_BTRS_SLOW);
        float lhs = orc_logf(v * alpha / (a / (us * us) + b));
        if (lhs <= btrs_log_ratio(hm, n, nf, mf, r, k, kf)) return k;
    }
    if (S->overflow) *S->overflow = 1;
    return m;
}

int32_t orc_binomial(int32_t n, float p, ustream *S)
{
    if (n <= 0 || !(p > 0.0f)) return 0;
    if (p >= 1.0f) return n;
    if (p > 0.5f) {
        float pc = 1.0f - p;           /* exact for p in (1/2, 1) */
        int32_t k = ((float)n * pc < BINOM_INV_NP) ? binom_inversion(n, pc, S) : binom_btrs(n, pc, S);
        return n - k;
    }
    return ((float)n * p < BINOM_INV_NP) ? binom_inversion(n, p, S) : binom_btrs(n, p, S);
}

/* Gamma(k, 1) for integer k >= 1 by Marsaglia & Tsang (2000), with normals from */
/* Marsaglia's polar method (the second normal of each pair is discarded).        */
float orc_gamma_int(int32_t k, ustream *S)
{
    float d = (float)k - 0x1.555556p-2f;   /* k - 1/3 */
    float c = 1.0f / sqrtf(9.0f * d);
    EV(EV_GAMMA);
    for (int it = 0; it < REJECT_CAP; ++it) {
        float x1, x2, s;
        EV(EV_GAMMA_TRY);
        do {
            EV(EV_GAMMA_POLAR);
            x1 = 2.0f * us_u01(S) - 1.0f;
            x2 = 2.0f * us_u01(S) - 1.0f;
            s = x1 * x1 + x2 * x2;
        } while (s >= 1.0f);
        float z = x1 * sqrtf(-2.0f * orc_logf(s) / s);
        float t = 1.0f + c * z;
        if (t <= 0.0f) continue;
        float v = t * t * t;
        float u = us_u01(S);
        float z2 = z * z;
        if (u < 1.0f - 0.0331f * (z2 * z2)) return d * v;
        EV(EV_GAMMA_SLOW);
        if (orc_logf(u) < 0.5f * z2 + d * ((1.0f - v) + orc_logf(v))) return d * v;
    }
    if (S->overflow) *S->overflow = 1;
    return d;
}

/* GenerateDeparture (Lemma 1 and Algorithm 3 of the paper):                    */
/*  x <= m : D ~ Binomial(x, 1 - e^{-mu h})                                      */
/*  x >  m : T ~ Erlang(x-m, m mu); T > h: D ~ Binomial(x-m-1, h/T);              */
/*           T <= h: D = x-m + Binomial(m, 1 - e^{-mu (h-T)}).                    */
/* pdep = fp32(1 - e^{-mu h}) and rate = fp32(m mu) come from the host tables.   */
/*                                                                               */
/* With score != NULL it also returns the likelihood-ratio score of the draw:    */
/* the mu-derivative of the log-density of the variables the draw consumed.       */
/*  x <= m : D kap - (x - D) h, kap = fp32(h e^{-mu h} / (1 - e^{-mu h}))         */
/*  x >  m : (x-m)/mu - m T   (Erlang density of T; the split given T > h is free */
/*           of mu), and if T <= h, with s = h - T, p2 = 1 - e^{-mu s} and        */
/*           D' = D - (x-m):  - (m - D') s + D' s (1 - p2) / p2.                  */
/* x = 0 consumes nothing and scores 0.                                          */
int32_t orc_gendep(int32_t x, int32_t m, float mu, float dt, float pdep, float rate, float kap,
                   ustream *S, float *score)
{
    if (score) *score = 0.0f;
    if (x <= 0) return 0;
    EV(EV_DEPART);
    if (x <= m) {
        int32_t D = orc_binomial(x, pdep, S);
        if (score) *score = (float)D * kap - (float)(x - D) * dt;
        return D;
    }
    int32_t k = x - m;
    float T = orc_gamma_int(k, S) / rate;
    float sc = (float)k / mu - (float)m * T;
    int32_t D;
    EV(EV_BIN_PREP);
    if (T > dt) {
        D = orc_binomial(k - 1, dt / T, S);
    } else {
        float s = dt - T;
        EV(EV_EXPM1);
        float p2 = -orc_expm1f(-(mu * s));
        int32_t Dp = orc_binomial(m, p2, S);
        sc = sc - (float)(m - Dp) * s;
        if (Dp > 0) sc = sc + (float)Dp * (s * (1.0f - p2) / p2);
        D = k + Dp;
    }
    if (score) *score = sc;
    return D;
}

/* Naive Euler departures, Eq. (1): D = min(x, S), S ~ Poisson(min(x, m) mu h).  */
/* Score (mu-derivative of the Poisson log-density of S): S/mu - min(x, m) h.     */
int32_t orc_gendep_naive(int32_t x, int32_t m, float mudt, float mu, float dt, ustream *S,
                         float *score)
{
    if (score) *score = 0.0f;
    if (x <= 0) return 0;
    int32_t b = x < m ? x : m;
    int32_t s = orc_poisson((float)b * mudt, S);
    if (score) *score = (float)s / mu - (float)b * dt;
    return s < x ? s : x;
}

/* Score of an external-arrival draw A ~ Poisson(lambda0 g) in lambda0: A/lambda0 - g. */
static float arrival_score(int32_t A, float l0, float g)
{
    return (float)A / l0 - g;
}

/* ------------------------------------------------------------------------- */
/* Network and host tables.                                                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    const int32_t *row_ptr;    /* [n+1] */
    const int32_t *col;        /* [nnz] */
    const float *prob;         /* [nnz] routing probabilities p_ij */
    const int32_t *servers;    /* [n] m_i >= 1 */
    const float *mu;           /* [n] per-server service rate */
    int32_t n_src;
    const int32_t *src;        /* [n_src] stations with external arrivals */
    const float *lambda0;      /* [n_src] base external rate */
    int32_t shape_kind;        /* 0 constant, 1 sinusoid, 2 piecewise constant */
    double amp, period, phase; /* sinusoid: shape(t) = 1 + amp sin(2 pi t / period + phase);     */
                               /* piecewise: period > 0 repeats the knots, 0 does not          */
    /* Staffing (time-varying servers, Section 2.1): n_seg = 0 keeps `servers`; else      */
    /* segment k starts at interval index seg_start[k] (seg_start[0] = 0, increasing) and  */
    /* station i has seg_servers[k n + i] >= 1 servers; period > 0 repeats the schedule.  */
    int32_t n_seg;
    const int32_t *seg_start;
    const int32_t *seg_servers;
    int32_t seg_period;
    /* Piecewise-constant shape: shape(t) = knot_shape[k] on [knot_t[k], knot_t[k+1]) with     */
    /* knot_t[0] = 0 increasing; the last piece runs to the period's end (periodic) or on.  */
    int32_t n_knots;
    const double *knot_t;
    const double *knot_shape;
} orc_net;

/* Integral of the piecewise-constant shape over [t0, t1]: every piece [lo, hi) of height c  */
/* adds c (min(t1, hi) - max(t0, lo)) when that length is positive, pieces taken in time     */
/* order (period j = floor(t0 / P) .. floor(t1 / P), piece k ascending); in period j a piece  */
/* spans j P + knot_t[k] .. j P + knot_t[k+1], the last one ending at (j + 1) P.             */
static double piecewise_integral(const orc_net *net, double t0, double t1)
{
    double val = 0.0;
    int32_t nk = net->n_knots;
    int periodic = net->period > 0.0;
    long long j0 = periodic ? (long long)floor(t0 / net->period) : 0;
    long long j1 = periodic ? (long long)floor(t1 / net->period) : 0;
    for (long long j = j0; j <= j1; ++j) {
        double base = periodic ? (double)j * net->period : 0.0;
        for (int32_t k = 0; k < nk; ++k) {
            double lo = base + net->knot_t[k];
            double hi = k + 1 < nk ? base + net->knot_t[k + 1] : (periodic ? (double)(j + 1) * net->period : INFINITY);
            double a = lo > t0 ? lo : t0;
            double b = hi < t1 ? hi : t1;
            if (b > a) val += net->knot_shape[k] * (b - a);
        }
    }
    return val;
}

/* Servers of station i during interval tau (step0 = tau - 1): the segment whose start is  */
/* the last one at or before step0 (mod the period).                                      */
static int32_t servers_at(const orc_net *net, int32_t i, int32_t step0)
{
    if (net->n_seg <= 0) return net->servers[i];
    int32_t t = net->seg_period > 0 ? step0 % net->seg_period : step0;
    int32_t k = 0;
    while (k + 1 < net->n_seg && net->seg_start[k + 1] <= t) ++k;
    return net->seg_servers[(size_t)k * net->n + i];
}

/* Conditional routing probabilities for the sequential-binomial multinomial:   */
/* q_e = p_e / (p_exit + sum_{l >= e} p_l), clamped to [0, 1], fp64 -> fp32.     */
/* Departure probability pdep_i = 1 - e^{-mu_i h}, service-capacity rate m_i mu_i, */
/* mu_i h, the departure score constant kap_i = h e^{-mu_i h} / (1 - e^{-mu_i h}),   */
/* and rate integrals g[tau-1] = int_{(tau-1)h}^{tau h} shape(t) dt.                */
int orc_tables(const orc_net *net, float dt, int32_t K, float *q, float *pdep, float *rate,
               float *mudt, float *kap, float *g)
{
    int32_t n = net->n;
    double dtd = (double)dt;
    if (q) {
        for (int32_t i = 0; i < n; ++i) {
            int32_t b = net->row_ptr[i], e = net->row_ptr[i + 1];
            double tot = 0.0;
            for (int32_t j = b; j < e; ++j) tot += (double)net->prob[j];
            double pexit = 1.0 - tot;
            if (pexit < 0.0) pexit = 0.0;
            double suffix = pexit;
            for (int32_t j = e - 1; j >= b; --j) {
                suffix += (double)net->prob[j];
                double qq = suffix > 0.0 ? (double)net->prob[j] / suffix : 1.0;
                if (qq > 1.0) qq = 1.0;
                if (qq < 0.0) qq = 0.0;
                q[j] = (float)qq;
            }
        }
    }
    for (int32_t i = 0; i < n; ++i) {
        double mud = (double)net->mu[i];
        if (pdep) pdep[i] = (float)(-expm1(-(mud * dtd)));
        if (rate) rate[i] = (float)((double)net->servers[i] * mud);
        if (mudt) mudt[i] = (float)(mud * dtd);
        if (kap) kap[i] = (float)(dtd * exp(-(mud * dtd)) / -expm1(-(mud * dtd)));
    }
    if (g) {
        if (net->shape_kind == 0) {
            for (int32_t t = 0; t < K; ++t) g[t] = (float)dtd;
        } else if (net->shape_kind == 2) {
            for (int32_t t = 0; t < K; ++t) g[t] = (float)piecewise_integral(net, (double)t * dtd, (double)(t + 1) * dtd);
        } else {
            double w = 2.0 * M_PI / net->period;
            for (int32_t t = 0; t < K; ++t) {
                double t0 = (double)t * dtd, t1 = (double)(t + 1) * dtd;
                double val = (t1 - t0) + net->amp / w * (cos(w * t0 + net->phase) - cos(w * t1 + net->phase));
                g[t] = (float)val;
            }
        }
    }
    return ORC_OK;
}

static int validate(const orc_net *net, int32_t scheme)
{
    if (!net || net->n <= 0 || !net->row_ptr || !net->servers || !net->mu) return ORC_EINVAL;
    int32_t n = net->n;
    if (net->row_ptr[0] != 0) return ORC_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        if (net->row_ptr[i + 1] < net->row_ptr[i]) return ORC_EINVAL;
        if (net->servers[i] < 1 || !(net->mu[i] > 0.0f)) return ORC_EINVAL;
        for (int32_t e = net->row_ptr[i]; e < net->row_ptr[i + 1]; ++e) {
            if (net->col[e] < 0 || net->col[e] >= n) return ORC_EINVAL;
            if (scheme == SCHEME_FORWARD && net->col[e] <= i) return ORC_ENOTDAG;
        }
    }
    for (int32_t s = 0; s < net->n_src; ++s)
        if (net->src[s] < 0 || net->src[s] >= n) return ORC_EINVAL;
    if (net->n_seg < 0) return ORC_EINVAL;
    if (net->n_seg > 0) {
        if (!net->seg_start || !net->seg_servers || net->seg_start[0] != 0 || net->seg_period < 0) return ORC_EINVAL;
        for (int32_t k = 1; k < net->n_seg; ++k)
            if (net->seg_start[k] <= net->seg_start[k - 1]) return ORC_EINVAL;
        if (net->seg_period > 0 && net->seg_start[net->n_seg - 1] >= net->seg_period) return ORC_EINVAL;
        for (int64_t j = 0; j < (int64_t)net->n_seg * n; ++j)
            if (net->seg_servers[j] < 1) return ORC_EINVAL;
    }
    if (net->shape_kind < 0 || net->shape_kind > 2) return ORC_EINVAL;
    if (net->shape_kind == 2) {
        if (net->n_knots < 1 || !net->knot_t || !net->knot_shape || net->knot_t[0] != 0.0) return ORC_EINVAL;
        if (!(net->period >= 0.0) || !isfinite(net->period)) return ORC_EINVAL;
        for (int32_t k = 0; k < net->n_knots; ++k) {
            if (!(net->knot_shape[k] >= 0.0) || !isfinite(net->knot_shape[k]) || !isfinite(net->knot_t[k]))
                return ORC_EINVAL;
            if (k > 0 && !(net->knot_t[k] > net->knot_t[k - 1])) return ORC_EINVAL;
        }
        if (net->period > 0.0 && !(net->knot_t[net->n_knots - 1] < net->period)) return ORC_EINVAL;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* The schemes (Section 2.2 and Algorithms 1-2).                                */
/* ------------------------------------------------------------------------- */
typedef struct {
    const orc_net *net;
    int32_t scheme, dep_mode, K;
    float dt;
    uint64_t seed;
    uint32_t net_id;
    const float *q, *pdep, *rate, *mudt, *kap, *g;
    const float *lam_of;        /* [n] lambda0 per station (0 if not a source) */
    const int32_t *src_of;      /* [n] index into the source list, or -1 */
    const int32_t *init_state;  /* [n] or NULL */
    const int32_t *inj_arr;     /* [K][n] injected external arrivals, or NULL */
    const int32_t *rep_ids;
    int32_t n_reps;
    int32_t *final_state;       /* [n_reps][n] */
    int64_t *sumN, *sumQ, *sumD;/* [n_reps][n] or NULL */
    float *score_mu;            /* [n_reps][n] or NULL: summed scores of the departure draws */
    float *score_lam;           /* [n_reps][n_src] or NULL: summed scores of the arrival draws */
    int32_t rec_t0, rec_len;    /* recorded steps tau = rec_t0 .. rec_t0 + rec_len - 1 */
    int32_t *rec_N, *rec_D;     /* [n_reps][rec_len][n] or NULL: N_tau and D_tau */
    int32_t *rec_R;             /* [n_reps][rec_len][nnz] or NULL: routed counts per edge */
    int next;                   /* work counter */
    pthread_mutex_t lock;
    int overflow;
} run_ctx;

/* External arrivals A^ex_{tau,i} ~ Poisson(int lambda_i) = Poisson(lambda0_i g[tau-1]). */
/* With scores on, a drawn arrival count adds its lambda0 score to the source's sum.    */
static int32_t external_arrivals(const run_ctx *c, int32_t i, int32_t tau, uint32_t rep, int *ovf,
                                 float *slam)
{
    if (c->inj_arr) return c->inj_arr[(size_t)(tau - 1) * c->net->n + i];
    float l0 = c->lam_of[i];
    if (!(l0 > 0.0f)) return 0;
    ustream S;
    us_init(&S, c->seed, c->net_id, rep, (uint32_t)i, (uint32_t)(tau - 1), SUB_ARRIVAL, ovf);
    int32_t A = orc_poisson(l0 * c->g[tau - 1], &S);
    if (slam) {
        int32_t j = c->src_of[i];
        slam[j] = slam[j] + arrival_score(A, l0, c->g[tau - 1]);
    }
    return A;
}

/* Departures of station i from x customers; with scores on, a draw (x > 0) adds its */
/* mu score to the station's sum.                                                    */
static int32_t departures(const run_ctx *c, int32_t i, int32_t x, int32_t tau, uint32_t rep, int *ovf,
                          float *smu)
{
    const orc_net *net = c->net;
    ustream S;
    us_init(&S, c->seed, c->net_id, rep, (uint32_t)i, (uint32_t)(tau - 1), SUB_DEPART, ovf);
    float sc = 0.0f;
    int32_t D;
    int32_t m = servers_at(net, i, tau - 1);
    /* fp32(m mu) for the servers of this interval, as the host tables make it */
    float rate = net->n_seg > 0 ? (float)((double)m * (double)net->mu[i]) : c->rate[i];
    if (c->dep_mode == DEP_NAIVE)
        D = orc_gendep_naive(x, m, c->mudt[i], net->mu[i], c->dt, &S, &sc);
    else
        D = orc_gendep(x, m, net->mu[i], c->dt, c->pdep[i], rate, c->kap[i], &S, &sc);
    if (smu && x > 0) smu[i] = smu[i] + sc;
    return D;
}

/* Multinomial(D, (p_i1..p_in, p_i,exit)) as sequential conditional binomials  */
/* in CSR order; what is left after the last edge exits the network.            */
/* With Rrow != NULL (a zeroed row of per-edge counts) the routed counts are recorded.   */
static void route(const run_ctx *c, int32_t i, int32_t D, int32_t tau, uint32_t rep,
                  int32_t *Ain, int *ovf, int32_t *Rrow)
{
    if (D <= 0) return;
    const orc_net *net = c->net;
    ustream S;
    us_init(&S, c->seed, c->net_id, rep, (uint32_t)i, (uint32_t)(tau - 1), SUB_ROUTE, ovf);
    int32_t rem = D;
    for (int32_t e = net->row_ptr[i]; e < net->row_ptr[i + 1] && rem > 0; ++e) {
        EV(EV_EDGE);
        int32_t R = orc_binomial(rem, c->q[e], &S);
        if (R) EV(EV_PUSH);
        Ain[net->col[e]] += R;
        if (Rrow) Rrow[e] = R;
        rem -= R;
    }
}

static void simulate_rep(run_ctx *c, int32_t slot, int32_t *N, int32_t *D, int32_t *A, int32_t *Ain)
{
    const orc_net *net = c->net;
    int32_t n = net->n;
    uint32_t rep = (uint32_t)c->rep_ids[slot];
    int ovf = 0;
    int64_t *sN = c->sumN ? c->sumN + (size_t)slot * n : NULL;
    int64_t *sQ = c->sumQ ? c->sumQ + (size_t)slot * n : NULL;
    int64_t *sD = c->sumD ? c->sumD + (size_t)slot * n : NULL;
    float *smu = c->score_mu ? c->score_mu + (size_t)slot * n : NULL;
    float *slam = c->score_lam ? c->score_lam + (size_t)slot * net->n_src : NULL;
    for (int32_t i = 0; i < n; ++i) {
        N[i] = c->init_state ? c->init_state[i] : 0;
        if (sN) { sN[i] = 0; sQ[i] = 0; sD[i] = 0; }
        if (smu) smu[i] = 0.0f;
    }
    for (int32_t j = 0; slam && j < net->n_src; ++j) slam[j] = 0.0f;
    int32_t nnz = net->row_ptr[n];
    for (int32_t tau = 1; tau <= c->K; ++tau) {
        for (int32_t i = 0; i < n; ++i) Ain[i] = 0;
        int32_t *Rrow = NULL;
        int32_t rt = tau - c->rec_t0;
        if (c->rec_N && rt >= 0 && rt < c->rec_len) {
            Rrow = c->rec_R + ((size_t)slot * c->rec_len + rt) * (size_t)nnz;
            for (int32_t e = 0; e < nnz; ++e) Rrow[e] = 0;
        }
        if (c->scheme == SCHEME_BACKWARD) {
            /* Algorithm 1: departures from N_{tau-1}; routing; external and internal */
            /* arrivals all land at the end of the interval.                          */
            for (int32_t i = 0; i < n; ++i) D[i] = departures(c, i, N[i], tau, rep, &ovf, smu);
            for (int32_t i = 0; i < n; ++i) route(c, i, D[i], tau, rep, Ain, &ovf, Rrow);
            for (int32_t i = 0; i < n; ++i) A[i] = external_arrivals(c, i, tau, rep, &ovf, slam);
            for (int32_t i = 0; i < n; ++i) N[i] = N[i] - D[i] + A[i] + Ain[i];
        } else {
            /* Node-by-node forward scheme in topological (index) order: arrivals  */
            /* of the interval are present at its start; departures are drawn from */
            /* N_{tau-1} + A^ex + A^in; routed customers reach later nodes at once. */
            for (int32_t i = 0; i < n; ++i) {
                A[i] = external_arrivals(c, i, tau, rep, &ovf, slam);
                int32_t x = N[i] + A[i] + Ain[i];
                D[i] = departures(c, i, x, tau, rep, &ovf, smu);
                N[i] = x - D[i];
                route(c, i, D[i], tau, rep, Ain, &ovf, Rrow);
            }
        }
        if (Rrow) {
            size_t row = ((size_t)slot * c->rec_len + rt) * (size_t)n;
            memcpy(c->rec_N + row, N, sizeof(int32_t) * (size_t)n);
            memcpy(c->rec_D + row, D, sizeof(int32_t) * (size_t)n);
        }
        if (sN) {
            for (int32_t i = 0; i < n; ++i) {
                int32_t qv = N[i] - servers_at(net, i, tau - 1);   /* N_tau against the servers of interval tau */
                sN[i] += N[i];
                sQ[i] += qv > 0 ? qv : 0;
                sD[i] += D[i];
            }
        }
    }
    memcpy(c->final_state + (size_t)slot * n, N, sizeof(int32_t) * (size_t)n);
    if (ovf) {
        pthread_mutex_lock(&c->lock);
        c->overflow = 1;
        pthread_mutex_unlock(&c->lock);
    }
}

static void *worker(void *arg)
{
    run_ctx *c = (run_ctx *)arg;
    int32_t n = c->net->n;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)n);
    if (!buf) return NULL;
    for (;;) {
        pthread_mutex_lock(&c->lock);
        int slot = c->next++;
        pthread_mutex_unlock(&c->lock);
        if (slot >= c->n_reps) break;
        simulate_rep(c, slot, buf, buf + n, buf + 2 * n, buf + 3 * n);
        tl_ev[EV_STATION_STEP] += (int64_t)n * c->K;
    }
    free(buf);
    ev_flush();
    return NULL;
}

/* Simulate the replications listed in rep_ids (global replication ids).       */
/* Outputs per listed replication: final state, and sums over tau = 1..K of N,  */
/* (N - m)^+ and D per station; optionally the per-station sums of the          */
/* departure-draw scores (in mu_i) and per-source sums of the arrival-draw      */
/* scores (in lambda0_s), each accumulated in fp32 in step order.              */
static int run_impl(const orc_net *net, int32_t scheme, int32_t dep_mode, float dt, int32_t K,
                    uint64_t seed, uint32_t net_id, int32_t n_reps, const int32_t *rep_ids,
                    const int32_t *init_state, const int32_t *inj_arr, int32_t *final_state,
                    int64_t *sumN, int64_t *sumQ, int64_t *sumD, float *score_mu, float *score_lam,
                    int32_t rec_t0, int32_t rec_len, int32_t *rec_N, int32_t *rec_D, int32_t *rec_R,
                    int32_t n_threads)
{
    pthread_once(&tab_once, init_tables);
    int rc = validate(net, scheme);
    if (rc) return rc;
    if (!(dt > 0.0f) || K < 0 || n_reps < 0 || !rep_ids || !final_state) return ORC_EINVAL;
    if ((sumN == NULL) != (sumQ == NULL) || (sumN == NULL) != (sumD == NULL)) return ORC_EINVAL;
    int32_t n = net->n, nnz = net->row_ptr[n];
    float *q = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float *tab = (float *)malloc(sizeof(float) * (5 * (size_t)n + (size_t)(K > 0 ? K : 1)));
    int32_t *src_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!q || !tab || !src_of) { free(q); free(tab); free(src_of); return ORC_ENOMEM; }
    float *pdep = tab, *rate = tab + n, *mudt = tab + 2 * n, *lam_of = tab + 3 * n, *kap = tab + 4 * n,
          *g = tab + 5 * n;
    orc_tables(net, dt, K, q, pdep, rate, mudt, kap, g);
    for (int32_t i = 0; i < n; ++i) { lam_of[i] = 0.0f; src_of[i] = -1; }
    for (int32_t s = 0; s < net->n_src; ++s) { lam_of[net->src[s]] = net->lambda0[s]; src_of[net->src[s]] = s; }

    run_ctx c;
    memset(&c, 0, sizeof c);
    c.net = net; c.scheme = scheme; c.dep_mode = dep_mode; c.K = K; c.dt = dt;
    c.seed = seed; c.net_id = net_id; c.q = q; c.pdep = pdep; c.rate = rate; c.mudt = mudt;
    c.kap = kap; c.g = g; c.lam_of = lam_of; c.src_of = src_of;
    c.init_state = init_state; c.inj_arr = inj_arr;
    c.rep_ids = rep_ids; c.n_reps = n_reps; c.final_state = final_state;
    c.sumN = sumN; c.sumQ = sumQ; c.sumD = sumD; c.score_mu = score_mu; c.score_lam = score_lam;
    c.rec_t0 = rec_t0; c.rec_len = rec_len; c.rec_N = rec_N; c.rec_D = rec_D; c.rec_R = rec_R;
    pthread_mutex_init(&c.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > n_reps) n_threads = n_reps > 0 ? n_reps : 1;
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    int started = 0;
    for (int t = 0; th && t < n_threads; ++t)
        if (pthread_create(&th[t], NULL, worker, &c) == 0) started++;
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    if (started == 0) worker(&c);
    free(th);
    pthread_mutex_destroy(&c.lock);
    free(q); free(tab); free(src_of);
    return c.overflow ? ORC_EOVERFLOW : ORC_OK;
}

int orc_run(const orc_net *net, int32_t scheme, int32_t dep_mode, float dt, int32_t K,
            uint64_t seed, uint32_t net_id, int32_t n_reps, const int32_t *rep_ids,
            const int32_t *init_state, const int32_t *inj_arr, int32_t *final_state,
            int64_t *sumN, int64_t *sumQ, int64_t *sumD, float *score_mu, float *score_lam,
            int32_t n_threads)
{
    return run_impl(net, scheme, dep_mode, dt, K, seed, net_id, n_reps, rep_ids, init_state, inj_arr,
                    final_state, sumN, sumQ, sumD, score_mu, score_lam, 0, 0, NULL, NULL, NULL, n_threads);
}

/* A run that also records the sample path over steps tau = rec_t0 .. rec_t0 + rec_len - 1:  */
/* N_tau (end of the interval), D_tau and the routed count of every edge in interval tau,     */
/* per listed replication ([n_reps][rec_len][n], [n_reps][rec_len][nnz]).                       */
int orc_run_record(const orc_net *net, int32_t scheme, int32_t dep_mode, float dt, int32_t K,
                   uint64_t seed, uint32_t net_id, int32_t n_reps, const int32_t *rep_ids,
                   const int32_t *init_state, int32_t *final_state, int32_t rec_t0, int32_t rec_len,
                   int32_t *rec_N, int32_t *rec_D, int32_t *rec_R, int32_t n_threads)
{
    if (rec_t0 < 1 || rec_len < 1 || !rec_N || !rec_D || !rec_R) return ORC_EINVAL;
    return run_impl(net, scheme, dep_mode, dt, K, seed, net_id, n_reps, rep_ids, init_state, NULL,
                    final_state, NULL, NULL, NULL, NULL, NULL, rec_t0, rec_len, rec_N, rec_D, rec_R,
                    n_threads);
}

/* ------------------------------------------------------------------------- */
/* Sojourn times (Section 6, Algorithm 4, Lemma 3).                            */
/* ------------------------------------------------------------------------- */
/* ((m-1)/m)^e in fp32; 1 for e = 0, 0 for m = 1 and e > 0.                    */
static float stay_pow(int32_t e, int32_t m)
{
    if (e <= 0) return 1.0f;
    if (m == 1) return 0.0f;
    return orc_expf((float)e * orc_log1pf(-1.0f / (float)m));
}

/* Lemma 3: probability that a server busy with the tagged customer at the start of an   */
/* interval still serves it at the end, given x customers at the start and d departures. */
static float p_stay(int32_t x, int32_t d, int32_t m)
{
    if (x <= m) return (float)(x - d) / (float)x;
    if (x <= m + d) return stay_pow(x - m, m) * ((float)(x - d) / (float)m);
    return stay_pow(d, m);
}

/* One tagged customer entering node i0 during interval tau0, walked through the recorded */
/* path of one replication (Algorithm 4).  Returns the sojourn time in intervals, or -1 if */
/* the walk needs an interval beyond the record.                                          */
static int32_t sojourn_one(const orc_net *net, int32_t scheme, int32_t t0, int32_t len, const int32_t *RN,
                           const int32_t *RD, const int32_t *RR, int32_t i0, int32_t tau0, ustream *S)
{
    int32_t n = net->n, nnz = net->row_ptr[n];
    int32_t i = i0, tau = tau0, T = 0;
#define REC_N(t, s) RN[(size_t)((t) - t0) * n + (s)]
#define REC_D(t, s) RD[(size_t)((t) - t0) * n + (s)]
#define IN_REC(t) ((t) >= t0 && (t) < t0 + len)
    for (;;) {
        /* setup: the tagged customer is the last of the N_{tau,i} present at tau h */
        if (!IN_REC(tau)) return -1;
        int32_t pos = REC_N(tau, i);
        if (pos > servers_at(net, i, tau)) {
            /* waiting: the first j with N_{tau,i} - D_{tau+1,i} - ... - D_{tau+j,i} <= m */
            int32_t j = 0;
            while (pos > servers_at(net, i, tau + j)) {
                j += 1;
                if (!IN_REC(tau + j)) return -1;
                pos -= REC_D(tau + j, i);
            }
            T += j;
            tau += j;
        }
        /* service: interval tau + 1 keeps the customer with the probability of Lemma 3 */
        for (;;) {
            if (!IN_REC(tau + 1)) return -1;
            int32_t d = REC_D(tau + 1, i);
            int32_t x = scheme == SCHEME_BACKWARD ? (IN_REC(tau) ? REC_N(tau, i) : 0) : REC_N(tau + 1, i) + d;
            if (x < 1) x = 1;                          /* the tagged customer is present */
            int32_t m = servers_at(net, i, tau);      /* servers of interval tau + 1 */
            float ps = p_stay(x, d, m);
            T += 1;
            tau += 1;
            if (us_u01(S) < ps) continue;
            /* departs: next node j with probability R_{tau,i,j} / D_{tau,i}, else exits */
            int32_t k = (int32_t)floorf(us_u01(S) * (float)d);
            if (k > d - 1) k = d - 1;
            const int32_t *Rrow = RR + (size_t)(tau - t0) * nnz;
            int32_t cum = 0, next = -1;
            for (int32_t e = net->row_ptr[i]; e < net->row_ptr[i + 1]; ++e) {
                cum += Rrow[e];
                if (k < cum) { next = net->col[e]; break; }
            }
            if (next < 0) return T;
            i = next;
            break;
        }
    }
#undef REC_N
#undef REC_D
#undef IN_REC
}

/* Lemma 3's stay probability, exported for its pins. */
float orc_lemma3(int32_t x, int32_t d, int32_t m)
{
    pthread_once(&tab_once, init_tables);
    return p_stay(x, d, m);
}

/* Sojourn samples from recorded paths: for listed replication r (global id rep_ids[r])  */
/* and sample k, a customer entering node i0[k] during interval tau0[k]; its uniforms are  */
/* the stream (rep, k, 0, substream 3).  out [n_reps][n_samples] in intervals, -1 when     */
/* the record is too short.                                                                 */
int orc_sojourn(const orc_net *net, int32_t scheme, uint64_t seed, uint32_t net_id, int32_t n_reps,
                const int32_t *rep_ids, int32_t rec_t0, int32_t rec_len, const int32_t *rec_N,
                const int32_t *rec_D, const int32_t *rec_R, int32_t n_samples, const int32_t *i0,
                const int32_t *tau0, int32_t *out)
{
    pthread_once(&tab_once, init_tables);
    int rc = validate(net, scheme);
    if (rc) return rc;
    if (rec_t0 < 1 || rec_len < 1 || n_reps < 0 || n_samples < 0) return ORC_EINVAL;
    int32_t n = net->n, nnz = net->row_ptr[n];
    int ovf = 0;
    for (int32_t r = 0; r < n_reps; ++r) {
        const int32_t *RN = rec_N + (size_t)r * rec_len * n, *RD = rec_D + (size_t)r * rec_len * n;
        const int32_t *RR = rec_R + (size_t)r * rec_len * nnz;
        for (int32_t k = 0; k < n_samples; ++k) {
            if (i0[k] < 0 || i0[k] >= n) return ORC_EINVAL;
            ustream S;
            us_init(&S, seed, net_id, (uint32_t)rep_ids[r], (uint32_t)k, 0u, SUB_SOJOURN, &ovf);
            out[(size_t)r * n_samples + k] = sojourn_one(net, scheme, rec_t0, rec_len, RN, RD, RR, i0[k], tau0[k], &S);
        }
    }
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Direct sampler access for distribution tests.  Sample s uses the stream     */
/* (rep = rep0 + s, station, step, substream).                                  */
/* ------------------------------------------------------------------------- */
enum { SMP_POISSON = 0, SMP_BINOMIAL = 1, SMP_GAMMA = 2, SMP_GENDEP = 3, SMP_GENDEP_NAIVE = 4 };

int orc_sample(int32_t kind, int64_t count, uint64_t seed, uint32_t rep0, uint32_t station,
               uint32_t step0, uint32_t sub, int32_t i0, int32_t i1, float f0, float f1,
               float f2, float f3, float *out)
{
    pthread_once(&tab_once, init_tables);
    int ovf = 0;
    for (int64_t s = 0; s < count; ++s) {
        ustream S;
        us_init(&S, seed, 0u, rep0 + (uint32_t)s, station, step0, sub, &ovf);
        float v = 0.0f;
        switch (kind) {
        case SMP_POISSON: v = (float)orc_poisson(f0, &S); break;
        case SMP_BINOMIAL: v = (float)orc_binomial(i0, f0, &S); break;
        case SMP_GAMMA: v = orc_gamma_int(i0, &S); break;
        case SMP_GENDEP: {
            /* i0 = x, i1 = m, f0 = mu, f1 = h, f2 = pdep, f3 = rate */
            v = (float)orc_gendep(i0, i1, f0, f1, f2, f3, 0.0f, &S, NULL);
            break;
        }
        case SMP_GENDEP_NAIVE: v = (float)orc_gendep_naive(i0, i1, f0, 0.0f, 0.0f, &S, NULL); break;
        default: return ORC_EINVAL;
        }
        out[s] = v;
    }
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* Draws with their likelihood-ratio scores, sample s on the stream (rep0 + s,    */
/* station, step0, sub).  kind 0: A ~ Poisson(lam0 g), score in lam0 (f0 = lam0,   */
/* f1 = g).  kind 3: GenerateDeparture(x = i0, m = i1, mu = f0, h = f1), score in   */
/* mu; the constants pdep, m mu and kap are made as the host tables make them.     */
/* kind 4: naive departures, same arguments.                                       */
int orc_sample_score(int32_t kind, int64_t count, uint64_t seed, uint32_t rep0, uint32_t station,
                     uint32_t step0, uint32_t sub, int32_t i0, int32_t i1, float f0, float f1,
                     float *value, float *score)
{
    pthread_once(&tab_once, init_tables);
    int ovf = 0;
    double mud = (double)f0, dtd = (double)f1;
    float pdep = (float)(-expm1(-(mud * dtd)));
    float rate = (float)((double)i1 * mud);
    float mudt = (float)(mud * dtd);
    float kap = (float)(dtd * exp(-(mud * dtd)) / -expm1(-(mud * dtd)));
    for (int64_t s = 0; s < count; ++s) {
        ustream S;
        us_init(&S, seed, 0u, rep0 + (uint32_t)s, station, step0, sub, &ovf);
        float sc = 0.0f;
        int32_t v;
        switch (kind) {
        case SMP_POISSON:
            v = orc_poisson(f0 * f1, &S);
            sc = arrival_score(v, f0, f1);
            break;
        case SMP_GENDEP: v = orc_gendep(i0, i1, f0, f1, pdep, rate, kap, &S, &sc); break;
        case SMP_GENDEP_NAIVE: v = orc_gendep_naive(i0, i1, mudt, f0, f1, &S, &sc); break;
        default: return ORC_EINVAL;
        }
        value[s] = (float)v;
        score[s] = sc;
    }
    return ovf ? ORC_EOVERFLOW : ORC_OK;
}

/* Vector access to the elementary functions (kind 0 log, 1 log1p, 2 exp, 3 expm1). */
int orc_math(int32_t kind, int64_t count, const float *x, float *y)
{
    for (int64_t i = 0; i < count; ++i) {
        switch (kind) {
        case 0: y[i] = orc_logf(x[i]); break;
        case 1: y[i] = orc_log1pf(x[i]); break;
        case 2: y[i] = orc_expf(x[i]); break;
        case 3: y[i] = orc_expm1f(x[i]); break;
        case 4: {
            uint32_t b;
            memcpy(&b, &x[i], sizeof b);
            y[i] = orc_u01(b);
            break;
        }
        default: return ORC_EINVAL;
        }
    }
    return ORC_OK;
}

void orc_philox_batch(int64_t count, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < count; ++i) orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}
