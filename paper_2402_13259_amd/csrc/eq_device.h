// eq_device.h -- device building blocks of the Euler-approximation simulator (gfx950).
//
// Counter-based randomness (Philox4x32-10), the fp32 elementary functions the samplers
// need, and the samplers: Poisson, binomial, integer-shape gamma, and the exact
// pure-departure sampler of Lemma 1 / Algorithm 3.
//
// Every floating-point operation that can decide an integer outcome is an IEEE fp32
// basic operation (+ - * / sqrt, correctly rounded: build with
// -fhip-fp32-correctly-rounded-divide-sqrt), an explicit fma, an int<->float conversion,
// floor or round-to-nearest-even.  The file is built with -ffp-contract=off so that the
// compiler never fuses a multiply and an add on its own.  Together with the fixed stream
// layout this makes every sample a pure function of (seed, net_id, rep, station, step,
// substream) and of the sampler's arguments, whatever the launch shape.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eq_internal.h"

#pragma clang fp contract(off)

namespace eq {

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two 32x32->64-bit
// products with multipliers 0xD2511F53 and 0xCD9E8D57, key bumped by the Weyl constants
// 0x9E3779B9 and 0xBB67AE85 after every round.
// ------------------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    // Three-way xors as one gfx950 bitop3 each (truth table 0x96), which the compiler
    // does not form by itself here.
    n.x = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96);
    n.y = (uint32_t)p1;
    n.z = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96);
    n.w = (uint32_t)p0;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Substreams of one (rep, station, step): external arrivals, departures, routing; substream 3
// of (rep, sample, 0) drives the sojourn sampler.
enum : uint32_t { SUB_ARR = 0u, SUB_DEP = 1u, SUB_ROUTE = 2u, SUB_SOJ = 3u };
constexpr uint32_t kBlockLimit = 1u << 24;

// A uniform stream: Philox counter (rep, station, step-1, sub<<24 | block), key
// (seed_lo, seed_hi ^ net_id); the four output words are used in order, then the block
// index advances.  The buffer is rotated instead of indexed so that it stays in VGPRs.
struct Stream {
  uint32_t k0, k1, rep, station, step0, hi, block, left;
  uint32_t b0, b1, b2, b3;
};

__device__ __forceinline__ Stream make_stream(uint32_t k0, uint32_t k1, uint32_t rep,
                                              uint32_t station, uint32_t step0, uint32_t sub) {
  Stream s;
  s.k0 = k0; s.k1 = k1; s.rep = rep; s.station = station; s.step0 = step0;
  s.hi = sub << 24; s.block = 0; s.left = 0;
  s.b0 = s.b1 = s.b2 = s.b3 = 0;
  return s;
}

__device__ __forceinline__ uint32_t draw_u32(Stream &s, uint32_t &flags) {
  if (s.left == 0) {
    if (s.block >= kBlockLimit) { flags |= 1u; s.block = 0; }
    const U4 o = philox10(U4{s.rep, s.station, s.step0, s.hi | s.block}, s.k0, s.k1);
    s.b0 = o.x; s.b1 = o.y; s.b2 = o.z; s.b3 = o.w;
    s.block += 1;
    s.left = 4;
  }
  const uint32_t v = s.b0;
  s.b0 = s.b1; s.b1 = s.b2; s.b2 = s.b3;
  s.left -= 1;
  return v;
}

// (2 * (x >> 9) + 1) * 2^-24: exact, never 0 or 1.  Formed as (1 + (x >> 9) 2^-23) - (1 - 2^-24):
// the first is the float with those mantissa bits, and the subtraction is exact (Sterbenz: both
// lie in [1/2, 2], within a factor 2 of each other), so this is the same value in three
// instructions instead of four.
__device__ __forceinline__ float to_unit(uint32_t x) {
  return __uint_as_float((x >> 9) | 0x3F800000u) - 0x1.fffffep-1f;
}

__device__ __forceinline__ float draw_unit(Stream &s, uint32_t &flags) {
  return to_unit(draw_u32(s, flags));
}

// ------------------------------------------------------------------------------------
// fp32 log / log1p / exp / expm1 from their series (Taylor coefficients rounded to fp32),
// with Cody-Waite reduction by ln 2 = LN2_HI (12 significant bits) + LN2_LO.
// ------------------------------------------------------------------------------------
constexpr float LN2_HI = 0x1.62ep-1f;
constexpr float LN2_LO = 0x1.0bfbe8p-15f;
constexpr float INV_LN2 = 0x1.715476p+0f;
constexpr float HALF_LN2 = 0x1.62e43p-2f;
constexpr float HALF_LOG_2PI = 0x1.d67f1cp-1f;

__device__ __forceinline__ float fma32(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// z * (2/3 + 2z/5 + 2z^2/7 + 2z^3/9 + 2z^4/11): 2 atanh(s) = 2s + s * this, z = s^2.
__device__ __forceinline__ float atanh_tail(float z) {
  float p = 0x1.745d18p-3f;
  p = fma32(p, z, 0x1.c71c72p-3f);
  p = fma32(p, z, 0x1.24924ap-2f);
  p = fma32(p, z, 0x1.99999ap-2f);
  p = fma32(p, z, 0x1.555556p-1f);
  return z * p;
}

// ln(1+f) = f - (h - s (h + R)),  s = f/(2+f),  h = f^2/2;  `lo` joins at the inner sum.
__device__ __forceinline__ float ln1p_small(float f, float lo) {
  const float s = f / (2.0f + f);
  const float R = atanh_tail(s * s);
  const float h = (0.5f * f) * f;
  return f - (h - fma32(s, h + R, lo));
}

// ln(u) + corr, u positive normal: u = 2^e (1+f), 1+f in (sqrt(2)/2, sqrt(2)].
__device__ __forceinline__ float ln_corr(float u, float corr) {
  const uint32_t b = __float_as_uint(u);
  int e = (int)(b >> 23) - 127;
  uint32_t mb = (b & 0x007FFFFFu) | 0x3F800000u;
  if (mb > 0x3FB504F3u) { mb -= 0x00800000u; e += 1; }
  const float f = __uint_as_float(mb) - 1.0f;
  const float ef = (float)e;
  return fma32(ef, LN2_HI, ln1p_small(f, fma32(ef, LN2_LO, corr)));
}

__device__ __forceinline__ float ln(float x) { return ln_corr(x, 0.0f); }

__device__ __forceinline__ float ln1p(float x) {
  if (fabsf(x) < 0.25f) return ln1p_small(x, 0.0f);
  const float u = 1.0f + x;
  const float c = (x < 1.0f) ? x - (u - 1.0f) : 1.0f - (u - x);   // exact rounding error of 1+x
  return ln_corr(u, c / u);
}

// e^r, |r| <= ln2/2: Taylor through r^7/7!.
__device__ __forceinline__ float exp_small(float r) {
  float p = 0x1.a01a02p-13f;
  p = fma32(p, r, 0x1.6c16c2p-10f);
  p = fma32(p, r, 0x1.111112p-7f);
  p = fma32(p, r, 0x1.555556p-5f);
  p = fma32(p, r, 0x1.555556p-3f);
  p = fma32(p, r, 0.5f);
  p = fma32(p, r, 1.0f);
  p = fma32(p, r, 1.0f);
  return p;
}

// e^x; 0 below -86 (never needed: only probabilities well above underflow use it).
__device__ __forceinline__ float ex(float x) {
  if (x < -86.0f) return 0.0f;
  if (x > 88.0f) return __builtin_huge_valf();
  const float k = __builtin_rintf(x * INV_LN2);
  float r = fma32(-k, LN2_HI, x);
  r = fma32(-k, LN2_LO, r);
  return exp_small(r) * __uint_as_float((uint32_t)((int)k + 127) << 23);
}

// e^r - 1, |r| <= ln2/2: r + r^2 (1/2 + r/3! + ... + r^6/8!).
__device__ __forceinline__ float expm1_small(float r) {
  float p = 0x1.a01a02p-16f;
  p = fma32(p, r, 0x1.a01a02p-13f);
  p = fma32(p, r, 0x1.6c16c2p-10f);
  p = fma32(p, r, 0x1.111112p-7f);
  p = fma32(p, r, 0x1.555556p-5f);
  p = fma32(p, r, 0x1.555556p-3f);
  p = fma32(p, r, 0.5f);
  return fma32(r * r, p, r);
}

__device__ __forceinline__ float exm1(float x) {
  if (fabsf(x) < HALF_LN2) return expm1_small(x);
  if (x < -16.0f || x > 16.0f) return ex(x) - 1.0f;
  const float k = __builtin_rintf(x * INV_LN2);
  float r = fma32(-k, LN2_HI, x);
  r = fma32(-k, LN2_LO, r);
  const float two_k = __uint_as_float((uint32_t)((int)k + 127) << 23);
  return fma32(two_k, expm1_small(r), two_k - 1.0f);   // 2^k (e^r - 1) + (2^k - 1)
}

// Servers of station s during interval step0 + 1 under a staffing schedule (segment of the
// interval, then the segment's servers), or the station's constant servers c.
__device__ __forceinline__ int servers_in(const int *segidx, const int *seg_m, int n, int s, int step0, int c) {
  return segidx ? seg_m[(long long)segidx[step0] * n + s] : c;
}

__device__ __forceinline__ float rate_in(const int *segidx, const float *seg_rate, int n, int s, int step0,
                                         float rate) {
  return segidx ? seg_rate[(long long)segidx[step0] * n + s] : rate;
}

// ------------------------------------------------------------------------------------
// Sampler tables (uploaded by the host at initialisation):
//   c_rcp[i] = fp32(1/(i+1)), i = 0..255 (16-byte aligned, read four at a time);
//   c_fc[j]  = ln j! - ((j + 1/2) ln(j+1) - (j+1) + ln(2 pi)/2), j = 0..9 (fp64 -> fp32).
// ------------------------------------------------------------------------------------
constexpr int kRcpTab = 256;
constexpr int kPoisInvMax = 63;      // Poisson inversion (lam < 10) stops at k = 63
constexpr int kBinomInvMax = 255;    // binomial inversion (n p < 80) stops at k = 255
// n p below this: inversion, else BTRS.  Both are exact samplers; the switch sits where a
// wavefront's cost of the two meets: inversion runs to its slowest lane's k, about n p +
// 2.4 sqrt(n p) steps over 64 lanes, and BTRS to its slowest lane's attempt, with the
// logarithmic test taken in nearly every attempt by some lane.
constexpr float kBinomInvNp = 80.0f;
extern __constant__ float4 c_rcp4[kRcpTab / 4];
extern __constant__ float c_fc[10];

__device__ __forceinline__ float rcp_tab(int k) {   // fp32(1/k), 1 <= k <= 256
  return reinterpret_cast<const float *>(c_rcp4)[k - 1];
}

// Remainder of Stirling's series for ln j!: table below 10, else 1/12a - 1/360a^3 + 1/1260a^5.
__device__ __forceinline__ float stirling_tail(int j) {
  if (j < 10) return c_fc[j];
  const float a = (float)j + 1.0f;
  const float ia = 1.0f / a;
  const float ia2 = ia * ia;
  float t = 0x1.a01a02p-11f;
  t = 0x1.6c16c2p-9f - ia2 * t;
  t = 0x1.555556p-4f - ia2 * t;
  return ia * t;
}

constexpr int kRejectCap = 100000;

// Poisson(lam): inversion by sequential search below 10 (one uniform), else PTRS
// (Hormann 1993, transformed rejection with squeeze, two uniforms per attempt).
__device__ __forceinline__ int poisson(float lam, Stream &S, uint32_t &flags) {
  if (!(lam > 0.0f)) return 0;
  if (lam < 10.0f) {
    float p = ex(-lam);
    float F = p;
    const float u = draw_unit(S, flags);
    int k = 0;
    while (u > F && k < kPoisInvMax) {
      k += 1;
      p = p * (lam * rcp_tab(k));
      const float Fn = F + p;
      if (Fn == F) break;
      F = Fn;
    }
    return k;
  }
  if (lam >= 0x1p24f) flags |= 4u;   // values beyond exact fp32 integers
  const float slam = __builtin_sqrtf(lam);
  const float loglam = ln(lam);
  const float b = 0.931f + 2.53f * slam;
  const float a = -0.059f + 0.02483f * b;
  const float two_a = 2.0f * a;
  const float invalpha = 1.1239f + 1.1328f / (b - 3.4f);
  const float vr = 0.9277f - 3.6224f / (b - 2.0f);
  for (int it = 0; it < kRejectCap; ++it) {
    const float U = draw_unit(S, flags) - 0.5f;
    const float V = draw_unit(S, flags);
    const float us = 0.5f - fabsf(U);
    const float kf = __builtin_floorf((two_a / us + b) * U + (lam + 0.43f));
    if (us >= 0.07f && V <= vr) return (int)kf;
    if (kf < 0.0f || (us < 0.013f && V > us)) continue;
    const float lhs = ln(V * invalpha / (a / (us * us) + b));
    const float t = (kf + 1.0f) - lam;
    const float rhs = t - (kf + 0.5f) * ln1p(t / lam) - 0.5f * loglam - HALF_LOG_2PI -
                      stirling_tail((int)kf);
    if (lhs <= rhs) return (int)kf;
  }
  flags |= 2u;
  return (int)__builtin_floorf(lam);
}

// Binomial(n, p), n p < 80, 0 < p <= 1/2: inversion from 0 with the pmf recurrence
// f_k = f_{k-1} ((n+1) r / k - r), r = p/q, the factor one fma of g = (n+1) r and the fp32
// reciprocal of k, f_0 = e^{n lq}, lq = ln(1 - p), at most 255 steps
// (P(X > 255) < 1e-40).  f_0 is formed as ex() forms it, exp(r) 2^e with n lq = e ln 2 + r, but
// with the binary exponent raised by sc = -120 - e when e < -120 (f_0 below the normal fp32
// range; n lq > -111 here), and the uniform raised by the same 2^sc: scaling by a power of two is
// exact, so every step and comparison is the one an fp32 without the lower exponent limit
// makes (sc = 0 for n p < 56, where f_0 >= e^-78 is normal anyway).  Every lane still searching
// is at the same k, so a pass takes four steps with one scalar load of their four
// reciprocals; a lane stops at exactly the step the one-step search stops at.
__device__ __forceinline__ int binom_inv(int n, float r, float lq, Stream &S, uint32_t &flags) {
  const float g = r * ((float)n + 1.0f);
  const float x = (float)n * lq;
  const float ek = __builtin_rintf(x * INV_LN2);
  float rr = fma32(-ek, LN2_HI, x);
  rr = fma32(-ek, LN2_LO, rr);
  const int e = (int)ek;
  const int sc = e < -120 ? -120 - e : 0;
  float f = exp_small(rr) * __uint_as_float((uint32_t)(e + sc + 127) << 23);   // P(X = 0) 2^sc
  float F = f;
  const float u = draw_unit(S, flags) * __uint_as_float((uint32_t)(sc + 127) << 23);
  const int kmax = n < kBinomInvMax ? n : kBinomInvMax;
  int k = 0;
  bool go = u > F && 0 < kmax;
  for (int base = 0; go; base += 4) {
    const float4 iv = c_rcp4[base >> 2];
    const float ivs[4] = {iv.x, iv.y, iv.z, iv.w};
    // The k < kmax test binds at the step k = kmax, inside this pass (steps base+1..base+4)
    // only for a searching lane with kmax <= base + 4; without one, the test is left out.
    if (__builtin_amdgcn_ballot_w64(go && kmax <= base + 4) == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // No branches: a lane that has stopped keeps only its k; its f and F run on unused.
        const float fn = f * fma32(g, ivs[j], -r);
        const float Fn = F + fn;
        k += go ? 1 : 0;   // a searching lane is at k = base + j
        go = go && Fn != F && u > Fn;   // Fn == F: the pmf no longer moves the sum
        f = fn;
        F = Fn;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float fn = f * fma32(g, ivs[j], -r);
        const float Fn = F + fn;
        const int kj = base + j + 1;
        k += go ? 1 : 0;
        go = go && Fn != F && u > Fn && kj < kmax;
        f = fn;
        F = Fn;
      }
    }
  }
  return k;
}

// Binomial(n, p), n p >= 80, p <= 1/2: BTRS (Hormann 1993), acceptance against
// ln f(k)/f(mode) from Stirling's series.
__device__ __forceinline__ int binom_btrs(int n, float p, float r, Stream &S, uint32_t &flags) {
  const float nf = (float)n;
  const float q = 1.0f - p;
  const float spq = __builtin_sqrtf(nf * p * q);
  const float b = 1.15f + 2.53f * spq;
  const float a = -0.0873f + 0.0248f * b + 0.01f * p;
  const float two_a = 2.0f * a;
  const float c = nf * p + 0.5f;
  const float alpha = (2.83f + 5.1f / b) * spq;
  const float vr = 0.92f - 4.2f / b;
  const float mf = __builtin_floorf((nf + 1.0f) * p);
  const int m = (int)mf;
  const float nm = nf - mf + 1.0f;
  // ln((m+1)/(r nm)) as ln1p((m + 1 - r nm)/(r nm)).  For a large mode the ratio is near 1, and
  // rounding it before the log, times m + 1/2, would swamp the log-ratio; so the difference is
  // one fp64 fma of exact integers (below 2^28, times the fp32 r: an exact product), rounded
  // once (likewise ln(nk r/(k+1)) below)
  const float rnm = r * nm;
  const float dm = (float)__builtin_fma(-(double)r, (double)(n - m + 1), (double)(m + 1));
  const float hm = (mf + 0.5f) * ln1p(dm / rnm) + stirling_tail(m) + stirling_tail(n - m);
  if (m >= (1 << 24)) flags |= 4u;   // a mode beyond exact fp32 integers
  for (int it = 0; it < kRejectCap; ++it) {
    const float u = draw_unit(S, flags) - 0.5f;
    const float v = draw_unit(S, flags);
    const float us = 0.5f - fabsf(u);
    const float kf = __builtin_floorf((two_a / us + b) * u + c);
    if (us >= 0.07f && v <= vr) return (int)kf;
    if (kf < 0.0f || kf > nf) continue;
    const int k = (int)kf;
    if (k > n) continue;   // nf may round n up when n >= 2^24
    const float lhs = ln(v * alpha / (a / (us * us) + b));
    const float nk = nf - kf + 1.0f;
    const float rhs = hm + (nf + 1.0f) * ln1p((kf - mf) / nk) +
                      (kf + 0.5f) * ln1p((float)__builtin_fma((double)r, (double)(n - k + 1), -(double)(k + 1)) /
                                         (kf + 1.0f)) - stirling_tail(k) -
                      stirling_tail(n - k);
    if (lhs <= rhs) return k;
  }
  flags |= 2u;
  return m;
}

// The constants of Binomial(., p) that depend on p alone (BinomP).  Per-edge and per-station
// copies are made once per network by a kernel with these same functions, so a draw with
// precomputed constants is the draw with constants computed in place.
__device__ __forceinline__ BinomP binom_prep(float p) {
  BinomP b;
  b.flip = p > 0.5f ? 1 : 0;
  b.ph = !(p > 0.0f) || p >= 1.0f ? 0.0f : (p > 0.5f ? 1.0f - p : p);
  const float q = 1.0f - b.ph;
  b.r = b.ph / q;
  b.lq = ln1p(-b.ph);
  return b;
}

__device__ __forceinline__ int binomial_c(int n, const BinomP &b, Stream &S, uint32_t &flags) {
  if (n <= 0) return 0;
  int k = 0;
  if (b.ph > 0.0f)
    k = ((float)n * b.ph < kBinomInvNp) ? binom_inv(n, b.r, b.lq, S, flags)
                                        : binom_btrs(n, b.ph, b.r, S, flags);
  return b.flip ? n - k : k;
}

// Binomial(n, p) with the constants computed in place; lq only where inversion needs it.
__device__ __forceinline__ int binomial(int n, float p, Stream &S, uint32_t &flags) {
  if (n <= 0 || !(p > 0.0f)) return 0;
  if (p >= 1.0f) return n;
  const float ph = p > 0.5f ? 1.0f - p : p;
  const float q = 1.0f - ph;
  const float r = ph / q;
  const int k = ((float)n * ph < kBinomInvNp) ? binom_inv(n, r, ln1p(-ph), S, flags)
                                              : binom_btrs(n, ph, r, S, flags);
  return p > 0.5f ? n - k : k;
}

// Gamma(k, 1), integer k >= 1: Marsaglia & Tsang (2000); normals by Marsaglia's polar
// method, second normal of each pair unused.
__device__ __forceinline__ float gamma_int(int k, Stream &S, uint32_t &flags) {
  const float d = (float)k - 0x1.555556p-2f;
  const float c = 1.0f / __builtin_sqrtf(9.0f * d);
  for (int it = 0; it < kRejectCap; ++it) {
    float x1, s;
    do {
      x1 = 2.0f * draw_unit(S, flags) - 1.0f;
      const float x2 = 2.0f * draw_unit(S, flags) - 1.0f;
      s = x1 * x1 + x2 * x2;
    } while (s >= 1.0f);
    const float z = x1 * __builtin_sqrtf(-2.0f * ln(s) / s);
    const float t = 1.0f + c * z;
    if (t <= 0.0f) continue;
    const float v = t * t * t;
    const float u = draw_unit(S, flags);
    const float z2 = z * z;
    if (u < 1.0f - 0.0331f * (z2 * z2)) return d * v;
    if (ln(u) < 0.5f * z2 + d * ((1.0f - v) + ln(v))) return d * v;
  }
  flags |= 2u;
  return d;
}

// GenerateDeparture (Lemma 1, Algorithm 3), written as offset + Binomial(n_b, p_b) so that a
// wavefront takes a single binomial call whatever branch each lane is in:
//   x <= m:            Binomial(x, pdep)
//   x > m, T > dt:     Binomial(x-m-1, dt/T)            T = Gamma(x-m)/(m mu)
//   x > m, T <= dt:    x-m + Binomial(m, 1 - e^{-mu (dt-T)})
// `dep` holds the constants of Binomial(., pdep), pdep = 1 - e^{-mu dt}.
__device__ __forceinline__ int gendep(int x, int m, float mu, float dt, const BinomP &dep, float rate,
                                      Stream &S, uint32_t &flags) {
  if (x <= 0) return 0;
  int nb = x, off = 0;
  BinomP bp = dep;
  if (x > m) {
    const int k = x - m;
    const float T = gamma_int(k, S, flags) / rate;
    float pb;
    if (T > dt) {
      nb = k - 1;
      pb = dt / T;
    } else {
      nb = m;
      off = k;
      pb = -exm1(-(mu * (dt - T)));
    }
    bp = binom_prep(pb);
  }
  return off + binomial_c(nb, bp, S, flags);
}

// Naive departures, Eq. (1): min(x, Poisson(min(x, m) mu dt)).
__device__ __forceinline__ int gendep_naive(int x, int m, float mudt, Stream &S, uint32_t &flags) {
  if (x <= 0) return 0;
  const int b = x < m ? x : m;
  const int s = poisson((float)b * mudt, S, flags);
  return s < x ? s : x;
}

// GenerateDeparture with the likelihood-ratio score of the draw in mu: the mu-derivative
// of the log-density of the variables it consumed.  Binomial branch (x <= m):
// D kap - (x - D) dt with kap = dt e^{-mu dt} / (1 - e^{-mu dt}).  x > m: the Erlang(k, m mu)
// time gives k/mu - m T; the split when T > dt does not depend on mu; when T <= dt the
// completions D' ~ Binomial(m, p2), p2 = 1 - e^{-mu s}, s = dt - T, add
// -(m - D') s + D' s (1 - p2) / p2.  Draws are the ones gendep makes, in the same order.
__device__ __forceinline__ int gendep_score(int x, int m, float mu, float dt, const BinomP &dep, float rate,
                                            float kap, Stream &S, uint32_t &flags, float &score) {
  score = 0.0f;
  if (x <= 0) return 0;
  int nb = x, off = 0, branch = 0;
  float pb = 0.0f, sc = 0.0f, s = 0.0f;
  BinomP bp = dep;
  if (x > m) {
    const int k = x - m;
    const float T = gamma_int(k, S, flags) / rate;
    sc = (float)k / mu - (float)m * T;
    if (T > dt) {
      nb = k - 1;
      pb = dt / T;
      branch = 1;
    } else {
      nb = m;
      off = k;
      s = dt - T;
      pb = -exm1(-(mu * s));
      branch = 2;
    }
    bp = binom_prep(pb);
  }
  const int B = binomial_c(nb, bp, S, flags);
  if (branch == 0) {
    sc = (float)B * kap - (float)(x - B) * dt;
  } else if (branch == 2) {
    sc = sc - (float)(m - B) * s;
    if (B > 0) sc = sc + (float)B * (s * (1.0f - pb) / pb);
  }
  score = sc;
  return off + B;
}

// Naive departures with the score of the Poisson draw S in mu: S/mu - min(x, m) dt.
__device__ __forceinline__ int gendep_naive_score(int x, int m, float mudt, float mu, float dt, Stream &S,
                                                  uint32_t &flags, float &score) {
  score = 0.0f;
  if (x <= 0) return 0;
  const int b = x < m ? x : m;
  const int s = poisson((float)b * mudt, S, flags);
  score = (float)s / mu - (float)b * dt;
  return s < x ? s : x;
}

}  // namespace eq
