// Shared device/host definitions of the shtx HIP library (gfx950).
//
// Notation: N = nside, L = lmax (= mmax), R = 4N-1 rings, Rp = 2N ring pairs.
// Ring pair p (0-based) joins north ring i = p+1 and south ring 4N-i (1-based
// ring numbers); p = 2N-1 is the equator, paired with itself.  Both rings of
// a pair have the same length n = 4*min(i, N) and the same first-pixel
// longitude phi0, and z_south = -z_north, which is what the north/south parity
// fold of the Legendre step (lambda_lm(-z) = (-1)^(l+m) lambda_lm(z), Eq. (15))
// relies on.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace shtx {

// l-recurrences start on l = m + kAlign*j; seeds are stored at such l.
constexpr int kAlign = 8;
// Largest supported nside (ring FFT of 4*nside points must fit in LDS).
constexpr int kMaxNside = 2048;
// A ring's Legendre term is skipped until |mu_lm| first reaches 2^kSkipExp.
constexpr int kSkipExp = -64;

__host__ __device__ inline size_t alm_idx(int l, int m, int lmax) {
  return (size_t)m * (size_t)(2 * lmax + 1 - m) / 2 + (size_t)l;
}
__host__ __device__ inline size_t nalm_of(int lmax) {
  return (size_t)(lmax + 1) * (size_t)(lmax + 2) / 2;
}
// Offset of the root table of ring length n = 4i (i = 1..N) inside the
// concatenated table: sum_{j<i} 4j.
__host__ __device__ inline size_t roots_offset(int i) {
  return (size_t)2 * (size_t)i * (size_t)(i - 1);
}

// Byte offsets of the pieces of the resident table buffer.
struct TableOffsets {
  size_t rp_n, rp_sN, rp_sS, rp_p0n, rp_p0d;  // int32 [Rp]
  size_t rp_z, rp_sth, rp_w;                  // double [Rp]
  size_t coefA, coefC;                        // double [nalm]
  size_t seed_l;                              // int32 [(L+1) * Rp]
  size_t seed_v;                              // double2 [(L+1) * Rp]
  size_t roots64;                             // double2 [2N(N+1)]
  size_t roots32;                             // float2  [2N(N+1)]
  size_t total;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline TableOffsets table_offsets(int nside, int lmax) {
  TableOffsets o{};
  const size_t Rp = 2 * (size_t)nside;
  const size_t nalm = nalm_of(lmax);
  const size_t nroots = roots_offset(nside + 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t here = off;
    off = align_up(off + bytes, 256);
    return here;
  };
  o.rp_n = take(Rp * 4);
  o.rp_sN = take(Rp * 4);
  o.rp_sS = take(Rp * 4);
  o.rp_p0n = take(Rp * 4);
  o.rp_p0d = take(Rp * 4);
  o.rp_z = take(Rp * 8);
  o.rp_sth = take(Rp * 8);
  o.rp_w = take(Rp * 8);
  o.coefA = take(nalm * 8);
  o.coefC = take(nalm * 8);
  o.seed_l = take((size_t)(lmax + 1) * Rp * 4);
  o.seed_v = take((size_t)(lmax + 1) * Rp * 16);
  o.roots64 = take(nroots * 16);
  o.roots32 = take(nroots * 8);
  o.total = off;
  return o;
}

struct Tables {
  int nside, lmax, npairs, npix;
  const int *rp_n, *rp_sN, *rp_sS, *rp_p0n, *rp_p0d;
  const double *rp_z, *rp_sth, *rp_w;
  const double *coefA, *coefC;
  const int *seed_l;
  const double2 *seed_v;
  const double2 *roots64;
  const float2 *roots32;
};

inline Tables tables_view(const void *base, int nside, int lmax) {
  const TableOffsets o = table_offsets(nside, lmax);
  const char *b = static_cast<const char *>(base);
  Tables t;
  t.nside = nside;
  t.lmax = lmax;
  t.npairs = 2 * nside;
  t.npix = 12 * nside * nside;
  t.rp_n = reinterpret_cast<const int *>(b + o.rp_n);
  t.rp_sN = reinterpret_cast<const int *>(b + o.rp_sN);
  t.rp_sS = reinterpret_cast<const int *>(b + o.rp_sS);
  t.rp_p0n = reinterpret_cast<const int *>(b + o.rp_p0n);
  t.rp_p0d = reinterpret_cast<const int *>(b + o.rp_p0d);
  t.rp_z = reinterpret_cast<const double *>(b + o.rp_z);
  t.rp_sth = reinterpret_cast<const double *>(b + o.rp_sth);
  t.rp_w = reinterpret_cast<const double *>(b + o.rp_w);
  t.coefA = reinterpret_cast<const double *>(b + o.coefA);
  t.coefC = reinterpret_cast<const double *>(b + o.coefC);
  t.seed_l = reinterpret_cast<const int *>(b + o.seed_l);
  t.seed_v = reinterpret_cast<const double2 *>(b + o.seed_v);
  t.roots64 = reinterpret_cast<const double2 *>(b + o.roots64);
  t.roots32 = reinterpret_cast<const float2 *>(b + o.roots32);
  return t;
}

// ---------------------------------------------------------------- complex
template <typename T> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename C> __device__ __forceinline__ C cmk(decltype(C{}.x) a, decltype(C{}.x) b) {
  C r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }

// Root table of the compute precision.
template <typename T> __device__ __forceinline__ const cplx<T> *roots_of(const Tables &t);
template <> __device__ __forceinline__ const float2 *roots_of<float>(const Tables &t) { return t.roots32; }
template <> __device__ __forceinline__ const double2 *roots_of<double>(const Tables &t) { return t.roots64; }

// exp(sign * i * pi * red / den) for an exactly reduced integer red in
// [0, 2*den), evaluated in the compute precision.
template <typename T> __device__ __forceinline__ cplx<T> phase_pi(int red, int den, T sign);
template <> __device__ __forceinline__ float2 phase_pi<float>(int red, int den, float sign) {
  float s, c;
  sincospif((float)red / (float)den, &s, &c);
  return make_float2(c, sign * s);
}
template <> __device__ __forceinline__ double2 phase_pi<double>(int red, int den, double sign) {
  double s, c;
  sincospi((double)red / (double)den, &s, &c);
  return make_double2(c, sign * s);
}

// Scalar element conversions for maps (bf16 stored as raw uint16).
struct bf16_t {
  uint16_t bits;
};
__device__ __forceinline__ float to_float(float v) { return v; }
__device__ __forceinline__ double to_double(double v) { return v; }
template <typename T, typename S> __device__ __forceinline__ T load_as(const S *p);
template <> __device__ __forceinline__ float load_as<float, float>(const float *p) { return *p; }
template <> __device__ __forceinline__ double load_as<double, double>(const double *p) { return *p; }
template <> __device__ __forceinline__ float load_as<float, bf16_t>(const bf16_t *p) {
  return __uint_as_float(((uint32_t)p->bits) << 16);
}
template <typename S, typename T> __device__ __forceinline__ void store_as(S *p, T v);
template <> __device__ __forceinline__ void store_as<float, float>(float *p, float v) { *p = v; }
template <> __device__ __forceinline__ void store_as<double, double>(double *p, double v) { *p = v; }
template <> __device__ __forceinline__ void store_as<bf16_t, float>(bf16_t *p, float v) {
  // round to nearest even
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    p->bits = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    return;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  p->bits = (uint16_t)(u >> 16);
}

}  // namespace shtx
