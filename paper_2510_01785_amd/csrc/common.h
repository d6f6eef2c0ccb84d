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
// Analysis on the matrix cores: a workgroup takes one (m, block of kBlockL
// consecutive l) item and starts every ring from a stored checkpoint of the
// recurrence at the block start.  Checkpoints are kept for nside <= this.
constexpr int kBlockL = 128;
constexpr int kMaxNsideCheckpoint = 2048;

inline size_t checkpoint_items(int nside, int lmax) {
  if (nside > kMaxNsideCheckpoint) return 0;
  size_t I = 0;
  for (int m = 0; m <= lmax; ++m) I += (size_t)((lmax - m + kBlockL) / kBlockL);
  return I;
}

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

// Ring lengths n = 4i whose odd part has a prime factor above this are
// transformed with Bluestein's chirp-z algorithm (Eq. (17)-(23)) on a
// power-of-two length; the others with mixed radix 4/2/3/5/7/11/13.
constexpr int kMaxDirectPrime = 13;

__host__ __device__ inline int largest_odd_prime(int i) {
  while ((i & 1) == 0 && i > 0) i >>= 1;
  int big = 1;
  for (int f = 3; f * f <= i; f += 2)
    while (i % f == 0) {
      big = f;
      i /= f;
    }
  if (i > 1) big = i > big ? i : big;
  return big;
}

// Bluestein convolution length for ring length 4i, or 0 for mixed radix.
// Such a ring is transformed as four DFTs of length i (its samples 4j + q,
// q = 0..3) combined by one radix-4 step; each length-i DFT is a cyclic
// convolution of length M >= 2i - 1.
__host__ __device__ inline int bluestein_len(int i) {
  if (largest_odd_prime(i) <= kMaxDirectPrime) return 0;
  const int need = 2 * i - 1;
  int M = 1;
  while (M < need) M <<= 1;
  return M;
}

// Sum of Bluestein lengths of cap rings 1..nside-1 and their maximum.
inline void bluestein_sizes(int nside, size_t *total, int *mmax) {
  size_t t = 0;
  int mx = 0;
  for (int i = 1; i < nside; ++i) {
    const int M = bluestein_len(i);
    t += (size_t)M;
    mx = M > mx ? M : mx;
  }
  *total = t;
  *mmax = mx;
}

// Ring FFT launch geometry (ring_fft.hip): workgroup size NT, channels per
// workgroup G (the channel slice of a ring pair), LDS bytes, offset of the
// twiddle table in LDS and how many of a Bluestein ring's four
// sub-transforms share one FFT call (4 or 1).
struct FftGeom {
  int NT, G, tq_off, bs_nb;
  size_t lds;
};
FftGeom fft_geometry(int nside, int mmax_bs, int batch, size_t csize);

// Layout of the synthesis spectra g_m (Legendre output, ring FFT input):
// element (p, c, m) at ((p ns + c/G) M + m) G + c%G, slices of G channels.
// Used with one slice of all channels (G = batch, ns = 1): [p][m][batch], so
// the synthesis Legendre kernels write whole rows of channels (128-byte lines
// at 16 FP32 channels) and the ring FFT's channel slices of one ring pair read
// parts of the same rows close in time.
struct SynLayout {
  int G, ns, M;
  __host__ __device__ size_t idx(int p, int c, int m) const {
    return (((size_t)p * ns + c / G) * M + m) * G + c % G;
  }
  __host__ __device__ size_t size(int npairs) const { return (size_t)npairs * ns * M * G; }
};
inline SynLayout syn_layout(int nside, int lmax, int mmax_bs, int batch, size_t csize) {
  (void)nside;
  (void)mmax_bs;
  (void)csize;
  return SynLayout{batch, 1, lmax + 1};
}

// Readable doubles after the last coefficient (recurrence kernels load
// groups of 8 coefficients without clamping at lmax; the values loaded past
// lmax only meet masked terms).
constexpr size_t kCoefPad = 8;
// Channel groups of the synthesis coefficient buffer ALMT (written by the
// input layout kernel, read by the synthesis Legendre kernels): channels
// [g0, g0 + w) are stored as [idx][w] from complex offset g0 (nalm +
// kCoefPad).  gmax = batch gives one group, the plain [idx][batch] layout of
// the matrix-core kernel; gmax = 4 or 2 (vector-ALU kernels) gives full groups
// of gmax, then one of 2 (if two or three channels remain with gmax = 4) and
// one of 1, the channel groups those kernels are launched on.
struct ChanGroup {
  int g0, w;
};
__host__ __device__ inline ChanGroup chan_group(int b, int batch, int gmax) {
  const int nfull = batch / gmax * gmax;
  if (b < nfull) return ChanGroup{b / gmax * gmax, gmax};
  if (batch - nfull >= 2 && b < nfull + 2) return ChanGroup{nfull, 2};
  return ChanGroup{batch - 1, 1};
}

// Zero doubles after the last recurrence coefficient in the table buffer: the
// analysis kernels load the coefficients of a whole 128-l block, and the 8
// after it ahead of time, without clamping at lmax (rows past lmax are never
// stored).
constexpr size_t kCoefPadTable = kBlockL + 8;

// Byte offsets of the pieces of the resident table buffer.
struct TableOffsets {
  size_t rp_n, rp_sN, rp_sS, rp_p0n, rp_p0d;  // int32 [Rp]
  size_t rp_M, rp_bsoff;                      // int32 [Rp]: Bluestein length (0: mixed radix), offset
  size_t rp_z, rp_sth, rp_w;                  // double [Rp]
  size_t coefA, coefC;                        // double [nalm + kCoefPadTable], zero padding
  size_t seed_l;                              // int32 [(L+1) * Rp]
  size_t seed_v;                              // double2 [(L+1) * Rp]
  size_t roots64;                             // double2 [2N(N+1)]  per ring length 4i
  size_t roots32;                             // float2  [2N(N+1)]
  size_t chirp64, chirp32;                    // Bluestein chirps, same layout as roots
  size_t bhat64, bhat32, bhat_tmp;            // FFT of the conjugate chirp, [sum M_i]
  size_t rootsP64, rootsP32;                  // roots of the largest Bluestein length
  size_t ck_items;                            // int2 [I]: (m, l0) of each analysis block, XCD-major
  size_t ck_xoff;                             // int32 [9]: first item of each XCD
  size_t ck_pos;                              // int32 [L+1]: item index of (m, l0 = m)
  size_t ck_t;                                // uint8 [I * Rp]: start offset in block (kBlockL: idle)
  size_t ck_v;                                // double2 [I * Rp]: (mu_{l-1}, mu_l) at that start
  size_t r2n;                                 // uint32 [Npix]: NESTED index of each RING pixel
  size_t total;
  size_t nitems;
  size_t nbhat;
  int mmax_bs;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline TableOffsets table_offsets(int nside, int lmax) {
  TableOffsets o{};
  const size_t Rp = 2 * (size_t)nside;
  const size_t nalm = nalm_of(lmax);
  const size_t nroots = roots_offset(nside + 1);
  bluestein_sizes(nside, &o.nbhat, &o.mmax_bs);
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
  o.rp_M = take(Rp * 4);
  o.rp_bsoff = take(Rp * 4);
  o.rp_z = take(Rp * 8);
  o.rp_sth = take(Rp * 8);
  o.rp_w = take(Rp * 8);
  o.coefA = take((nalm + kCoefPadTable) * 8);
  o.coefC = take((nalm + kCoefPadTable) * 8);
  o.seed_l = take((size_t)(lmax + 1) * Rp * 4);
  o.seed_v = take((size_t)(lmax + 1) * Rp * 16);
  o.roots64 = take(nroots * 16);
  o.roots32 = take(nroots * 8);
  o.chirp64 = take(nroots * 16);
  o.chirp32 = take(nroots * 8);
  o.bhat64 = take(o.nbhat * 16);
  o.bhat32 = take(o.nbhat * 8);
  o.bhat_tmp = take(o.nbhat * 16);
  o.rootsP64 = take((size_t)o.mmax_bs * 16);
  o.rootsP32 = take((size_t)o.mmax_bs * 8);
  o.nitems = checkpoint_items(nside, lmax);
  o.ck_items = take(o.nitems * 8);
  o.ck_xoff = take(9 * 4);
  o.ck_pos = take((size_t)(lmax + 1) * 4);
  o.ck_t = take(o.nitems * Rp);
  o.ck_v = take(o.nitems * Rp * 16);
  o.r2n = take(12 * (size_t)nside * (size_t)nside * 4);
  o.total = off;
  return o;
}

struct Tables {
  int nside, lmax, npairs, npix, mmax_bs, nitems;
  const int *rp_n, *rp_sN, *rp_sS, *rp_p0n, *rp_p0d, *rp_M, *rp_bsoff;
  const double *rp_z, *rp_sth, *rp_w;
  const double *coefA, *coefC;
  const int *seed_l;
  const double2 *seed_v;
  const double2 *roots64;
  const float2 *roots32;
  const double2 *chirp64, *bhat64, *rootsP64;
  const float2 *chirp32, *bhat32, *rootsP32;
  const int2 *ck_items;
  const int *ck_xoff, *ck_pos;
  const uint8_t *ck_t;
  const double2 *ck_v;
  const uint32_t *r2n;
};

inline Tables tables_view(const void *base, int nside, int lmax) {
  const TableOffsets o = table_offsets(nside, lmax);
  const char *b = static_cast<const char *>(base);
  Tables t;
  t.nside = nside;
  t.lmax = lmax;
  t.npairs = 2 * nside;
  t.npix = 12 * nside * nside;
  t.mmax_bs = o.mmax_bs;
  t.nitems = (int)o.nitems;
  t.rp_n = reinterpret_cast<const int *>(b + o.rp_n);
  t.rp_sN = reinterpret_cast<const int *>(b + o.rp_sN);
  t.rp_sS = reinterpret_cast<const int *>(b + o.rp_sS);
  t.rp_p0n = reinterpret_cast<const int *>(b + o.rp_p0n);
  t.rp_p0d = reinterpret_cast<const int *>(b + o.rp_p0d);
  t.rp_M = reinterpret_cast<const int *>(b + o.rp_M);
  t.rp_bsoff = reinterpret_cast<const int *>(b + o.rp_bsoff);
  t.rp_z = reinterpret_cast<const double *>(b + o.rp_z);
  t.rp_sth = reinterpret_cast<const double *>(b + o.rp_sth);
  t.rp_w = reinterpret_cast<const double *>(b + o.rp_w);
  t.coefA = reinterpret_cast<const double *>(b + o.coefA);
  t.coefC = reinterpret_cast<const double *>(b + o.coefC);
  t.seed_l = reinterpret_cast<const int *>(b + o.seed_l);
  t.seed_v = reinterpret_cast<const double2 *>(b + o.seed_v);
  t.roots64 = reinterpret_cast<const double2 *>(b + o.roots64);
  t.roots32 = reinterpret_cast<const float2 *>(b + o.roots32);
  t.chirp64 = reinterpret_cast<const double2 *>(b + o.chirp64);
  t.chirp32 = reinterpret_cast<const float2 *>(b + o.chirp32);
  t.bhat64 = reinterpret_cast<const double2 *>(b + o.bhat64);
  t.bhat32 = reinterpret_cast<const float2 *>(b + o.bhat32);
  t.rootsP64 = reinterpret_cast<const double2 *>(b + o.rootsP64);
  t.rootsP32 = reinterpret_cast<const float2 *>(b + o.rootsP32);
  t.ck_items = reinterpret_cast<const int2 *>(b + o.ck_items);
  t.ck_xoff = reinterpret_cast<const int *>(b + o.ck_xoff);
  t.ck_pos = reinterpret_cast<const int *>(b + o.ck_pos);
  t.ck_t = reinterpret_cast<const uint8_t *>(b + o.ck_t);
  t.ck_v = reinterpret_cast<const double2 *>(b + o.ck_v);
  t.r2n = reinterpret_cast<const uint32_t *>(b + o.r2n);
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

// Tables of the compute precision.
template <typename T> struct TabOf;
template <> struct TabOf<float> {
  __device__ static const float2 *roots(const Tables &t) { return t.roots32; }
  __device__ static const float2 *chirp(const Tables &t) { return t.chirp32; }
  __device__ static const float2 *bhat(const Tables &t) { return t.bhat32; }
  __device__ static const float2 *rootsP(const Tables &t) { return t.rootsP32; }
};
template <> struct TabOf<double> {
  __device__ static const double2 *roots(const Tables &t) { return t.roots64; }
  __device__ static const double2 *chirp(const Tables &t) { return t.chirp64; }
  __device__ static const double2 *bhat(const Tables &t) { return t.bhat64; }
  __device__ static const double2 *rootsP(const Tables &t) { return t.rootsP64; }
};

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

// Two floats rounded to BF16 (nearest even) in one 32-bit word, `lo` in bits
// 0-15: a complex value (re, im) of the BF16 ring spectra, or two Legendre
// values of the BF16 matrix-core operands.
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}

}  // namespace shtx
