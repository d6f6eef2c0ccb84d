// Per-ring Fourier step of the transforms (Eq. (13), the longitude sum of
// Eq. (24)/(26)), one workgroup per north/south ring pair.
//
// Forward: the two real rings of a pair are packed into one complex sequence
// g = (f_N + f_S) + i (f_N - f_S), transformed with a mixed-radix Stockham FFT
// held in LDS, and split by Hermitian symmetry into the DFTs of f_N + f_S and
// f_N - f_S.  Those are read at k = m mod n (the exact aliasing of
// frequencies m > n/2 on short polar rings), multiplied by the ring weight
// and exp(-i m phi0), and stored as the even/odd parity spectra
// E_m = F_N + F_S and O_m = F_N - F_S of the Legendre step.
//
// Inverse: the per-ring, per-m sums g_m of the Legendre step get the phase
// exp(+i m phi0) and are folded onto k = m mod n (with conj(g_m) on -m mod n
// for the negative frequencies of the real field); the two rings' folded
// spectra are packed as C_N + i C_S, one inverse DFT gives f_N (real part) and
// f_S (imaginary part).
//
// Spectra layout in the workspace: [ring pair p][m][batch], complex.
#include "common.h"

namespace shtx {

constexpr int kFftOutMax = 16;    // complex values per thread per stage
constexpr int kFftThreads = 512;  // threads per workgroup

// Index of logical element o in the LDS work buffer.  Transforms of length
// >= 256 insert one padding slot every 16 elements, so that the stride-R
// writes of a Stockham stage fall into different banks; with that rule a
// channel of length n occupies n + n/16 slots and element o + r*s sits at
// lidx(o) + r*(s + s/16) for any stride s that is a multiple of 16, so every
// stage addresses its R values from one base with a constant stride.
__device__ __forceinline__ int lidx(int o, int pad) { return pad ? o + (o >> 4) : o; }
__device__ __forceinline__ int lstride(int s, int pad) { return pad ? s + (s >> 4) : s; }
inline size_t lds_elems(size_t n) { return n + (n >> 4) + 1; }
constexpr int kPadMin = 256;  // transform length from which the buffer is padded

// Index quotients floor(x / d) for 0 <= x < 2^20, 1 <= d < 2^24, by a
// workgroup-uniform d, without the integer division sequence (about twenty
// instructions per quotient): (x + 1/2) / d lies at least 1/(2d) from every
// integer, and fma(x, r, r/2) with r the hardware reciprocal of d (1 ulp)
// is within a relative 2^-22 of it, an absolute error below
// 2^20 2^-22 / d = 1/(4d), so truncation gives the quotient exactly.  Every
// quotient of this file has x below 16 channels times 4 * 2048 + 8 samples.
struct FastDiv {
  float r, h;
  int d;
  __device__ __forceinline__ explicit FastDiv(int dd) : d(dd) {
    r = __builtin_amdgcn_rcpf((float)dd);
    h = 0.5f * r;
  }
  __device__ __forceinline__ int quo(int x) const { return (int)__builtin_fmaf((float)x, r, h); }
  __device__ __forceinline__ int rem(int x, int q) const { return x - __mul24(q, d); }
};

// Lanes per fold item of the inverse: on short rings every k collects many
// aliases m = +-k mod n (about (lmax + 1) / n per direction), so the aliases
// of one item are dealt to S consecutive lanes of a wave (S a power of two,
// at most 64 and at most the alias count), as long as the items times S fit
// in the workgroup; the lanes' partial sums are added by a fixed butterfly of
// shuffles (deterministic).  Uniform across the workgroup.
__device__ __forceinline__ int fold_lanes(int items, int n, int M, int NT) {
  const int aliases = (M + n - 1) / n;
  int S = 1;
  while (S < 64 && 2 * S * items <= NT && S < aliases) S <<= 1;
  return S;
}
template <typename C> __device__ __forceinline__ C group_sum(C v, int S) {
  for (int o = 1; o < S; o <<= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  return v;
}

// w^e = exp(-2 pi i e / N) for 0 <= e < N from an octant table in LDS,
// tq[r] = w^r for r = 0..N/8 (N = 4 << lq): with e = q N/4 + r,
// w^e = (-i)^q w^r, and for r > N/8, w^r = (sin phi, -cos phi) where
// (cos phi, -sin phi) = tq[N/4 - r].  Branch-free: selects and sign flips.
template <typename C> __device__ __forceinline__ C tw_oct(const C *tq, int e, int lq) {
  const int Q = 1 << lq;
  const int q = e >> lq;
  const int r = e & (Q - 1);
  const bool hi = r > (Q >> 1);
  const C v = tq[hi ? Q - r : r];
  const auto x0 = hi ? -v.y : v.x;
  const auto y0 = hi ? -v.x : v.y;
  const auto a = (q & 1) ? y0 : x0;
  const auto b = (q & 1) ? x0 : y0;
  return cmk<C>((q & 2) ? -a : a, ((q + 1) & 2) ? -b : b);
}

// In-register DFTs of 2, 4, 8 and 16 points (forward, exp(-2 pi i/R)).
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return cmk<C>(a.y, -a.x); }  // * (-i)

template <typename C> __device__ __forceinline__ void dft2(C &a, C &b) {
  const C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename C> __device__ __forceinline__ void dft4(C &u0, C &u1, C &u2, C &u3) {
  const C s02 = cadd(u0, u2), d02 = csub(u0, u2);
  const C s13 = cadd(u1, u3), d13 = mul_mi(csub(u1, u3));
  u0 = cadd(s02, s13);
  u2 = csub(s02, s13);
  u1 = cadd(d02, d13);
  u3 = csub(d02, d13);
}

// multiply by exp(-2 pi i j / 16) for a compile-time j
template <typename C, int J> __device__ __forceinline__ C w16(C a) {
  using R = decltype(C{}.x);
  constexpr int j = J & 15;
  const R c1 = (R)0.92387953251128675613, s1 = (R)0.38268343236508977173, h = (R)0.70710678118654752440;
  if (j == 0) return a;
  if (j == 4) return mul_mi(a);
  if (j == 8) return cmk<C>(-a.x, -a.y);
  if (j == 12) return cmk<C>(-a.y, a.x);
  // exp(-i pi j/8) = cos - i sin
  const R cs = (j == 1 || j == 15) ? c1 : (j == 2 || j == 14) ? h : (j == 3 || j == 13) ? s1
             : (j == 5 || j == 11) ? -s1 : (j == 6 || j == 10) ? -h : -c1;
  const R sn = (j == 1 || j == 7) ? s1 : (j == 2 || j == 6) ? h : (j == 3 || j == 5) ? c1
             : (j == 9 || j == 15) ? -s1 : (j == 10 || j == 14) ? -h : -c1;
  return cmk<C>(a.x * cs + a.y * sn, a.y * cs - a.x * sn);
}

// 8 = 4 x 2:  X[q1 + 4 q2] = sum_r2 W2^{r2 q2} W8^{r2 q1} sum_r1 u[r2 + 2 r1] W4^{r1 q1}
template <typename C> __device__ __forceinline__ void dft8(C (&u)[8]) {
  dft4(u[0], u[2], u[4], u[6]);
  dft4(u[1], u[3], u[5], u[7]);
  u[3] = w16<C, 2>(u[3]);
  u[5] = w16<C, 4>(u[5]);
  u[7] = w16<C, 6>(u[7]);
  dft2(u[0], u[1]);
  dft2(u[2], u[3]);
  dft2(u[4], u[5]);
  dft2(u[6], u[7]);
  // now u[2 q1 + q2] holds X[q1 + 4 q2]; reorder into natural order
  C t[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) t[q] = u[q];
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
    for (int q2 = 0; q2 < 2; ++q2) u[q1 + 4 * q2] = t[2 * q1 + q2];
}

// 16 = 4 x 4:  X[q1 + 4 q2] = sum_r2 W4^{r2 q2} W16^{r2 q1} sum_r1 u[r2 + 4 r1] W4^{r1 q1}
template <typename C> __device__ __forceinline__ void dft16(C (&u)[16]) {
  dft4(u[0], u[4], u[8], u[12]);
  dft4(u[1], u[5], u[9], u[13]);
  dft4(u[2], u[6], u[10], u[14]);
  dft4(u[3], u[7], u[11], u[15]);
  // u[r2 + 4 q1] now holds the inner DFT; twiddle by W16^{r2 q1}
  u[5] = w16<C, 1>(u[5]);
  u[9] = w16<C, 2>(u[9]);
  u[13] = w16<C, 3>(u[13]);
  u[6] = w16<C, 2>(u[6]);
  u[10] = w16<C, 4>(u[10]);
  u[14] = w16<C, 6>(u[14]);
  u[7] = w16<C, 3>(u[7]);
  u[11] = w16<C, 6>(u[11]);
  u[15] = w16<C, 9>(u[15]);
  dft4(u[0], u[1], u[2], u[3]);
  dft4(u[4], u[5], u[6], u[7]);
  dft4(u[8], u[9], u[10], u[11]);
  dft4(u[12], u[13], u[14], u[15]);
  // u[4 q1 + q2] holds X[q1 + 4 q2]: transpose the 4x4 index
  C t[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) t[q] = u[q];
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1)
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) u[q1 + 4 * q2] = t[4 * q1 + q2];
}

template <typename C, int R> __device__ __forceinline__ void dftR(C (&u)[R]) {
  if constexpr (R == 16) dft16(u);
  else if constexpr (R == 8) dft8(u);
  else if constexpr (R == 4) dft4(u[0], u[1], u[2], u[3]);
  else dft2(u[0], u[1]);
}

// u[r] *= w^{r e} for r = 1..R-1 (e < N/R, so no exponent wraps).  One
// table lookup, w^e; the other powers are products (radix 16: w^2e, w^3e,
// w^4e, w^8e, w^12e by squaring and one product each, then the nine
// w^{(r1 + 4 r2) e} = w^{4 r2 e} w^{r1 e}).  A power is at most six roundings
// from the table value.
template <typename C, int R> __device__ __forceinline__ void twiddle(C (&u)[R], const C *tq, int e, int lq) {
  const C w1 = tw_oct(tq, e, lq);
  if constexpr (R == 2) {
    u[1] = cmul(u[1], w1);
  } else if constexpr (R == 4) {
    const C w2 = cmul(w1, w1);
    u[1] = cmul(u[1], w1);
    u[2] = cmul(u[2], w2);
    u[3] = cmul(u[3], cmul(w2, w1));
  } else if constexpr (R == 8) {
    const C w2 = cmul(w1, w1), w3 = cmul(w2, w1), w4 = cmul(w2, w2);
    u[1] = cmul(u[1], w1);
    u[2] = cmul(u[2], w2);
    u[3] = cmul(u[3], w3);
    u[4] = cmul(u[4], w4);
    u[5] = cmul(u[5], cmul(w4, w1));
    u[6] = cmul(u[6], cmul(w4, w2));
    u[7] = cmul(u[7], cmul(w4, w3));
  } else {
    C lo[4], hi[4];
    lo[1] = w1;
    lo[2] = cmul(w1, w1);
    lo[3] = cmul(lo[2], w1);
    hi[1] = cmul(lo[2], lo[2]);
    hi[2] = cmul(hi[1], hi[1]);
    hi[3] = cmul(hi[2], hi[1]);
#pragma unroll
    for (int r1 = 1; r1 < 4; ++r1) u[r1] = cmul(u[r1], lo[r1]);
#pragma unroll
    for (int r2 = 1; r2 < 4; ++r2) {
      u[4 * r2] = cmul(u[4 * r2], hi[r2]);
#pragma unroll
      for (int r1 = 1; r1 < 4; ++r1) u[4 * r2 + r1] = cmul(u[4 * r2 + r1], cmul(hi[r2], lo[r1]));
    }
  }
}

// Optional fused operations on the first stage's inputs / last stage's
// outputs of a power-of-two transform (Bluestein chirp products).
enum FuseIn { kInPlain = 0, kInChirp = 1 };        // x_j * c_j for j < nvalid, 0 beyond
enum FuseOut { kOutPlain = 0, kOutBhat = 1, kOutChirp = 2 };  // conj(y * bhat) / c_o * conj(y) / M

// The tables are read through buffer resources: a 32-bit element offset per
// load (no 64-bit address arithmetic), and a read at or beyond the resource's
// size returns zero instead of touching memory, so the loads need no bounds
// branch.
constexpr int kBufWord3 = 0x00020000;  // untyped 32-bit data, no swizzle
template <typename T> struct Fuse {
  __amdgpu_buffer_rsrc_t chirp;  // c_j for j < nvalid
  __amdgpu_buffer_rsrc_t bhat;   // M values
  int nvalid;
  T scale;
};
// A workgroup-uniform pointer, made visibly uniform (a resource built from a
// value the compiler takes as divergent costs a loop over lanes per load).
template <typename P> __device__ __forceinline__ P *uniform_ptr(P *p) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  return reinterpret_cast<P *>(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ Fuse<T> make_fuse(const cplx<T> *chirp, int nvalid, const cplx<T> *bhat, int M, T scale) {
  nvalid = __builtin_amdgcn_readfirstlane(nvalid);
  M = __builtin_amdgcn_readfirstlane(M);
  return Fuse<T>{__builtin_amdgcn_make_buffer_rsrc(const_cast<cplx<T> *>(uniform_ptr(chirp)), 0,
                                                   nvalid * (int)sizeof(cplx<T>), kBufWord3),
                 __builtin_amdgcn_make_buffer_rsrc(const_cast<cplx<T> *>(uniform_ptr(bhat)), 0,
                                                   M * (int)sizeof(cplx<T>), kBufWord3),
                 nvalid, scale};
}
__device__ __forceinline__ float2 tab_load(__amdgpu_buffer_rsrc_t r, int e, float2) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, 0);
  return make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
}
__device__ __forceinline__ double2 tab_load(__amdgpu_buffer_rsrc_t r, int e, double2) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, e * 16, 0, 0);
  return make_double2(__hiloint2double(v[1], v[0]), __hiloint2double(v[3], v[2]));
}

// Stockham stage of power-of-two radix R on G channels of length n = 2^logn
// with span p = 2^logp: butterfly i of channel c reads x[i + r n/R], twiddles
// by w^{r k n/(R p)} (k = i mod p) and writes y[R(i-k) + k + q p].  The first
// stage (p = 1) has no twiddles.  All inputs are read into registers before
// the workgroup barrier, so the buffer is updated in place.  Every index is a
// shift or a mask; the R values of a butterfly sit at a constant LDS stride
// from one base (padding rule of lidx).  fin / fout select the fused
// operations (uniform across the workgroup).
template <typename T, int NT, int R>
__device__ __forceinline__ void stage_p2(cplx<T> *buf, int logn, int G, int logp, int pad, const cplx<T> *tq,
                                         const Fuse<T> &fz, int fin, int fout) {
  using C = cplx<T>;
  constexpr int LR = R == 16 ? 4 : R == 8 ? 3 : R == 4 ? 2 : 1;
  constexpr int NB = kFftOutMax / R;
  const int n = 1 << logn;
  const int lq = logn - 2;
  const int logTq = logn - LR;
  const int Tq = 1 << logTq;
  const int nb = G << logTq;
  const int p = 1 << logp;
  int cs = __builtin_amdgcn_readfirstlane(lstride(n, pad));
  int is = __builtin_amdgcn_readfirstlane(lstride(Tq, pad));
  int os = __builtin_amdgcn_readfirstlane(logp == 0 ? 1 : lstride(p, pad));
  // Opaque strides: the R offsets r * is and q * os are formed here, per
  // stage (hoisted to the kernel entry they occupy ~30 scalar registers per
  // stage form and spill).
  asm volatile("" : "+s"(cs), "+s"(is), "+s"(os));
  // Opaque copy of the thread index: keeps the per-butterfly index arithmetic
  // inside the stage (hoisted out of the stage loop it would stay live over
  // the whole transform and spill).
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  C v[NB][R];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = tid + s * NT;
    if (b < nb) {
      const int c = b >> logTq, i = b & (Tq - 1);
      const int ib = c * cs + lidx(i, pad);
#pragma unroll
      for (int r = 0; r < R; ++r) v[s][r] = buf[ib + r * is];
      if (fin == kInChirp) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int j = i + r * Tq;
          // zero padding: the buffer beyond nvalid holds no samples (a select,
          // not a product: the LDS there is unset); the load itself reads 0 there
          const C cj = tab_load(fz.chirp, j, C{});
          v[s][r] = (j < fz.nvalid) ? cmul(v[s][r], cj) : cmk<C>(0, 0);
        }
      }
      if (logp > 0) twiddle<C, R>(v[s], tq, (i & (p - 1)) << (logTq - logp), lq);
      dftR<C, R>(v[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = tid + s * NT;
    if (b < nb) {
      const int c = b >> logTq, i = b & (Tq - 1);
      const int k = i & (p - 1);
      const int o0 = ((i - k) << LR) + k;
      const int ob = c * cs + lidx(o0, pad);
      if (fout == kOutPlain) {
#pragma unroll
        for (int q = 0; q < R; ++q) buf[ob + q * os] = v[s][q];
      } else if (fout == kOutBhat) {
#pragma unroll
        for (int q = 0; q < R; ++q) buf[ob + q * os] = cconj(cmul(v[s][q], tab_load(fz.bhat, o0 + q * p, C{})));
      } else {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int o = o0 + q * p;
          const C cv = cconj(v[s][q]);
          const C ch = tab_load(fz.chirp, o, C{});
          if (o < fz.nvalid) buf[ob + q * os] = cmul(ch, cmk<C>(cv.x * fz.scale, cv.y * fz.scale));
        }
      }
    }
  }
  __syncthreads();
}

// Stockham FFT of G channels of power-of-two length n = 2^logn in LDS:
// radix-16 stages, then one radix 2/4/8 stage for the remaining factor (or a
// single radix-4/8 stage for n = 4, 8); twiddles from the LDS octant table tq
// of length n; fused input operation fin on the first stage and output
// operation fout on the last.
template <typename T, int NT>
__device__ __forceinline__ void fft_p2(cplx<T> *buf, int logn, int G, int pad, const cplx<T> *tq, const Fuse<T> &fz,
                                       int fin, int fout) {
  const int n16 = logn >> 2, rem = logn & 3;
  int logp = 0;
#pragma unroll 1
  for (int st = 0; st < n16; ++st, logp += 4) {
    const int fi = st == 0 ? fin : kInPlain;
    const int fo = (st == n16 - 1 && rem == 0) ? fout : kOutPlain;
    stage_p2<T, NT, 16>(buf, logn, G, logp, pad, tq, fz, fi, fo);
  }
  const int fi = n16 == 0 ? fin : kInPlain;
  if (rem == 1) stage_p2<T, NT, 2>(buf, logn, G, logp, pad, tq, fz, fi, fout);
  else if (rem == 2) stage_p2<T, NT, 4>(buf, logn, G, logp, pad, tq, fz, fi, fout);
  else if (rem == 3) stage_p2<T, NT, 8>(buf, logn, G, logp, pad, tq, fz, fi, fout);
}

// Mixed-radix stages for ring lengths n = 4i with odd factors <= 13 (short
// polar rings): twiddles from the ring's full root table in global memory.
// Radix-4/2 stage (span p):
template <typename T, int NT, int R>
__device__ __forceinline__ void stage_mix_p2(cplx<T> *buf, int n, int G, int p, int pad,
                                             const cplx<T> *__restrict__ roots) {
  using C = cplx<T>;
  constexpr int NB = kFftOutMax / R;
  const int Tq = n / R;
  const int nb = G * Tq;
  const int step = n / (R * p);
  const FastDiv dq(Tq);  // p is a power of two here: k = i mod p by a mask
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  C v[NB][R];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = tid + s * NT;
    if (b < nb) {
      const int c = dq.quo(b), i = dq.rem(b, c);
      const int k = i & (p - 1);
      const int e = k * step;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const C u = buf[lidx(c * n + i + r * Tq, pad)];
        v[s][r] = (r == 0) ? u : cmul(u, roots[r * e]);
      }
      dftR<C, R>(v[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = tid + s * NT;
    if (b < nb) {
      const int c = dq.quo(b), i = dq.rem(b, c);
      const int k = i & (p - 1);
      const int o0 = (i - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) buf[lidx(c * n + o0 + q * p, pad)] = v[s][q];
    }
  }
  __syncthreads();
}

// Stage of odd radix R (span p, R <= kMaxDirectPrime): thread per output,
//   y[g pR + q p + k] = sum_r x[g p + k + r n/R] w^{r (n/(pR)) (k + q p)}.
// The root-table loads of an output are issued four at a time (indices by
// integer adds), so an output waits for ceil((R - 1) / 4) load latencies
// rather than for R - 1 in a row.
template <typename T, int NT>
__device__ __forceinline__ void stage_odd(cplx<T> *buf, int n, int G, int p, int R, int pad,
                                          const cplx<T> *__restrict__ roots) {
  using C = cplx<T>;
  const int tot = G * n;
  const int Tn = n / R;
  const int pR = p * R;
  const int step = n / pR;
  const FastDiv dn(n), dpr(pR), dp(p);
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  C out[kFftOutMax];
#pragma unroll
  for (int s = 0; s < kFftOutMax; ++s) {
    const int o = tid + s * NT;
    if (o < tot) {
      const int c = dn.quo(o);
      const int oo = dn.rem(o, c);
      const int g = dpr.quo(oo);
      const int rr = dpr.rem(oo, g);
      const int q = dp.quo(rr);
      const int k = dp.rem(rr, q);
      const int xb = c * n + g * p + k;
      const int be = step * (k + q * p);
      C acc = buf[lidx(xb, pad)];
      int e = be;
#pragma unroll 1
      for (int r0 = 1; r0 < R; r0 += 4) {
        C wr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (r0 + u < R) wr[u] = roots[e];
          e += be;
          if (e >= n) e -= n;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (r0 + u < R) acc = cadd(acc, cmul(buf[lidx(xb + (r0 + u) * Tn, pad)], wr[u]));
      }
      out[s] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kFftOutMax; ++s) {
    const int o = tid + s * NT;
    if (o < tot) buf[lidx(o, pad)] = out[s];
  }
  __syncthreads();
}

// Mixed-radix Stockham FFT of G channels of length n = 4i: radix-4 stages over
// the power-of-two part, one radix-2 stage if needed, then one direct stage
// per remaining odd prime factor (all <= kMaxDirectPrime on this path).
template <typename T, int NT>
__device__ __forceinline__ void fft_mixed(cplx<T> *buf, int n, int G, int pad, const cplx<T> *__restrict__ roots) {
  int rem = n, p = 1;
  while ((rem & 3) == 0) {
    stage_mix_p2<T, NT, 4>(buf, n, G, p, pad, roots);
    p <<= 2;
    rem >>= 2;
  }
  if ((rem & 1) == 0) {
    stage_mix_p2<T, NT, 2>(buf, n, G, p, pad, roots);
    p <<= 1;
    rem >>= 1;
  }
  while (rem > 1) {
    int R = rem;
    for (int r = 3; r * r <= rem; r += 2)
      if (rem % r == 0) {
        R = r;
        break;
      }
    stage_odd<T, NT>(buf, n, G, p, R, pad, roots);
    p *= R;
    rem /= R;
  }
}

// Octant root table of the power-of-two length N into LDS; the source is the
// root table of length N * rs.
template <typename T, int NT>
__device__ __forceinline__ void load_octant(cplx<T> *tq, const cplx<T> *__restrict__ src, int N, int rs) {
  for (int r = threadIdx.x; r <= N / 8; r += NT) tq[r] = src[r * rs];
}

// Forward DFT of gc channels of ring-pair p held in buf (channel-major, LDS
// layout lidx(., pad)); tq is LDS space for an octant root table.  Every
// thread of the workgroup calls this (it synchronises internally).  Ring
// lengths with a power-of-two part only take radix-16 Stockham stages, the
// others (prime factors <= kMaxDirectPrime) mixed-radix stages.
template <typename T, int NT>
__device__ __forceinline__ void ring_dft(const Tables &tb, cplx<T> *buf, cplx<T> *tq, int n, int gc, int pad,
                                         bool tq_ready) {
  if (n & (n - 1)) {
    fft_mixed<T, NT>(buf, n, gc, pad, TabOf<T>::roots(tb) + roots_offset(n >> 2));
    return;
  }
  if (!tq_ready) {
    load_octant<T, NT>(tq, TabOf<T>::roots(tb) + roots_offset(n >> 2), n, 1);
    __syncthreads();
  }
  const Fuse<T> fz = make_fuse<T>(nullptr, 0, nullptr, 0, (T)1);
  fft_p2<T, NT>(buf, __builtin_ctz(n), gc, pad, tq, fz, kInPlain, kOutPlain);
}

// A Bluestein ring's four length-i sub-transforms run as the channels of
// power-of-two FFT calls, nb = 4, 2 or 1 per call (as many as one stage and
// the LDS hold).  The results of the calls before the last wait in LDS; with
// nb = 1, FP64 keeps the third in registers, which makes the LDS need fit at
// nside 2048.
template <typename T> struct BsLayout {
  static constexpr int kLdsY1 = sizeof(T) == 8 ? 2 : 3;  // results kept in LDS when nb = 1
};
template <int NT> struct BsSlots {  // values of s < i per thread (i < kMaxNside)
  static constexpr int value = (kMaxNside + NT - 1) / NT;
};

// Forward DFT of one channel of a ring of length n = 4i whose i has a prime
// factor above kMaxDirectPrime (Bluestein ring, convolution length M):
//   X[s + i r] = sum_q w_n^{q s} (-i)^{q r} Y_q[s],  s < i, r, q = 0..3,
// with Y_q the length-i DFT of the samples x[4j + q].  Each Y_q is Bluestein's
// DFT (Eq. (17)-(23)): with the chirp c_j = exp(-i pi j^2 / i),
// Y_q[s] = c_s sum_j (x[4j + q] c_j) conj(c_{s-j}), the convolution done
// cyclically on length M with the precomputed transform bhat of conj(c) and
// two power-of-two FFTs (the inverse one through conjugation); the chirp
// products, the zero padding and the product with bhat are fused into their
// first and last stages.  input(c, k) returns x[k] of channel c < gc (gc > 1
// only with nb = 4).  LDS: the results kept there at [q i, (q+1) i), then the
// gc nb convolution channels (layout lidx(., M >= kPadMin) each).  X of
// channel c ends in buf[c n, (c+1) n) unpadded.  tq holds (or receives) the
// octant table of M.
template <typename T, int NT, typename In>
__device__ __forceinline__ void ring_dft_bs4(const Tables &tb, int p, int M, int nb, int gc, cplx<T> *buf,
                                             cplx<T> *tq, int n, bool tq_ready, In input, int S = 1) {
  using C = cplx<T>;
  constexpr int NS = BsSlots<NT>::value;
  const int i = n >> 2;
  const int padM = M >= kPadMin;
  const int cs = lstride(M, padM);                                   // convolution channel stride
  const int ylds = nb == 4 ? 0 : nb == 2 ? 2 : BsLayout<T>::kLdsY1;  // results kept in LDS
  const int qlast = 4 - nb;                                          // first result of the last call
  C *wb = buf + ylds * i;                                            // convolution buffer
  if (!tq_ready) {
    load_octant<T, NT>(tq, TabOf<T>::rootsP(tb), M, tb.mmax_bs / M);
    __syncthreads();
  }
  const Fuse<T> fz = make_fuse<T>(TabOf<T>::chirp(tb) + roots_offset(i), i, TabOf<T>::bhat(tb) + tb.rp_bsoff[p], M,
                                  (T)1 / (T)M);
  const int logM = __builtin_ctz(M);
  const int lnb = nb >> 1;  // log2 nb for nb = 1, 2, 4
  const FastDiv di(i);
  // opaque copies of the thread index per phase (as in stage_p2): index
  // arithmetic hoisted out of the pass loop would stay live and spill
  int tid = threadIdx.x;
  C yr[NS];  // a result kept in registers (nb = 1, FP64)
#pragma unroll 1
  for (int q0 = 0; q0 < 4; q0 += nb) {
    tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (S == 1) {
      for (int e = tid; e < gc * nb * i; e += NT) {
        const int cc = di.quo(e), j = di.rem(e, cc);  // convolution channel cc = (channel, sub-transform)
        wb[cc * cs + lidx(j, padM)] = input(cc >> lnb, 4 * j + q0 + (cc & (nb - 1)), 0, 1);
      }
    } else {
      // S lanes per sample, each returning its share (a wave-uniform loop:
      // every lane of a wave takes part in the shuffles)
      const int ls = __builtin_ctz(S), tot = (gc * nb * i) << ls;
      for (int e0 = tid & ~63; e0 < tot; e0 += NT) {
        const int e = e0 + (tid & 63);
        const bool ok = e < tot;
        const int it = e >> ls, r = e & (S - 1);
        const int cc = di.quo(it), j = di.rem(it, cc);
        C v = cmk<C>(0, 0);
        if (ok) v = input(cc >> lnb, 4 * j + q0 + (cc & (nb - 1)), r, S);
        v = group_sum(v, S);
        if (ok && r == 0) wb[cc * cs + lidx(j, padM)] = v;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int ps = 0; ps < 2; ++ps)
      fft_p2<T, NT>(wb, logM, gc * nb, padM, tq, fz, ps == 0 ? kInChirp : kInPlain,
                    ps == 0 ? kOutBhat : kOutChirp);
    if (q0 == qlast) break;  // the last results stay in the convolution buffer
    tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (BsLayout<T>::kLdsY1 < 3 && q0 >= ylds) {  // nb = 1: the result kept in registers
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int s = tid + u * NT;
        if (s < i) yr[u] = wb[lidx(s, padM)];
      }
    } else {
      for (int e = tid; e < nb * i; e += NT) {
        const int c = di.quo(e), s = di.rem(e, c);
        buf[(q0 + c) * i + s] = wb[c * cs + lidx(s, padM)];
      }
    }
    __syncthreads();
  }
  // radix-4 combination: all four results of this thread's s into registers,
  // then X over the same LDS
  const C *w = TabOf<T>::roots(tb) + roots_offset(i);  // w_n^e, e < n
  tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  C z[NS][4];
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int e = tid + u * NT;  // (channel, s)
    const int c = di.quo(e), s = di.rem(e, c);
    if (c < gc) {
      C y[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) y[q] = q >= qlast ? wb[(c * nb + q - qlast) * cs + lidx(s, padM)] : buf[q * i + s];
      if (BsLayout<T>::kLdsY1 < 3) {  // Y_2 from registers (a value select: yr stays in registers)
        const bool reg = qlast > 2 && ylds <= 2;
        y[2].x = reg ? yr[u].x : y[2].x;
        y[2].y = reg ? yr[u].y : y[2].y;
      }
      z[u][0] = y[0];
      z[u][1] = cmul(y[1], w[s]);
      z[u][2] = cmul(y[2], w[2 * s]);
      z[u][3] = cmul(y[3], w[3 * s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NS; ++u) {
    const int e = tid + u * NT;
    const int c = di.quo(e), s = di.rem(e, c);
    if (c < gc) {
      dft4(z[u][0], z[u][1], z[u][2], z[u][3]);
#pragma unroll
      for (int r = 0; r < 4; ++r) buf[c * n + s + r * i] = z[u][r];
    }
  }
  __syncthreads();
}

// Channels of a Bluestein ring per call of ring_dft_bs4: several when all
// four sub-transforms share one call (nb = 4) and the stage (kFftOutMax per
// thread), the LDS buffer (buf_elems) and the result slots hold them.
template <int NT>
__device__ __forceinline__ int bs_channels(int G, int nb, int M, int n, int buf_elems) {
  if (nb != 4) return 1;
  const int cs = lstride(M, M >= kPadMin);
  int g = min(G, NT * kFftOutMax / (4 * M));
  g = min(g, buf_elems / (4 * cs));
  g = min(g, NT * BsSlots<NT>::value / (n >> 2));
  return max(g, 1);
}

// Ring phase exp(+-i m phi0): phi0 = pi num / den with num = 0, or num = 1
// and den = n, the ring length (HEALPix caps: pi/(4i); belt: pi/(4 nside) on
// every other ring).  From the ring's root table w^q = exp(-2 pi i q / n):
// for m mod 2n = 2q + b, exp(i pi m / n) = conj(w^q) h^b with h = exp(i pi/n)
// (a lookup and one product instead of a sine and cosine).  mm = m mod 2n.
template <typename T> struct RingPhase {
  const cplx<T> *w;  // roots of the ring length
  cplx<T> h;         // exp(i pi / n)
  bool on;           // num = 1
  __device__ __forceinline__ cplx<T> plus(int mm) const {  // exp(+i m phi0)
    using C = cplx<T>;
    if (!on) return cmk<C>(1, 0);
    const C r = cconj(w[mm >> 1]);
    const C hb = (mm & 1) ? h : cmk<C>(1, 0);
    return cmul(r, hb);
  }
  __device__ __forceinline__ cplx<T> minus(int mm) const { return cconj(plus(mm)); }  // exp(-i m phi0)
};
template <typename T>
__device__ __forceinline__ RingPhase<T> ring_phase(const Tables &tb, int n, int num) {
  return RingPhase<T>{TabOf<T>::roots(tb) + roots_offset(n >> 2), phase_pi<T>(1, n, (T)1), num != 0};
}

// Workgroup -> (ring pair, channel slice).  A ring pair's channels are split
// into ceil(B / G) slices of G; the slices of one ring pair get consecutive
// workgroup ids of one XCD (ids x, x+8, x+16, ... go to XCD x), so the
// partial writes and reads of their shared [p][m][batch] spectrum lines meet
// in that XCD's L2.
__device__ __forceinline__ bool fft_work(int Rp, int B, int G, int *p, int *b0, int *b1) {
  const int ncg = (B + G - 1) / G;
  const int g = blockIdx.x;
  const int x = g & 7, k = g >> 3;
  const int pp = x + 8 * (k / ncg);
  const int cg = k % ncg;
  if (pp >= Rp) return false;
  *p = pp;
  *b0 = cg * G;
  *b1 = min(B, *b0 + G);
  return true;
}

// The same for maps in NESTED order (the analysis reads them in place, the
// RING order of Sec. III-B applied to its loads): ring pairs in bands of
// kNestBand consecutive pairs, bands dealt round-robin to the XCDs, so that
// the neighbouring rings that share the 128-byte lines of a NESTED map
// (a line holds an 8 x 4 block of a face, which spans 11 rings) are read by
// one XCD close in time and meet in its L2.
constexpr int kNestBand = 32;
__device__ __forceinline__ bool fft_work_banded(int Rp, int B, int G, int *p, int *b0, int *b1) {
  const int ncg = (B + G - 1) / G;
  const int g = blockIdx.x;
  const int x = g & 7, k = g >> 3;
  const int t = k / ncg, cg = k % ncg;
  const int pp = ((t / kNestBand) * 8 + x) * kNestBand + t % kNestBand;
  if (pp >= Rp) return false;
  *p = pp;
  *b0 = cg * G;
  *b1 = min(B, *b0 + G);
  return true;
}

// Four consecutive map pixels as T (the caller guarantees 4-element
// alignment of p: ring starts and lengths are multiples of 4 pixels).
template <typename T, typename S> __device__ __forceinline__ void load4(const S *p, T (&v)[4]);
template <> __device__ __forceinline__ void load4<float, float>(const float *p, float (&v)[4]) {
  const float4 q = *reinterpret_cast<const float4 *>(p);
  v[0] = q.x;
  v[1] = q.y;
  v[2] = q.z;
  v[3] = q.w;
}
template <> __device__ __forceinline__ void load4<double, double>(const double *p, double (&v)[4]) {
  const double2 a = reinterpret_cast<const double2 *>(p)[0];
  const double2 b = reinterpret_cast<const double2 *>(p)[1];
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
template <> __device__ __forceinline__ void load4<float, bf16_t>(const bf16_t *p, float (&v)[4]) {
  const uint2 q = *reinterpret_cast<const uint2 *>(p);
  v[0] = __uint_as_float(q.x << 16);
  v[1] = __uint_as_float(q.x & 0xffff0000u);
  v[2] = __uint_as_float(q.y << 16);
  v[3] = __uint_as_float(q.y & 0xffff0000u);
}

// Four consecutive map pixels (the caller guarantees 4-element alignment, as
// for load4): one 16-byte store (FP32), two (FP64) or one 8-byte store of
// four rounded bfloat16 values.
template <typename S, typename T> __device__ __forceinline__ void store4(S *p, const T (&v)[4]);
template <> __device__ __forceinline__ void store4<float, float>(float *p, const float (&v)[4]) {
  *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
template <> __device__ __forceinline__ void store4<double, double>(double *p, const double (&v)[4]) {
  reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}
template <> __device__ __forceinline__ void store4<bf16_t, float>(bf16_t *p, const float (&v)[4]) {
  bf16_t t[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) store_as<bf16_t, float>(&t[e], v[e]);
  *reinterpret_cast<uint2 *>(p) = make_uint2((uint32_t)t[0].bits | ((uint32_t)t[1].bits << 16),
                                             (uint32_t)t[2].bits | ((uint32_t)t[3].bits << 16));
}

// Analysis spectra are stored as the compute type's complex, or as BF16
// complex words (re in bits 0-15) for the BF16 matrix-core Legendre step.
__device__ __forceinline__ void store_spec(float2 *p, float2 v) { *p = v; }
__device__ __forceinline__ void store_spec(double2 *p, double2 v) { *p = v; }
__device__ __forceinline__ void store_spec(uint32_t *p, float2 v) { *p = pack_bf16x2(v.x, v.y); }

// Two adjacent complex values (FP32: one 16-byte store; BF16: one 8-byte store).
__device__ __forceinline__ void store_pair(float2 *p, float2 a, float2 b) {
  *reinterpret_cast<float4 *>(p) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void store_pair(double2 *p, double2 a, double2 b) {
  p[0] = a;
  p[1] = b;
}
__device__ __forceinline__ void store_pair(uint32_t *p, float2 a, float2 b) {
  *reinterpret_cast<uint2 *>(p) = make_uint2(pack_bf16x2(a.x, a.y), pack_bf16x2(b.x, b.y));
}

constexpr int kLoadUnroll = 2;  // quads of pixels in flight per thread

// Pixels j..j+3 of a ring (first pixel s) of one channel `row`: RING maps are
// read as one vector, NESTED maps (NEST) pixel by pixel at the NESTED index
// of each RING pixel (tables: r2n).
template <bool NEST, typename T, typename TIn>
__device__ __forceinline__ void load_ring4(const Tables &tb, const TIn *row, int s, int j, T (&v)[4]) {
  if constexpr (NEST) {
    const uint4 ix = *reinterpret_cast<const uint4 *>(tb.r2n + s + j);
    v[0] = load_as<T, TIn>(row + ix.x);
    v[1] = load_as<T, TIn>(row + ix.y);
    v[2] = load_as<T, TIn>(row + ix.z);
    v[3] = load_as<T, TIn>(row + ix.w);
  } else {
    load4<T, TIn>(row + s + j, v);
  }
}

// Per-pixel quadrature weights (RING order, FP64) on four consecutive pixels.
template <typename T> __device__ __forceinline__ void weigh4(const double *pw, int s, int j, T (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2 *>(pw + s + j);
  const double2 b = *reinterpret_cast<const double2 *>(pw + s + j + 2);
  v[0] *= (T)a.x;
  v[1] *= (T)a.y;
  v[2] *= (T)b.x;
  v[3] *= (T)b.y;
}

template <typename TIn, typename T, typename TS, bool NEST, int NT>
__global__ void __launch_bounds__(NT, sizeof(T) == 4 ? 4 : 2)
    k_ring_fft_fwd(Tables tb, int B, int G, int tq_off, int bs_nb, const TIn *__restrict__ map,
                   const double *__restrict__ wtab, double wscale, const double *__restrict__ pixw,
                   TS *__restrict__ XE, TS *__restrict__ XO) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf = reinterpret_cast<C *>(smem_raw);
  C *tq = buf + tq_off;
  int p, bg0, bg1;
  if (!(NEST ? fft_work_banded(tb.npairs, B, G, &p, &bg0, &bg1) : fft_work(tb.npairs, B, G, &p, &bg0, &bg1))) return;
  const int n = tb.rp_n[p];
  const int sN = tb.rp_sN[p], sS = tb.rp_sS[p];
  const bool equator = (sN == sS);
  const int L = tb.lmax, M = L + 1;
  const T w = (T)(wtab ? wtab[p] * wscale : wscale);
  const int num = tb.rp_p0n[p];  // phase numerator (the denominator is n when num = 1)
  const size_t npix = (size_t)tb.npix;
  const int Mbs = tb.rp_M[p];
  const int pad = Mbs == 0 && n >= kPadMin;  // Bluestein rings leave their DFT unpadded
  const int Gp = Mbs ? bs_channels<NT>(G, bs_nb, Mbs, n, tq_off) : G;
  const int nq = n >> 2;  // quads of pixels per ring
  const FastDiv dnq(nq);
  const RingPhase<T> rph = ring_phase<T>(tb, n, num);
  const int tid = threadIdx.x;
#pragma unroll 1
  for (int b0 = bg0; b0 < bg1; b0 += Gp) {
    const int gc = min(Gp, bg1 - b0);
    if (Mbs) {
      // Bluestein ring: samples read per sub-transform, packed on the fly
      auto input = [&](int c, int k, int, int) {
        const TIn *row = map + (size_t)(b0 + c) * npix;
        const int kN = NEST ? (int)tb.r2n[sN + k] : sN + k;
        const int kS = NEST ? (int)tb.r2n[sS + k] : sS + k;
        T a = load_as<T, TIn>(row + kN), b = equator ? (T)0 : load_as<T, TIn>(row + kS);
        if (pixw) {
          a *= (T)pixw[sN + k];
          if (!equator) b *= (T)pixw[sS + k];
        }
        return cmk<C>(a + b, a - b);
      };
      ring_dft_bs4<T, NT>(tb, p, Mbs, bs_nb, gc, buf, tq, n, b0 != bg0, input);
    } else {
      // rings -> LDS, packed as (f_N + f_S) + i (f_N - f_S); every load of the
      // pass is issued before the LDS writes
#pragma unroll 1
      for (int q0 = tid; q0 < gc * nq; q0 += kLoadUnroll * NT) {
        T fN[kLoadUnroll][4], fS[kLoadUnroll][4];
#pragma unroll
        for (int u = 0; u < kLoadUnroll; ++u) {
          const int q = q0 + u * NT;
          if (q < gc * nq) {
            const int c = dnq.quo(q), j = 4 * dnq.rem(q, c);
            const TIn *row = map + (size_t)(b0 + c) * npix;
            load_ring4<NEST, T, TIn>(tb, row, sN, j, fN[u]);
            if (!equator) load_ring4<NEST, T, TIn>(tb, row, sS, j, fS[u]);
            if (pixw) {
              weigh4<T>(pixw, sN, j, fN[u]);
              if (!equator) weigh4<T>(pixw, sS, j, fS[u]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kLoadUnroll; ++u) {
          const int q = q0 + u * NT;
          if (q < gc * nq) {
            const int c = dnq.quo(q), j = 4 * dnq.rem(q, c);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const T a = fN[u][e], b = equator ? (T)0 : fS[u][e];
              buf[lidx(c * n + j + e, pad)] = cmk<C>(a + b, a - b);
            }
          }
        }
      }
      __syncthreads();
      ring_dft<T, NT>(tb, buf, tq, n, gc, pad, b0 != bg0);
    }
    // E/O spectra for m = 0..L; one phase per m, channels contiguous
    const size_t obase = (size_t)p * M * B + b0;
    const bool pairs = ((B | b0) & 1) == 0;  // channel pairs start 16-byte aligned
    const FastDiv d2n(2 * n);
    for (int m = tid; m < M; m += NT) {
      const int mm = m < 2 * n ? m : d2n.rem(m, d2n.quo(m));  // m mod 2n
      const int k = mm < n ? mm : mm - n;          // m mod n
      const int kc = (k == 0) ? 0 : n - k;
      C ph = rph.minus(mm);
      ph.x *= w;
      ph.y *= w;
      TS *xe = XE + obase + (size_t)m * B;
      TS *xo = XO + obase + (size_t)m * B;
      int c = 0;
      // U = DFT(fN+fS)[k] = (G[k] + conj(G[-k]))/2 ; V = DFT(fN-fS)[k] = (G[k] - conj(G[-k]))/(2i)
      auto uv = [&](int cc, C &U, C &V) {
        const C Gk = buf[lidx(cc * n + k, pad)];
        const C Gc = buf[lidx(cc * n + kc, pad)];
        U = cmul(ph, cmk<C>((T)0.5 * (Gk.x + Gc.x), (T)0.5 * (Gk.y - Gc.y)));
        V = cmul(ph, cmk<C>((T)0.5 * (Gk.y + Gc.y), (T)0.5 * (Gc.x - Gk.x)));
      };
      if (pairs) {
        for (; c + 1 < gc; c += 2) {
          C U0, V0, U1, V1;
          uv(c, U0, V0);
          uv(c + 1, U1, V1);
          store_pair(xe + c, U0, U1);
          store_pair(xo + c, V0, V1);
        }
      }
      for (; c < gc; ++c) {
        C U, V;
        uv(c, U, V);
        store_spec(xe + c, U);
        store_spec(xo + c, V);
      }
    }
    __syncthreads();
  }
}

constexpr int kFoldUnroll = 2;  // (k, channel) items per thread with loads in flight


template <typename TOut, typename T, int NT>
__global__ void __launch_bounds__(NT, sizeof(T) == 4 ? 4 : 2)
    k_ring_fft_inv(Tables tb, int B, int G, int tq_off, int bs_nb, const cplx<T> *__restrict__ GN,
                   const cplx<T> *__restrict__ GS, const TOut *__restrict__ sub, TOut *__restrict__ map) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf = reinterpret_cast<C *>(smem_raw);
  C *tq = buf + tq_off;
  int p, bg0, bg1;
  if (!fft_work(tb.npairs, B, G, &p, &bg0, &bg1)) return;
  const int n = tb.rp_n[p];
  const int sN = tb.rp_sN[p], sS = tb.rp_sS[p];
  const bool equator = (sN == sS);
  const int L = tb.lmax, M = L + 1;
  const int num = tb.rp_p0n[p];  // phase numerator (the denominator is n when num = 1)
  const size_t npix = (size_t)tb.npix;
  const int Mbs = tb.rp_M[p];
  const int pad = Mbs == 0 && n >= kPadMin;  // Bluestein rings leave their DFT unpadded
  const int Gp = Mbs ? bs_channels<NT>(G, bs_nb, Mbs, n, tq_off) : G;
  int tid = threadIdx.x;
  // c_m = g_m exp(+i m phi0), mm = m mod 2n
  const RingPhase<T> rph = ring_phase<T>(tb, n, num);
  // synthesis spectra [p][m][B]: this workgroup reads channels [bg0, bg1) of
  // each m row (the other channel slices of the row are read by the
  // workgroups of the same ring pair, dealt to the same XCD at the same time)
  auto phased = [&](const C *src, int m, int mm) { return cmul(src[(size_t)m * B], rph.plus(mm)); };
  const size_t sbase = (size_t)p * M * B + bg0;
  // Fold onto k = m mod n (positive frequencies) and k = -m mod n (negative,
  // conj) for channel c of the slice at gn / gs: the first term of each sum is
  // loaded by fold_load (so that several items can have their loads in
  // flight), fold_value adds the phases and further aliases (short rings) and
  // returns conj(h), h = C_N + i C_S, so that a forward DFT gives conj(IDFT(h)).
  auto fold_load = [&](const C *gn, const C *gs, int k, int c, C &pn, C &ps, C &qn, C &qs) {
    const int m1 = k, m2 = (k == 0) ? n : n - k;
    pn = ps = qn = qs = cmk<C>(0, 0);
    if (m1 < M) {
      pn = gn[(size_t)m1 * B + c];
      if (!equator) ps = gs[(size_t)m1 * B + c];
    }
    if (m2 < M) {
      qn = gn[(size_t)m2 * B + c];
      if (!equator) qs = gs[(size_t)m2 * B + c];
    }
  };
  // C_N, C_S at k (the sums over the aliases m = +-k mod n of g_m exp(i m phi0),
  // the negative ones conjugated).  At n - k the sums are the conjugates: the
  // aliases of +k are those of -(n - k) and vice versa.
  auto fold_sums = [&](const C *gn, const C *gs, int k, int c, C pn, C ps, C qn, C qs, C &cn, C &cs) {
    cn = cmk<C>(0, 0);
    cs = cmk<C>(0, 0);
    const int m1 = k, m2 = (k == 0) ? n : n - k;  // both below 2n
    if (m1 < M) {
      const C ph = rph.plus(m1);
      cn = cmul(pn, ph);
      cs = cmul(ps, ph);
      if (m1 == 0) {
        cn.y = 0;
        cs.y = 0;
      }
    }
    if (m2 < M) {
      const C ph = rph.plus(m2);
      cn = cadd(cn, cconj(cmul(qn, ph)));
      cs = cadd(cs, cconj(cmul(qs, ph)));
    }
    // further aliases m + t n: m mod 2n alternates between m and m + n
    for (int m = m1 + n, mm = m1 + n; m < M; m += n, mm = mm >= n ? mm - n : mm + n) {
      cn = cadd(cn, phased(gn + c, m, mm));
      if (!equator) cs = cadd(cs, phased(gs + c, m, mm));
    }
    for (int m = m2 + n, mm = m2 + n >= 2 * n ? m2 - n : m2 + n; m < M;
         m += n, mm = mm >= n ? mm - n : mm + n) {
      cn = cadd(cn, cconj(phased(gn + c, m, mm)));
      if (!equator) cs = cadd(cs, cconj(phased(gs + c, m, mm)));
    }
  };
  auto fold_value = [&](const C *gn, const C *gs, int k, int c, C pn, C ps, C qn, C qs) {
    C cn, cs;
    fold_sums(gn, gs, k, c, pn, ps, qn, qs, cn, cs);
    return cmk<C>(cn.x - cs.y, -(cn.y + cs.x));
  };
  // The share of lane r of S (0 <= r < S) in C_N, C_S at k: lane 0 takes the
  // base terms m1 = k and m2 = n - k (as fold_sums), lane r the aliases
  // m1 + t n and m2 + t n with t >= 1, t = r mod S.  With S even the aliases
  // of one lane share m mod 2n, so their phase is applied once to their sum.
  auto fold_part = [&](const C *gn, const C *gs, int k, int c, int r, int S, C &cn, C &cs) {
    cn = cmk<C>(0, 0);
    cs = cmk<C>(0, 0);
    const int m1 = k, m2 = (k == 0) ? n : n - k;
    if (r == 0) {
      C pn, ps, qn, qs;
      fold_load(gn, gs, k, c, pn, ps, qn, qs);
      if (m1 < M) {
        const C ph = rph.plus(m1);
        cn = cmul(pn, ph);
        cs = cmul(ps, ph);
        if (m1 == 0) {
          cn.y = 0;
          cs.y = 0;
        }
      }
      if (m2 < M) {
        const C ph = rph.plus(m2);
        cn = cadd(cn, cconj(cmul(qn, ph)));
        cs = cadd(cs, cconj(cmul(qs, ph)));
      }
    }
    const int t0 = r == 0 ? S : r;
    // positive frequencies: m = m1 + t n
    {
      C an = cmk<C>(0, 0), as = cmk<C>(0, 0);
      const int mm = m1 + (t0 & 1) * n;  // m mod 2n (the same for every t of this lane)
#pragma unroll 4
      for (int m = m1 + t0 * n; m < M; m += S * n) {
        an = cadd(an, gn[(size_t)m * B + c]);
        if (!equator) as = cadd(as, gs[(size_t)m * B + c]);
      }
      const C ph = rph.plus(mm);
      cn = cadd(cn, cmul(an, ph));
      cs = cadd(cs, cmul(as, ph));
    }
    // negative frequencies: m = m2 + t n, conjugated
    {
      C an = cmk<C>(0, 0), as = cmk<C>(0, 0);
      int mm = m2 + (t0 & 1) * n;
      if (mm >= 2 * n) mm -= 2 * n;
#pragma unroll 4
      for (int m = m2 + t0 * n; m < M; m += S * n) {
        an = cadd(an, gn[(size_t)m * B + c]);
        if (!equator) as = cadd(as, gs[(size_t)m * B + c]);
      }
      const C ph = rph.plus(mm);
      cn = cadd(cn, cconj(cmul(an, ph)));
      cs = cadd(cs, cconj(cmul(as, ph)));
    }
  };
#pragma unroll 1
  for (int b0 = bg0; b0 < bg1; b0 += Gp) {
    // opaque thread index per channel pass: keeps the pass's index and
    // address arithmetic inside the loop (hoisted, it would spill)
    tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int gc = min(Gp, bg1 - b0);
    const C *gn = GN + sbase + (b0 - bg0);
    const C *gs = GS + sbase + (b0 - bg0);
    if (Mbs) {
      // Bluestein ring: folded values computed per sub-transform sample
      auto input = [&](int c, int k, int r, int S) {
        if (S == 1) {
          C pn, ps, qn, qs;
          fold_load(gn, gs, k, c, pn, ps, qn, qs);
          return fold_value(gn, gs, k, c, pn, ps, qn, qs);
        }
        C cn, cs;
        fold_part(gn, gs, k, c, r, S, cn, cs);
        return cmk<C>(cn.x - cs.y, -(cn.y + cs.x));
      };
      ring_dft_bs4<T, NT>(tb, p, Mbs, bs_nb, gc, buf, tq, n, b0 != bg0, input,
                          fold_lanes(gc * min(bs_nb, 4) * (n >> 2), n, M, NT));
    } else {
      // k = 0..n/2; each item also writes k' = n - k (conjugate sums)
      const int nk = gc * ((n >> 1) + 1);
      const int S = fold_lanes(nk, n, M, NT);
      const FastDiv dgc(gc);
      if (S > 1) {
        // short ring: S lanes per item (a wave-uniform loop: every lane of a
        // wave takes part in the shuffles)
        const int ls = __builtin_ctz(S), tot = nk << ls;
#pragma unroll 1
        for (int e0 = tid & ~63; e0 < tot; e0 += NT) {
          const int e = e0 + (tid & 63);
          const bool ok = e < tot;
          const int j = e >> ls, r = e & (S - 1);
          const int k = dgc.quo(j), c = dgc.rem(j, k);
          C cn = cmk<C>(0, 0), cs = cmk<C>(0, 0);
          if (ok) fold_part(gn, gs, k, c, r, S, cn, cs);
          cn = group_sum(cn, S);
          cs = group_sum(cs, S);
          if (ok && r == 0) {
            buf[lidx(c * n + k, pad)] = cmk<C>(cn.x - cs.y, -(cn.y + cs.x));
            if (k != 0 && 2 * k != n) buf[lidx(c * n + n - k, pad)] = cmk<C>(cn.x + cs.y, cn.y - cs.x);
          }
        }
      }
#pragma unroll 1
      for (int j0 = tid; S == 1 && j0 < nk; j0 += kFoldUnroll * NT) {
        C pn[kFoldUnroll], ps[kFoldUnroll], qn[kFoldUnroll], qs[kFoldUnroll];
#pragma unroll
        for (int u = 0; u < kFoldUnroll; ++u) {
          const int j = j0 + u * NT;
          const int k = dgc.quo(j), c = dgc.rem(j, k);  // channel fastest: adjacent channels adjacent in memory
          if (j < nk) fold_load(gn, gs, k, c, pn[u], ps[u], qn[u], qs[u]);
        }
#pragma unroll
        for (int u = 0; u < kFoldUnroll; ++u) {
          const int j = j0 + u * NT;
          if (j >= nk) continue;
          const int k = dgc.quo(j), c = dgc.rem(j, k);
          C cn, cs;
          fold_sums(gn, gs, k, c, pn[u], ps[u], qn[u], qs[u], cn, cs);
          // conj(h) at k and at n - k, h = C_N + i C_S
          buf[lidx(c * n + k, pad)] = cmk<C>(cn.x - cs.y, -(cn.y + cs.x));
          if (k != 0 && 2 * k != n) buf[lidx(c * n + n - k, pad)] = cmk<C>(cn.x + cs.y, cn.y - cs.x);
        }
      }
      __syncthreads();
      ring_dft<T, NT>(tb, buf, tq, n, gc, pad, b0 != bg0);
    }
    // IDFT(h) = conj(F): f_N = F.x, f_S = -F.y; four consecutive pixels per
    // item (ring starts and lengths are multiples of 4 pixels)
    const int nq = n >> 2;
    const FastDiv dnq(nq);
    for (int q = tid; q < gc * nq; q += NT) {
      const int c = dnq.quo(q), jj = 4 * dnq.rem(q, c);
      const int j = c * n + jj;
      T fn[4], fs[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const C F = buf[lidx(j + e, pad)];
        fn[e] = F.x;
        fs[e] = -F.y;
      }
      const size_t r = (size_t)(b0 + c) * npix;
      if (sub) {
        // residual sub - S a of an iterative refinement (TOut = T)
        T sv[4];
        load4<T, TOut>(sub + r + sN + jj, sv);
#pragma unroll
        for (int e = 0; e < 4; ++e) fn[e] = sv[e] - fn[e];
        if (!equator) {
          load4<T, TOut>(sub + r + sS + jj, sv);
#pragma unroll
          for (int e = 0; e < 4; ++e) fs[e] = sv[e] - fs[e];
        }
      }
      store4<TOut, T>(map + r + sN + jj, fn);
      if (!equator) store4<TOut, T>(map + r + sS + jj, fs);
    }
    __syncthreads();
  }
}

// Launch geometry: channels per workgroup and LDS bytes.  One stage holds
// kFftThreads * kFftOutMax complex values in registers, which covers ring
// lengths up to 4 * 2048; Bluestein rings use convolution lengths M < 2 nside.
constexpr size_t kMaxLds = 160 * 1024;  // LDS of one gfx950 workgroup

static FftGeom fft_geometry_nt(int nside, int mmax_bs, int batch, size_t csize, int NT, size_t lds_limit) {
  FftGeom g{};
  const int nmax = 4 * nside;
  g.NT = NT;
  const int cap = g.NT * kFftOutMax;  // complex values one stage can hold
  int G = cap / nmax;
  const int lds_cap = (int)((72 * 1024) / (nmax * csize));
  if (G > lds_cap) G = lds_cap;
  if (G > batch) G = batch;
  if (G > 16) G = 16;
  if (G < 1) G = 1;
  g.G = G;
  size_t need = lds_elems((size_t)G * nmax);
  // octant root table of the largest power-of-two length used
  const int npow = mmax_bs > nmax ? mmax_bs : nmax;
  const size_t tqn = npow / 8 + 1;
  g.bs_nb = 4;
  if (mmax_bs > 0) {
    // Bluestein rings (i < nside): the most sub-transforms per FFT call that
    // one stage (cap values) and the LDS hold
    const size_t cs = mmax_bs + (mmax_bs >= kPadMin ? mmax_bs / 16 : 0);
    const size_t ylds1 = csize == 16 ? BsLayout<double>::kLdsY1 : BsLayout<float>::kLdsY1;
    size_t bs = 0;
    for (int nb = 4; nb >= 1; nb >>= 1) {
      const size_t ylds = nb == 4 ? 0 : nb == 2 ? 2 : ylds1;
      bs = ylds * (size_t)(nside - 1) + nb * cs;
      g.bs_nb = nb;
      if ((size_t)nb * mmax_bs <= (size_t)cap && ((bs > need ? bs : need) + tqn) * csize <= lds_limit) break;
    }
    if (bs > need) need = bs;
  }
  g.tq_off = (int)need;
  g.lds = (need + tqn) * csize;
  return g;
}

// FP64 transforms of 4 or more channels whose channel slice and Bluestein
// sub-transforms fit a 256-thread stage run 256-thread workgroups with at
// most half the LDS, two per CU (a 512-thread FP64 workgroup holds one
// channel of the longest ring in half its threads and, with the Bluestein
// buffers, most of the LDS: one workgroup per CU).  Measured at Nside 1024,
// B 16: forward 2.65 -> 2.50 ms, inverse 3.42 -> 2.91 ms; at one channel the
// Bluestein rings' sub-transforms one at a time made the inverse 8% slower,
// so smaller batches keep 512 threads.
FftGeom fft_geometry(int nside, int mmax_bs, int batch, size_t csize) {
  const FftGeom g = fft_geometry_nt(nside, mmax_bs, batch, csize, kFftThreads, kMaxLds);
  if (csize == 16 && batch >= 4 && (size_t)g.G * 4 * nside <= 256 * kFftOutMax && mmax_bs <= 256 * kFftOutMax) {
    const FftGeom h = fft_geometry_nt(nside, mmax_bs, batch, csize, 256, kMaxLds / 2);
    if (h.lds <= kMaxLds / 2 && h.G == g.G) return h;
  }
  return g;
}

inline unsigned fft_grid(int Rp, int B, int G) {
  const int ncg = (B + G - 1) / G;
  return 8u * (unsigned)((Rp + 7) / 8) * (unsigned)ncg;
}
// banded dealing (fft_work_banded): whole bands of kNestBand pairs per XCD
inline unsigned fft_grid_banded(int Rp, int B, int G) {
  const int ncg = (B + G - 1) / G;
  const int bands_per_xcd = (Rp + 8 * kNestBand - 1) / (8 * kNestBand);
  return 8u * (unsigned)(bands_per_xcd * kNestBand) * (unsigned)ncg;
}

template <typename K> hipError_t allow_lds(K kern, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename TIn, typename T, typename TS>
hipError_t launch_ring_fft_fwd(Tables tb, int B, const TIn *map, const double *wtab, double wscale,
                               const double *pixw, TS *XE, TS *XO, hipStream_t st, bool nested) {
  const FftGeom g = fft_geometry(tb.nside, tb.mmax_bs, B, sizeof(cplx<T>));
  if (g.lds > kMaxLds) return hipErrorInvalidValue;
  auto kern = nested ? k_ring_fft_fwd<TIn, T, TS, true, kFftThreads> : k_ring_fft_fwd<TIn, T, TS, false, kFftThreads>;
  if constexpr (sizeof(T) == 8) {
    if (g.NT == 256) kern = nested ? k_ring_fft_fwd<TIn, T, TS, true, 256> : k_ring_fft_fwd<TIn, T, TS, false, 256>;
  }
  hipError_t e = allow_lds(kern, g.lds);
  if (e != hipSuccess) return e;
  const unsigned grid = nested ? fft_grid_banded(tb.npairs, B, g.G) : fft_grid(tb.npairs, B, g.G);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(g.NT), g.lds, st, tb, B, g.G, g.tq_off, g.bs_nb, map, wtab, wscale,
                     pixw, XE, XO);
  return hipGetLastError();
}

template <typename TOut, typename T>
hipError_t launch_ring_fft_inv(Tables tb, int B, const cplx<T> *GN, const cplx<T> *GS, const TOut *sub, TOut *map,
                               hipStream_t st) {
  const FftGeom g = fft_geometry(tb.nside, tb.mmax_bs, B, sizeof(cplx<T>));
  if (g.lds > kMaxLds) return hipErrorInvalidValue;
  auto kern = k_ring_fft_inv<TOut, T, kFftThreads>;
  if constexpr (sizeof(T) == 8) {
    if (g.NT == 256) kern = k_ring_fft_inv<TOut, T, 256>;
  }
  hipError_t e = allow_lds(kern, g.lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(fft_grid(tb.npairs, B, g.G)), dim3(g.NT), g.lds, st, tb, B, g.G, g.tq_off,
                     g.bs_nb, GN, GS, sub, map);
  return hipGetLastError();
}

template hipError_t launch_ring_fft_fwd<double, double, double2>(Tables, int, const double *, const double *, double,
                                                                 const double *, double2 *, double2 *, hipStream_t,
                                                                 bool);
template hipError_t launch_ring_fft_fwd<float, float, float2>(Tables, int, const float *, const double *, double,
                                                              const double *, float2 *, float2 *, hipStream_t, bool);
template hipError_t launch_ring_fft_fwd<bf16_t, float, float2>(Tables, int, const bf16_t *, const double *, double,
                                                               const double *, float2 *, float2 *, hipStream_t, bool);
template hipError_t launch_ring_fft_fwd<bf16_t, float, uint32_t>(Tables, int, const bf16_t *, const double *,
                                                                 double, const double *, uint32_t *, uint32_t *,
                                                                 hipStream_t, bool);
template hipError_t launch_ring_fft_inv<double, double>(Tables, int, const double2 *, const double2 *,
                                                        const double *, double *, hipStream_t);
template hipError_t launch_ring_fft_inv<float, float>(Tables, int, const float2 *, const float2 *, const float *,
                                                      float *, hipStream_t);
template hipError_t launch_ring_fft_inv<bf16_t, float>(Tables, int, const float2 *, const float2 *, const bf16_t *,
                                                       bf16_t *, hipStream_t);

}  // namespace shtx
