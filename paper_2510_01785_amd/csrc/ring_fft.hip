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

constexpr int kFftOutMax = 16;  // complex values per thread per stage

// LDS index of logical element o of the FFT work buffer: one padding slot
// every 16 elements, so that the stride-R writes of a Stockham stage (thread
// i writing elements R i + q) fall into different banks.
__device__ __forceinline__ int lp_idx(int o) { return o + (o >> 4); }
inline size_t lds_elems(size_t n) { return n + (n >> 4) + 1; }

// Twiddles of power-of-two transforms of length N come from an octant table
// in LDS, tq[r] = exp(-2 pi i r / N) for r = 0..N/8: for e = q N/4 + r,
// w^e = (-i)^q w^r, and for r > N/8, w^r = (sin phi, -cos phi) with
// (cos phi, -sin phi) = tq[N/4 - r].
template <typename C>
__device__ __forceinline__ C tw_quarter(const C *tq, int e, int lq /* log2(N/4) */) {
  const int q = e >> lq;
  const int r = e - (q << lq);
  const int h = (1 << lq) >> 1;
  C w;
  if (r <= h) {
    w = tq[r];
  } else {
    const C v = tq[(1 << lq) - r];
    w = cmk<C>(-v.y, -v.x);
  }
  switch (q & 3) {
    case 0: return w;
    case 1: return cmk<C>(w.y, -w.x);
    case 2: return cmk<C>(-w.x, -w.y);
    default: return cmk<C>(-w.y, w.x);
  }
}

// Root access of one stage: either a full table in global memory (any n)
// or an octant table in LDS (power-of-two n).
template <typename C> struct Roots {
  const C *tab;
  int lq;  // >= 0: octant table in LDS for length 4 << lq; < 0: full table
  __device__ __forceinline__ C operator()(int e) const { return lq >= 0 ? tw_quarter(tab, e, lq) : tab[e]; }
};

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

// Optional fused operations on the first stage's inputs / last stage's
// outputs of a power-of-two transform (Bluestein chirp products).
enum FuseIn { kInPlain = 0, kInChirp = 1 };        // x_j * c_j for j < nvalid, 0 beyond
enum FuseOut { kOutPlain = 0, kOutBhat = 1, kOutChirp = 2 };  // conj(y * bhat) / c_o * conj(y) / M

template <typename T> struct Fuse {
  const cplx<T> *chirp;
  const cplx<T> *bhat;
  int nvalid;
  T scale;
};

// Stockham stage of power-of-two radix R on G channels of length n (span p):
// butterfly i of channel c reads x[i + r n/R], twiddles by w^{r k n/(R p)}
// (k = i mod p), and writes y[R(i-k) + k + q p].  All inputs are read into
// registers before the workgroup barrier, so the buffer is updated in place.
template <typename T, int NT, int R, int fin, int fout>
__device__ __noinline__ void stage_pow2(cplx<T> *buf, int n, int G, int p, int lp, Roots<cplx<T>> roots,
                                        Fuse<T> fz) {
  using C = cplx<T>;
  constexpr int NB = kFftOutMax / R;
  const int Tq = n / R;
  const int nb = G * Tq;
  const int step = n >> (lp + __builtin_ctz(R));
  C v[NB][R];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = threadIdx.x + s * NT;
    if (b < nb) {
      const int c = b / Tq, i = b - c * Tq;
      const int k = i & (p - 1);
      const int xb = c * n + i;
      const int e = k * step;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        C u;
        if constexpr (fin == kInChirp) {
          const int j = i + r * Tq;
          u = (j < fz.nvalid) ? cmul(buf[lp_idx(xb + r * Tq)], fz.chirp[j]) : cmk<C>(0, 0);
        } else {
          u = buf[lp_idx(xb + r * Tq)];
        }
        v[s][r] = (r == 0) ? u : cmul(u, roots(r * e));
      }
      dftR<C, R>(v[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = threadIdx.x + s * NT;
    if (b < nb) {
      const int c = b / Tq, i = b - c * Tq;
      const int k = i & (p - 1);
      const int o0 = (i - k) * R + k;
      const int yb = c * n + o0;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        C val = v[s][q];
        const int o = o0 + q * p;
        if constexpr (fout == kOutBhat) {
          val = cconj(cmul(val, fz.bhat[o]));
        } else if constexpr (fout == kOutChirp) {
          if (o >= fz.nvalid) continue;
          const C cv = cconj(val);
          val = cmul(fz.chirp[o], cmk<C>(cv.x * fz.scale, cv.y * fz.scale));
        }
        buf[lp_idx(yb + q * p)] = val;
      }
    }
  }
  __syncthreads();
}

// Stage of odd radix R (span p): thread per output,
//   y[g pR + q p + k] = sum_r x[g p + k + r n/R] w^{r (n/(pR)) (k + q p)}.
// Used for R <= kMaxDirectPrime only.
template <typename T, int NT>
__device__ __noinline__ void stage_odd(cplx<T> *buf, int n, int G, int p, int R,
                                       const cplx<T> *__restrict__ roots) {
  using C = cplx<T>;
  const int tot = G * n;
  const int Tn = n / R;
  const int pR = p * R;
  const int step = n / pR;
  C out[kFftOutMax];
#pragma unroll
  for (int s = 0; s < kFftOutMax; ++s) {
    const int o = threadIdx.x + s * NT;
    if (o < tot) {
      const int c = o / n;
      const int oo = o - c * n;
      const int g = oo / pR;
      const int rr = oo - g * pR;
      const int q = rr / p;
      const int k = rr - q * p;
      const int xb = c * n + g * p + k;
      const int be = step * (k + q * p);
      C acc = buf[lp_idx(xb)];
      int e = be;
      for (int r = 1; r < R; ++r) {
        acc = cadd(acc, cmul(buf[lp_idx(xb + r * Tn)], roots[e]));
        e += be;
        if (e >= n) e -= n;
      }
      out[s] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < kFftOutMax; ++s) {
    const int o = threadIdx.x + s * NT;
    if (o < tot) buf[lp_idx(o)] = out[s];
  }
  __syncthreads();
}

// Stockham FFT of G channels of power-of-two length n (radix 16 stages and
// one radix 2/4/8 stage), twiddles from the LDS octant table tq; optional
// fused first-stage input and last-stage output operations.
template <typename T, int NT, int R>
__device__ __forceinline__ void stage_pow2_any(cplx<T> *buf, int n, int G, int p, int lp, Roots<cplx<T>> roots,
                                               int fin, int fout, const Fuse<T> &fz) {
  if (fin == kInChirp) {
    if (fout == kOutBhat) stage_pow2<T, NT, R, kInChirp, kOutBhat>(buf, n, G, p, lp, roots, fz);
    else stage_pow2<T, NT, R, kInChirp, kOutPlain>(buf, n, G, p, lp, roots, fz);
  } else if (fout == kOutBhat) {
    stage_pow2<T, NT, R, kInPlain, kOutBhat>(buf, n, G, p, lp, roots, fz);
  } else if (fout == kOutChirp) {
    stage_pow2<T, NT, R, kInPlain, kOutChirp>(buf, n, G, p, lp, roots, fz);
  } else {
    stage_pow2<T, NT, R, kInPlain, kOutPlain>(buf, n, G, p, lp, roots, fz);
  }
}

template <typename T, int NT>
__device__ __noinline__ void fft_pow2(cplx<T> *buf, int n, int G, const cplx<T> *tq, int fin, int fout,
                                      Fuse<T> fz) {
  const Roots<cplx<T>> roots{tq, __builtin_ctz(n) - 2};
  const int e2 = __builtin_ctz(n);
  const int nst = e2 / 4 + ((e2 & 3) ? 1 : 0);
  int p = 1, lp = 0, st = 0;
  // the remainder radix first
  const int rr = e2 & 3;
  if (rr) {
    const int fo = (st == nst - 1) ? fout : kOutPlain;
    if (rr == 1) stage_pow2_any<T, NT, 2>(buf, n, G, p, lp, roots, fin, fo, fz);
    else if (rr == 2) stage_pow2_any<T, NT, 4>(buf, n, G, p, lp, roots, fin, fo, fz);
    else stage_pow2_any<T, NT, 8>(buf, n, G, p, lp, roots, fin, fo, fz);
    p <<= rr;
    lp += rr;
    ++st;
  }
  while (st < nst) {
    const int fi = (st == 0) ? fin : kInPlain;
    const int fo = (st == nst - 1) ? fout : kOutPlain;
    stage_pow2_any<T, NT, 16>(buf, n, G, p, lp, roots, fi, fo, fz);
    p <<= 4;
    lp += 4;
    ++st;
  }
}

// Mixed-radix Stockham FFT of G channels of length n = 4i: radix-4 stages over
// the power-of-two part, one radix-2 stage if needed, then one direct stage
// per remaining odd prime factor (all <= kMaxDirectPrime on this path).
template <typename T, int NT>
__device__ void fft_mixed(cplx<T> *buf, int n, int G, const cplx<T> *__restrict__ roots) {
  const Roots<cplx<T>> rg{roots, -1};
  int rem = n, p = 1, lp = 0;
  const Fuse<T> fz{nullptr, nullptr, 0, (T)0};
  while ((rem & 3) == 0) {
    stage_pow2<T, NT, 4, kInPlain, kOutPlain>(buf, n, G, p, lp, rg, fz);
    p <<= 2;
    lp += 2;
    rem >>= 2;
  }
  if ((rem & 1) == 0) {
    stage_pow2<T, NT, 2, kInPlain, kOutPlain>(buf, n, G, p, lp, rg, fz);
    p <<= 1;
    lp += 1;
    rem >>= 1;
  }
  while (rem > 1) {
    int R = rem;
    for (int r = 3; r * r <= rem; r += 2)
      if (rem % r == 0) {
        R = r;
        break;
      }
    stage_odd<T, NT>(buf, n, G, p, R, roots);
    p *= R;
    rem /= R;
  }
}

// Bluestein DFT of one channel of length n (Eq. (17)-(23)): with the chirp
// c_j = exp(-i pi j^2/n), X_k = c_k sum_j (x_j c_j) conj(c_{k-j}); the
// convolution is done cyclically on the power-of-two length M >= 2n-1 with
// the precomputed transform bhat of conj(c) and two power-of-two FFTs in LDS
// (the inverse one through conjugation).  The chirp products, the zero
// padding and the product with bhat are fused into the first and last FFT
// stages.  On return buf[0..n) holds X.
template <typename T, int NT>
__device__ void fft_bluestein(cplx<T> *buf, int n, int M, const cplx<T> *__restrict__ chirp,
                              const cplx<T> *__restrict__ bhat, const cplx<T> *tq) {
  const Fuse<T> fz{chirp, bhat, n, (T)1 / (T)M};
  fft_pow2<T, NT>(buf, M, 1, tq, kInChirp, kOutBhat, fz);
  fft_pow2<T, NT>(buf, M, 1, tq, kInPlain, kOutChirp, fz);
}

// Octant root table of the power-of-two length N into LDS; the source is the
// root table of length N * rs.
template <typename T, int NT>
__device__ __forceinline__ void load_octant(cplx<T> *tq, const cplx<T> *__restrict__ src, int N, int rs) {
  for (int r = threadIdx.x; r <= N / 8; r += NT) tq[r] = src[r * rs];
}

// Forward DFT of gc channels of ring-pair p held in buf (channel-major);
// tq is LDS space for an octant root table.  Every thread of the workgroup
// calls this (it synchronises internally).
template <typename T, int NT>
__device__ __forceinline__ void ring_dft(const Tables &tb, int p, int M, cplx<T> *buf, cplx<T> *tq, int n, int gc,
                                         bool tq_ready) {
  if (M == 0) {
    const cplx<T> *roots = TabOf<T>::roots(tb) + roots_offset(n >> 2);
    if ((n & (n - 1)) == 0) {
      if (!tq_ready) {
        load_octant<T, NT>(tq, roots, n, 1);
        __syncthreads();
      }
      fft_pow2<T, NT>(buf, n, gc, tq, kInPlain, kOutPlain, Fuse<T>{nullptr, nullptr, 0, (T)0});
    } else {
      fft_mixed<T, NT>(buf, n, gc, roots);
    }
  } else {
    // Bluestein rings run one channel at a time (gc == 1)
    if (!tq_ready) {
      load_octant<T, NT>(tq, TabOf<T>::rootsP(tb), M, tb.mmax_bs / M);
      __syncthreads();
    }
    const size_t co = roots_offset(n >> 2);
    fft_bluestein<T, NT>(buf, n, M, TabOf<T>::chirp(tb) + co, TabOf<T>::bhat(tb) + tb.rp_bsoff[p], tq);
  }
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

template <typename TIn, typename T, int NT>
__global__ void __launch_bounds__(NT, (sizeof(T) == 4 && NT == 512) ? 4 : 1)
    k_ring_fft_fwd(Tables tb, int B, int G, int use_bs, int tq_off, const TIn *__restrict__ map,
                   const double *__restrict__ wtab, double wscale, cplx<T> *__restrict__ XE,
                   cplx<T> *__restrict__ XO) {
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
  const T w = (T)(wtab ? wtab[p] * wscale : wscale);
  const int num = tb.rp_p0n[p], den = tb.rp_p0d[p];
  const size_t npix = (size_t)tb.npix;
  const int Mbs = use_bs ? tb.rp_M[p] : 0;
  const int Gp = Mbs ? 1 : G;
  for (int b0 = bg0; b0 < bg1; b0 += Gp) {
    const int gc = min(Gp, bg1 - b0);
    for (int j = threadIdx.x; j < gc * n; j += NT) {
      const int c = j / n, jj = j - c * n;
      const TIn *row = map + (size_t)(b0 + c) * npix;
      const T fN = load_as<T, TIn>(row + sN + jj);
      const T fS = equator ? (T)0 : load_as<T, TIn>(row + sS + jj);
      buf[lp_idx(j)] = cmk<C>(fN + fS, fN - fS);
    }
    __syncthreads();
    ring_dft<T, NT>(tb, p, Mbs, buf, tq, n, gc, b0 != bg0);
    // E/O spectra for m = 0..L; one phase per m, channels contiguous
    for (int m = threadIdx.x; m < M; m += NT) {
      const int k = m % n;
      const int kc = (k == 0) ? 0 : n - k;
      const int red = (int)(((long long)m * num) % (2 * den));
      C ph = phase_pi<T>(red, den, (T)-1);
      ph.x *= w;
      ph.y *= w;
      const size_t o = ((size_t)p * M + m) * B + b0;
      for (int c = 0; c < gc; ++c) {
        const C Gk = buf[lp_idx(c * n + k)];
        const C Gc = buf[lp_idx(c * n + kc)];
        // U = DFT(fN+fS)[k] = (G[k] + conj(G[-k]))/2 ; V = DFT(fN-fS)[k] = (G[k] - conj(G[-k]))/(2i)
        const C U = cmk<C>((T)0.5 * (Gk.x + Gc.x), (T)0.5 * (Gk.y - Gc.y));
        const C V = cmk<C>((T)0.5 * (Gk.y + Gc.y), (T)0.5 * (Gc.x - Gk.x));
        XE[o + c] = cmul(ph, U);
        XO[o + c] = cmul(ph, V);
      }
    }
    __syncthreads();
  }
}

template <typename TOut, typename T, int NT>
__global__ void __launch_bounds__(NT, (sizeof(T) == 4 && NT == 512) ? 4 : 1)
    k_ring_fft_inv(Tables tb, int B, int G, int use_bs, int tq_off, const cplx<T> *__restrict__ GN,
                   const cplx<T> *__restrict__ GS, TOut *__restrict__ map) {
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
  const int num = tb.rp_p0n[p], den = tb.rp_p0d[p];
  const size_t npix = (size_t)tb.npix;
  const int Mbs = use_bs ? tb.rp_M[p] : 0;
  const int Gp = Mbs ? 1 : G;
  for (int b0 = bg0; b0 < bg1; b0 += Gp) {
    const int gc = min(Gp, bg1 - b0);
    for (int j = threadIdx.x; j < gc * n; j += NT) {
      const int k = j / gc, c = j - k * gc;  // channel fastest: adjacent channels adjacent in memory
      C cn = cmk<C>(0, 0), cs = cmk<C>(0, 0);
      // positive frequencies m = k (mod n)
      for (int m = k; m < M; m += n) {
        const int red = (int)(((long long)m * num) % (2 * den));
        const C ph = phase_pi<T>(red, den, (T)1);
        const size_t o = ((size_t)p * M + m) * B + b0 + c;
        C a = cmul(GN[o], ph);
        C b = equator ? cmk<C>(0, 0) : cmul(GS[o], ph);
        if (m == 0) {
          a.y = 0;
          b.y = 0;
        }
        cn = cadd(cn, a);
        cs = cadd(cs, b);
      }
      // negative frequencies -m = k (mod n), m >= 1, contribute conj(c_m)
      for (int m = (k == 0) ? n : n - k; m < M; m += n) {
        const int red = (int)(((long long)m * num) % (2 * den));
        const C ph = phase_pi<T>(red, den, (T)1);
        const size_t o = ((size_t)p * M + m) * B + b0 + c;
        const C a = cmul(GN[o], ph);
        const C b = equator ? cmk<C>(0, 0) : cmul(GS[o], ph);
        cn = cadd(cn, cconj(a));
        cs = cadd(cs, cconj(b));
      }
      // h = C_N + i C_S ; store conj(h) so that a forward DFT gives conj(IDFT(h))
      buf[lp_idx(c * n + k)] = cmk<C>(cn.x - cs.y, -(cn.y + cs.x));
    }
    __syncthreads();
    ring_dft<T, NT>(tb, p, Mbs, buf, tq, n, gc, b0 != bg0);
    for (int j = threadIdx.x; j < gc * n; j += NT) {
      const int c = j / n, jj = j - c * n;
      const C F = buf[lp_idx(j)];  // IDFT(h) = conj(F): f_N = F.x, f_S = -F.y
      TOut *row = map + (size_t)(b0 + c) * npix;
      store_as<TOut, T>(row + sN + jj, F.x);
      if (!equator) store_as<TOut, T>(row + sS + jj, -F.y);
    }
    __syncthreads();
  }
}

// Launch geometry: threads per workgroup, channels per mixed-radix group and
// LDS bytes.  One stage holds NT * kFftOutMax complex values in registers, so
// NT = 512 covers ring and Bluestein lengths up to 8192 without spilling; the
// 16384-point Bluestein transforms of FP32 at nside 2048 take NT = 1024.
// Bluestein rings need M complex values of LDS; where that does not fit
// 128 KB (FP64 at nside 2048) every ring takes the mixed-radix path
// (use_bs = 0).
constexpr size_t kMaxLds = 160 * 1024;  // LDS of one gfx950 workgroup

template <typename T> int fft_threads(const Tables &tb) {
  const int need = (4 * tb.nside > tb.mmax_bs) ? 4 * tb.nside : tb.mmax_bs;
  return (sizeof(T) == 4 && need > 512 * kFftOutMax) ? 1024 : 512;
}

template <typename T> bool fft_geometry(const Tables &tb, int B, int NT, int *G, size_t *lds, int *tq_off) {
  const int nmax = 4 * tb.nside;
  const int cap = NT * kFftOutMax;  // complex values one stage can hold
  int g = cap / nmax;
  const int lds_cap = (int)((72 * 1024) / (nmax * sizeof(cplx<T>)));
  if (g > lds_cap) g = lds_cap;
  if (g > B) g = B;
  if (g > 16) g = 16;
  if (g < 1) g = 1;
  *G = g;
  size_t need = (size_t)g * nmax;
  const bool use_bs = tb.mmax_bs > 0 && tb.mmax_bs <= cap &&
                      (lds_elems(tb.mmax_bs) + tb.mmax_bs / 8 + 1) * sizeof(cplx<T>) <= kMaxLds;
  if (use_bs && (size_t)tb.mmax_bs > need) need = tb.mmax_bs;
  // quarter root table of the largest power-of-two length used
  const int npow = use_bs && tb.mmax_bs > nmax ? tb.mmax_bs : nmax;
  *tq_off = (int)lds_elems(need);
  *lds = (lds_elems(need) + npow / 8 + 1) * sizeof(cplx<T>);
  return use_bs;
}

inline unsigned fft_grid(int Rp, int B, int G) {
  const int ncg = (B + G - 1) / G;
  return 8u * (unsigned)((Rp + 7) / 8) * (unsigned)ncg;
}

template <typename K> hipError_t allow_lds(K kern, size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename TIn, typename T>
hipError_t launch_ring_fft_fwd(Tables tb, int B, const TIn *map, const double *wtab, double wscale, cplx<T> *XE,
                               cplx<T> *XO, hipStream_t st) {
  const int NT = fft_threads<T>(tb);
  int G, tq_off;
  size_t lds;
  const int use_bs = fft_geometry<T>(tb, B, NT, &G, &lds, &tq_off) ? 1 : 0;
  const dim3 grid(fft_grid(tb.npairs, B, G));
  if (NT == 512) {
    auto kern = k_ring_fft_fwd<TIn, T, 512>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(512), lds, st, tb, B, G, use_bs, tq_off, map, wtab, wscale, XE, XO);
  } else {
    auto kern = k_ring_fft_fwd<TIn, T, 1024>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(1024), lds, st, tb, B, G, use_bs, tq_off, map, wtab, wscale, XE, XO);
  }
  return hipGetLastError();
}

template <typename TOut, typename T>
hipError_t launch_ring_fft_inv(Tables tb, int B, const cplx<T> *GN, const cplx<T> *GS, TOut *map, hipStream_t st) {
  const int NT = fft_threads<T>(tb);
  int G, tq_off;
  size_t lds;
  const int use_bs = fft_geometry<T>(tb, B, NT, &G, &lds, &tq_off) ? 1 : 0;
  const dim3 grid(fft_grid(tb.npairs, B, G));
  if (NT == 512) {
    auto kern = k_ring_fft_inv<TOut, T, 512>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(512), lds, st, tb, B, G, use_bs, tq_off, GN, GS, map);
  } else {
    auto kern = k_ring_fft_inv<TOut, T, 1024>;
    hipError_t e = allow_lds(kern, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(1024), lds, st, tb, B, G, use_bs, tq_off, GN, GS, map);
  }
  return hipGetLastError();
}

template hipError_t launch_ring_fft_fwd<double, double>(Tables, int, const double *, const double *, double,
                                                        double2 *, double2 *, hipStream_t);
template hipError_t launch_ring_fft_fwd<float, float>(Tables, int, const float *, const double *, double, float2 *,
                                                      float2 *, hipStream_t);
template hipError_t launch_ring_fft_fwd<bf16_t, float>(Tables, int, const bf16_t *, const double *, double,
                                                       float2 *, float2 *, hipStream_t);
template hipError_t launch_ring_fft_inv<double, double>(Tables, int, const double2 *, const double2 *, double *,
                                                        hipStream_t);
template hipError_t launch_ring_fft_inv<float, float>(Tables, int, const float2 *, const float2 *, float *,
                                                      hipStream_t);
template hipError_t launch_ring_fft_inv<bf16_t, float>(Tables, int, const float2 *, const float2 *, bf16_t *,
                                                       hipStream_t);

}  // namespace shtx
