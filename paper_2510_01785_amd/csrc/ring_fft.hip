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

// Stage of radix 4 (span p, a power of two): butterfly i of channel c reads
// x[i + r n/4] (r = 0..3), twiddles them by w^{r k n/(4p)} (k = i mod p) and
// writes y[4(i-k) + k + q p] = sum_r u_r (-i)^{qr}.  Roots are read as
// roots[e * rs] from a table of length n * rs.
template <typename T, int NT>
__device__ __forceinline__ void stage_r4(cplx<T> *buf, int n, int G, int p, int lp,
                                         const cplx<T> *__restrict__ roots, int rs) {
  using C = cplx<T>;
  constexpr int NB = kFftOutMax / 4;
  const int Tq = n >> 2;
  const int nb = G * Tq;
  const int step = (n >> (lp + 2)) * rs;
  C v[NB][4];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = threadIdx.x + s * NT;
    if (b < nb) {
      const int c = b / Tq, i = b - c * Tq;
      const int k = i & (p - 1);
      const C *x = buf + c * n + i;
      const int e = k * step;
      const C u0 = x[0];
      const C u1 = cmul(x[Tq], roots[e]);
      const C u2 = cmul(x[2 * Tq], roots[2 * e]);
      const C u3 = cmul(x[3 * Tq], roots[3 * e]);
      const C s02 = cadd(u0, u2), d02 = csub(u0, u2);
      const C s13 = cadd(u1, u3), d13 = csub(u1, u3);
      v[s][0] = cadd(s02, s13);
      v[s][2] = csub(s02, s13);
      // -i * d13 = (d13.y, -d13.x)
      v[s][1] = cmk<C>(d02.x + d13.y, d02.y - d13.x);
      v[s][3] = cmk<C>(d02.x - d13.y, d02.y + d13.x);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = threadIdx.x + s * NT;
    if (b < nb) {
      const int c = b / Tq, i = b - c * Tq;
      const int k = i & (p - 1);
      C *y = buf + c * n + ((i - k) << 2) + k;
      y[0] = v[s][0];
      y[p] = v[s][1];
      y[2 * p] = v[s][2];
      y[3 * p] = v[s][3];
    }
  }
  __syncthreads();
}

// Stage of radix 2 (span p, a power of two).
template <typename T, int NT>
__device__ __forceinline__ void stage_r2(cplx<T> *buf, int n, int G, int p, int lp,
                                         const cplx<T> *__restrict__ roots, int rs) {
  using C = cplx<T>;
  constexpr int NB = kFftOutMax / 2;
  const int Th = n >> 1;
  const int nb = G * Th;
  const int step = (n >> (lp + 1)) * rs;
  C v[NB][2];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = threadIdx.x + s * NT;
    if (b < nb) {
      const int c = b / Th, i = b - c * Th;
      const int k = i & (p - 1);
      const C *x = buf + c * n + i;
      const C u0 = x[0];
      const C u1 = cmul(x[Th], roots[k * step]);
      v[s][0] = cadd(u0, u1);
      v[s][1] = csub(u0, u1);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = threadIdx.x + s * NT;
    if (b < nb) {
      const int c = b / Th, i = b - c * Th;
      const int k = i & (p - 1);
      C *y = buf + c * n + ((i - k) << 1) + k;
      y[0] = v[s][0];
      y[p] = v[s][1];
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
      const C *x = buf + c * n + g * p + k;
      const int be = step * (k + q * p);
      C acc = x[0];
      int e = be;
      for (int r = 1; r < R; ++r) {
        acc = cadd(acc, cmul(x[r * Tn], roots[e]));
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
    if (o < tot) buf[o] = out[s];
  }
  __syncthreads();
}

// Radix-4/2 Stockham FFT of G channels of power-of-two length n.
template <typename T, int NT>
__device__ void fft_pow2(cplx<T> *buf, int n, int G, const cplx<T> *__restrict__ roots, int rs) {
  int rem = n, p = 1, lp = 0;
  while ((rem & 3) == 0) {
    stage_r4<T, NT>(buf, n, G, p, lp, roots, rs);
    p <<= 2;
    lp += 2;
    rem >>= 2;
  }
  if (rem == 2) stage_r2<T, NT>(buf, n, G, p, lp, roots, rs);
}

// Mixed-radix Stockham FFT of G channels of length n = 4i: radix-4 stages over
// the power-of-two part, one radix-2 stage if needed, then one direct stage
// per remaining odd prime factor (all <= kMaxDirectPrime on this path).
template <typename T, int NT>
__device__ void fft_mixed(cplx<T> *buf, int n, int G, const cplx<T> *__restrict__ roots) {
  int rem = n, p = 1, lp = 0;
  while ((rem & 3) == 0) {
    stage_r4<T, NT>(buf, n, G, p, lp, roots, 1);
    p <<= 2;
    lp += 2;
    rem >>= 2;
  }
  if ((rem & 1) == 0) {
    stage_r2<T, NT>(buf, n, G, p, lp, roots, 1);
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
// the precomputed transform bhat of conj(c) and two radix-4 FFTs in LDS (the
// inverse one through conjugation).  On return buf[0..n) holds X.
template <typename T, int NT>
__device__ void fft_bluestein(cplx<T> *buf, int n, int M, const cplx<T> *__restrict__ chirp,
                              const cplx<T> *__restrict__ bhat, const cplx<T> *__restrict__ rootsP, int rs) {
  using C = cplx<T>;
  for (int j = threadIdx.x; j < M; j += NT) buf[j] = (j < n) ? cmul(buf[j], chirp[j]) : cmk<C>(0, 0);
  __syncthreads();
  fft_pow2<T, NT>(buf, M, 1, rootsP, rs);
  for (int j = threadIdx.x; j < M; j += NT) buf[j] = cconj(cmul(buf[j], bhat[j]));
  __syncthreads();
  fft_pow2<T, NT>(buf, M, 1, rootsP, rs);
  const T inv = (T)1 / (T)M;
  for (int j = threadIdx.x; j < n; j += NT) {
    const C v = cconj(buf[j]);
    buf[j] = cmul(chirp[j], cmk<C>(v.x * inv, v.y * inv));
  }
  __syncthreads();
}

// Forward DFT of gc channels of ring-pair p held in buf (channel-major).
template <typename T, int NT>
__device__ __forceinline__ void ring_dft(const Tables &tb, int p, int M, cplx<T> *buf, int n, int gc) {
  if (M == 0) {
    fft_mixed<T, NT>(buf, n, gc, TabOf<T>::roots(tb) + roots_offset(n >> 2));
  } else {
    // Bluestein rings run one channel at a time (gc == 1)
    const size_t co = roots_offset(n >> 2);
    fft_bluestein<T, NT>(buf, n, M, TabOf<T>::chirp(tb) + co, TabOf<T>::bhat(tb) + tb.rp_bsoff[p],
                         TabOf<T>::rootsP(tb), tb.mmax_bs / M);
  }
}

template <typename TIn, typename T, int NT>
__global__ void __launch_bounds__(NT)
    k_ring_fft_fwd(Tables tb, int B, int G, int use_bs, const TIn *__restrict__ map,
                   const double *__restrict__ wtab, double wscale, cplx<T> *__restrict__ XE,
                   cplx<T> *__restrict__ XO) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf = reinterpret_cast<C *>(smem_raw);
  const int p = blockIdx.x;
  const int n = tb.rp_n[p];
  const int sN = tb.rp_sN[p], sS = tb.rp_sS[p];
  const bool equator = (sN == sS);
  const int L = tb.lmax, M = L + 1;
  const T w = (T)(wtab ? wtab[p] * wscale : wscale);
  const int num = tb.rp_p0n[p], den = tb.rp_p0d[p];
  const size_t npix = (size_t)tb.npix;
  const int Mbs = use_bs ? tb.rp_M[p] : 0;
  const int Gp = Mbs ? 1 : G;
  for (int b0 = 0; b0 < B; b0 += Gp) {
    const int gc = min(Gp, B - b0);
    for (int j = threadIdx.x; j < gc * n; j += NT) {
      const int c = j / n, jj = j - c * n;
      const TIn *row = map + (size_t)(b0 + c) * npix;
      const T fN = load_as<T, TIn>(row + sN + jj);
      const T fS = equator ? (T)0 : load_as<T, TIn>(row + sS + jj);
      buf[j] = cmk<C>(fN + fS, fN - fS);
    }
    __syncthreads();
    ring_dft<T, NT>(tb, p, Mbs, buf, n, gc);
    // E/O spectra for m = 0..L, channel fastest for contiguous stores
    for (int t = threadIdx.x; t < M * gc; t += NT) {
      const int m = t / gc, c = t - m * gc;
      const int k = m % n;
      const int kc = (k == 0) ? 0 : n - k;
      const C Gk = buf[c * n + k];
      const C Gc = buf[c * n + kc];
      // U = DFT(fN+fS)[k] = (G[k] + conj(G[-k]))/2 ; V = DFT(fN-fS)[k] = (G[k] - conj(G[-k]))/(2i)
      const C U = cmk<C>((T)0.5 * (Gk.x + Gc.x), (T)0.5 * (Gk.y - Gc.y));
      const C V = cmk<C>((T)0.5 * (Gk.y + Gc.y), (T)0.5 * (Gc.x - Gk.x));
      const int red = (int)(((long long)m * num) % (2 * den));
      C ph = phase_pi<T>(red, den, (T)-1);
      ph.x *= w;
      ph.y *= w;
      const size_t o = ((size_t)p * M + m) * B + b0 + c;
      XE[o] = cmul(ph, U);
      XO[o] = cmul(ph, V);
    }
    __syncthreads();
  }
}

template <typename TOut, typename T, int NT>
__global__ void __launch_bounds__(NT)
    k_ring_fft_inv(Tables tb, int B, int G, int use_bs, const cplx<T> *__restrict__ GN,
                   const cplx<T> *__restrict__ GS, TOut *__restrict__ map) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C *buf = reinterpret_cast<C *>(smem_raw);
  const int p = blockIdx.x;
  const int n = tb.rp_n[p];
  const int sN = tb.rp_sN[p], sS = tb.rp_sS[p];
  const bool equator = (sN == sS);
  const int L = tb.lmax, M = L + 1;
  const int num = tb.rp_p0n[p], den = tb.rp_p0d[p];
  const size_t npix = (size_t)tb.npix;
  const int Mbs = use_bs ? tb.rp_M[p] : 0;
  const int Gp = Mbs ? 1 : G;
  for (int b0 = 0; b0 < B; b0 += Gp) {
    const int gc = min(Gp, B - b0);
    for (int j = threadIdx.x; j < gc * n; j += NT) {
      const int c = j / n, k = j - c * n;
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
      buf[j] = cmk<C>(cn.x - cs.y, -(cn.y + cs.x));
    }
    __syncthreads();
    ring_dft<T, NT>(tb, p, Mbs, buf, n, gc);
    for (int j = threadIdx.x; j < gc * n; j += NT) {
      const int c = j / n, jj = j - c * n;
      const C F = buf[j];  // IDFT(h) = conj(F): f_N = F.x, f_S = -F.y
      TOut *row = map + (size_t)(b0 + c) * npix;
      store_as<TOut, T>(row + sN + jj, F.x);
      if (!equator) store_as<TOut, T>(row + sS + jj, -F.y);
    }
    __syncthreads();
  }
}

// Launch geometry: threads per workgroup, channels per mixed-radix group and
// LDS bytes.  Bluestein rings need M complex values of LDS; precisions or
// sizes where that does not fit 128 KB (FP64 at nside 2048) take the
// mixed-radix path for every ring (use_bs = 0).
template <typename T> struct FftCfg {
  static constexpr int NT = sizeof(T) == 8 ? 512 : 1024;
};

template <typename T> bool fft_geometry(const Tables &tb, int B, int *G, size_t *lds) {
  constexpr int NT = FftCfg<T>::NT;
  const int nmax = 4 * tb.nside;
  const int cap = NT * kFftOutMax;  // complex values one stage can hold
  int g = cap / nmax;
  const int lds_cap = (64 * 1024) / (int)(nmax * sizeof(cplx<T>));
  if (g > lds_cap) g = lds_cap;
  if (g > B) g = B;
  if (g > 16) g = 16;
  if (g < 1) g = 1;
  *G = g;
  size_t need = (size_t)g * nmax;
  const bool use_bs = tb.mmax_bs > 0 && tb.mmax_bs <= cap && (size_t)tb.mmax_bs * sizeof(cplx<T>) <= 128 * 1024;
  if (use_bs && (size_t)tb.mmax_bs > need) need = tb.mmax_bs;
  *lds = need * sizeof(cplx<T>);
  return use_bs;
}

template <typename TIn, typename T>
hipError_t launch_ring_fft_fwd(Tables tb, int B, const TIn *map, const double *wtab, double wscale, cplx<T> *XE,
                               cplx<T> *XO, hipStream_t st) {
  constexpr int NT = FftCfg<T>::NT;
  int G;
  size_t lds;
  const int use_bs = fft_geometry<T>(tb, B, &G, &lds) ? 1 : 0;
  auto kern = k_ring_fft_fwd<TIn, T, NT>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(tb.npairs), dim3(NT), lds, st, tb, B, G, use_bs, map, wtab, wscale, XE, XO);
  return hipGetLastError();
}

template <typename TOut, typename T>
hipError_t launch_ring_fft_inv(Tables tb, int B, const cplx<T> *GN, const cplx<T> *GS, TOut *map, hipStream_t st) {
  constexpr int NT = FftCfg<T>::NT;
  int G;
  size_t lds;
  const int use_bs = fft_geometry<T>(tb, B, &G, &lds) ? 1 : 0;
  auto kern = k_ring_fft_inv<TOut, T, NT>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(tb.npairs), dim3(NT), lds, st, tb, B, G, use_bs, GN, GS, map);
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
