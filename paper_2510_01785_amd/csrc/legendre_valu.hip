// Legendre step on the vector ALUs: the FP64 recurrence of Eq. (16) (run on
// mu_l = lambda_l / c_l, see tables.hip) fused with the contraction of
// Eq. (14)/(26) (analysis) or Eq. (24) (synthesis), using the north/south
// parity fold: a ring pair contributes lambda_lm(z) E_m for even l-m and
// lambda_lm(z) O_m for odd l-m to a_lm; conversely the synthesis sums
// S_e = sum_{l-m even} lambda a, S_o = sum_{l-m odd} lambda a give
// g_N = S_e + S_o and g_S = S_e - S_o.
//
// These kernels serve any batch size and both FP64 and FP32 contraction.
// Each ring starts at its stored seed l_s (a multiple of 8 above m, below
// which |lambda_lm| < 2^-64) and runs to lmax.
#include "common.h"

namespace shtx {

constexpr int kChunk = kAlign;  // l values per reduction round (8)

// Sum over the 64 lanes of a wave of 8 per-lane values v[0..7]; afterwards
// lane L holds the total of v[(L>>5&1)*4 + (L>>4&1)*2 + (L>>3&1)].
template <typename T> __device__ __forceinline__ T wave_reduce_scatter8(const T (&v)[8]) {
  const int lane = threadIdx.x & 63;
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
  T w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T send = b5 ? v[q] : v[q + 4];
    const T keep = b5 ? v[q + 4] : v[q];
    w[q] = keep + __shfl_xor(send, 32);
  }
  T u[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const T send = b4 ? w[q] : w[q + 2];
    const T keep = b4 ? w[q + 2] : w[q];
    u[q] = keep + __shfl_xor(send, 16);
  }
  T t = (b3 ? u[1] : u[0]) + __shfl_xor(b3 ? u[0] : u[1], 8);
  t += __shfl_xor(t, 4);
  t += __shfl_xor(t, 2);
  t += __shfl_xor(t, 1);
  return t;
}

// Analysis: one workgroup per m (balanced order: m = blockIdx.x gives the
// longest rows first), NT threads, each owning up to RPT ring pairs
// p = tid + NT*j, with the pair's E/O spectra for BG channels in registers.
// Per chunk of 8 l's every lane accumulates its rings' contributions, the
// wave reduces them with a reduce-scatter, and the waves' totals are summed
// through LDS.  Output: ALMT[idx(l,m)][b] = c_lm * sum_p mu_lm(p) X(p).
template <typename T, int BG, int NT, int RPT>
__global__ void __launch_bounds__(NT)
    k_legendre_fwd_valu(Tables tb, int B, int b0, const cplx<T> *__restrict__ XE,
                        const cplx<T> *__restrict__ XO, cplx<T> *__restrict__ ALMT) {
  using C = cplx<T>;
  constexpr int NW = NT / 64;
  __shared__ C red[2][kChunk][BG][NW];
  const int m = blockIdx.x;
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double *A = tb.coefA + alm_idx(m, m, L) - m;
  const double *Cn = tb.coefC + alm_idx(m, m, L) - m;

  double z[RPT], prv[RPT], cur[RPT];
  int ls[RPT];
  double2 sd[RPT];
  C xe[RPT][BG], xo[RPT][BG];
  int lmin = L + 1;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    const int p = tid + NT * j;
    prv[j] = 0.0;
    cur[j] = 0.0;
    if (p < Rp) {
      z[j] = tb.rp_z[p];
      ls[j] = tb.seed_l[(size_t)m * Rp + p];
      sd[j] = tb.seed_v[(size_t)m * Rp + p];
#pragma unroll
      for (int b = 0; b < BG; ++b) {
        const bool ok = (b0 + b) < B;
        const size_t o = ((size_t)p * M + m) * B + b0 + b;
        xe[j][b] = ok ? XE[o] : cmk<C>(0, 0);
        xo[j][b] = ok ? XO[o] : cmk<C>(0, 0);
      }
    } else {
      z[j] = 0.0;
      ls[j] = L + 1;
      sd[j] = make_double2(0.0, 0.0);
#pragma unroll
      for (int b = 0; b < BG; ++b) xe[j][b] = xo[j][b] = cmk<C>(0, 0);
    }
    lmin = min(lmin, ls[j]);
  }
  // first chunk any ring of the workgroup needs
  __shared__ int s_lmin;
  if (tid == 0) s_lmin = L + 1;
  __syncthreads();
  atomicMin(&s_lmin, lmin);
  __syncthreads();
  const int l_begin = s_lmin;

  int buf = 0;
  for (int l0 = l_begin; l0 <= L; l0 += kChunk) {
    T acc[kChunk][BG][2];
#pragma unroll
    for (int c = 0; c < kChunk; ++c)
#pragma unroll
      for (int b = 0; b < BG; ++b) acc[c][b][0] = acc[c][b][1] = (T)0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      if (ls[j] > l0 + kChunk - 1) continue;  // not started within this chunk
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        const int l = l0 + c;
        if (l > L) break;
        if (l == ls[j]) {
          prv[j] = sd[j].x;
          cur[j] = sd[j].y;
        } else if (l > ls[j]) {
          const double nx = fma(A[l] * z[j], cur[j], -prv[j]);
          prv[j] = cur[j];
          cur[j] = nx;
        } else {
          continue;
        }
        const T mu = (T)cur[j];
        const bool odd = (l - m) & 1;
#pragma unroll
        for (int b = 0; b < BG; ++b) {
          const C x = odd ? xo[j][b] : xe[j][b];
          acc[c][b][0] += mu * x.x;
          acc[c][b][1] += mu * x.y;
        }
      }
    }
    // reduce each (b, re/im) over the wave, 8 l's at a time
#pragma unroll
    for (int b = 0; b < BG; ++b) {
      T vr[kChunk], vi[kChunk];
#pragma unroll
      for (int c = 0; c < kChunk; ++c) {
        vr[c] = acc[c][b][0];
        vi[c] = acc[c][b][1];
      }
      const T sr = wave_reduce_scatter8<T>(vr);
      const T si = wave_reduce_scatter8<T>(vi);
      if ((lane & 7) == 0) {
        const int c = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
        red[buf][c][b][wave] = cmk<C>(sr, si);
      }
    }
    __syncthreads();
    if (tid < kChunk * BG) {
      const int c = tid / BG, b = tid - c * BG;
      const int l = l0 + c;
      if (l <= L && b0 + b < B) {
        T sr = 0, si = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          sr += red[buf][c][b][w].x;
          si += red[buf][c][b][w].y;
        }
        const T cl = (T)Cn[l];
        ALMT[alm_idx(l, m, L) * B + b0 + b] = cmk<C>(cl * sr, cl * si);
      }
    }
    buf ^= 1;
  }
  // coefficients below the first seed are exactly zero contributions
  for (int l = m + tid; l < min(l_begin, L + 1); l += NT)
#pragma unroll
    for (int b = 0; b < BG; ++b)
      if (b0 + b < B) ALMT[alm_idx(l, m, L) * B + b0 + b] = cmk<C>(0, 0);
}

// Synthesis: one wave per workgroup = (m, 64 ring pairs), one ring pair per
// lane; every lane runs its ring's recurrence and accumulates S_e and S_o
// for BG channels itself (no reduction).  The lanes step through l together
// from the wave's earliest seed, 8 steps per group: seeds sit at l = m + 8j,
// so within a group l - m is even exactly at the even steps.  The recurrence
// coefficients and the coefficients a_l of the BG channels are wave-uniform
// and come through scalar loads (32-bit offsets into the constant address
// space).  Workgroups are dealt so that the 64-ring chunks of one m run on
// one XCD.
template <typename T, int BG>
__global__ void __launch_bounds__(64)
    k_legendre_inv_valu(Tables tb, int B, int b0, const cplx<T> *__restrict__ ALMT, SynLayout lay,
                        cplx<T> *__restrict__ GN, cplx<T> *__restrict__ GS) {
  using C = cplx<T>;
  typedef __attribute__((address_space(4))) const double cdouble;
  typedef __attribute__((address_space(4))) const T creal;
  const int L = tb.lmax, Rp = tb.npairs;
  const int nch = (Rp + 63) / 64;
  const int g = blockIdx.x;
  const int x = g & 7, q = g >> 3;
  const int m = x + 8 * (q / nch);
  const int chunk = q % nch;
  if (m > L) return;  // uniform
  const int j = threadIdx.x;
  const int p = chunk * 64 + j;
  const bool valid = p < Rp;
  const double z = valid ? tb.rp_z[p] : 0.0;
  const int ls = valid ? tb.seed_l[(size_t)m * Rp + p] : L + 1;
  const double2 sd = valid ? tb.seed_v[(size_t)m * Rp + p] : make_double2(0.0, 0.0);
  int wlv = ls;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) wlv = min(wlv, __shfl_xor(wlv, o));
  const int wl = __builtin_amdgcn_readfirstlane(wlv);
  const int aoff = m * (2 * L + 1 - m) / 2;  // alm_idx(m, m, L) - m
  const cdouble *A = (const cdouble *)tb.coefA + aoff;
  // a[l][b] (re, im) of this channel group: T index (aoff + l) * 2B + 2(b0 + b) + {0, 1}
  const creal *a = (const creal *)ALMT + (size_t)aoff * 2 * B + 2 * b0;
  const int arow = 2 * B;
  T se[BG][2], so[BG][2];
#pragma unroll
  for (int b = 0; b < BG; ++b) se[b][0] = se[b][1] = so[b][0] = so[b][1] = (T)0;
  double prv = 0.0, cur = 0.0;
#pragma unroll 1
  for (int lq = wl; lq <= L; lq += 8) {
    T lam[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double nx = fma(A[lq + u] * z, cur, -prv);  // coefficients padded past lmax (unused values)
      if (u == 0) {
        const bool inj = (lq == ls);
        prv = inj ? sd.x : cur;
        cur = inj ? sd.y : nx;
      } else {
        prv = cur;
        cur = nx;
      }
      lam[u] = (T)cur;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (lq + u > L) break;  // last group: rows past lmax (padding) are not read
      const creal *row = a + (size_t)(lq + u) * arow;
#pragma unroll
      for (int b = 0; b < BG; ++b) {
        const T ar = row[2 * b], ai = row[2 * b + 1];
        if (u & 1) {
          so[b][0] = fma(lam[u], ar, so[b][0]);
          so[b][1] = fma(lam[u], ai, so[b][1]);
        } else {
          se[b][0] = fma(lam[u], ar, se[b][0]);
          se[b][1] = fma(lam[u], ai, se[b][1]);
        }
      }
    }
  }
  if (!valid) return;
#pragma unroll
  for (int b = 0; b < BG; ++b) {
    if (b0 + b >= B) continue;
    const size_t o = lay.idx(p, b0 + b, m);
    GN[o] = cmk<C>(se[b][0] + so[b][0], se[b][1] + so[b][1]);
    GS[o] = cmk<C>(se[b][0] - so[b][0], se[b][1] - so[b][1]);
  }
}

template <typename T, int BG, int NT, int RPT>
static void launch_fwd_cfg(const Tables &tb, int B, int b0, const cplx<T> *XE, const cplx<T> *XO, cplx<T> *ALMT,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_legendre_fwd_valu<T, BG, NT, RPT>), dim3(tb.lmax + 1), dim3(NT), 0, st, tb, B, b0, XE, XO,
                     ALMT);
}

template <typename T>
hipError_t launch_legendre_fwd_valu(const Tables &tb, int B, const cplx<T> *XE, const cplx<T> *XO, cplx<T> *ALMT,
                                    hipStream_t st) {
  constexpr int BG = sizeof(T) == 8 ? 1 : 2;
  const int Rp = tb.npairs;
  for (int b0 = 0; b0 < B; b0 += BG) {
    if (Rp <= 64)
      launch_fwd_cfg<T, BG, 64, 1>(tb, B, b0, XE, XO, ALMT, st);
    else if (Rp <= 1024)
      launch_fwd_cfg<T, BG, 256, 4>(tb, B, b0, XE, XO, ALMT, st);
    else if (Rp <= 2048)
      launch_fwd_cfg<T, BG, 1024, 2>(tb, B, b0, XE, XO, ALMT, st);
    else
      launch_fwd_cfg<T, BG, 1024, 4>(tb, B, b0, XE, XO, ALMT, st);
  }
  return hipGetLastError();
}

template <typename T, int BG>
static void launch_inv_cfg(const Tables &tb, int B, int b0, const cplx<T> *ALMT, SynLayout lay, cplx<T> *GN,
                           cplx<T> *GS, hipStream_t st) {
  const int nch = (tb.npairs + 63) / 64;
  const int nm = (tb.lmax + 1 + 7) / 8;
  hipLaunchKernelGGL((k_legendre_inv_valu<T, BG>), dim3(8 * nm * nch), dim3(64), 0, st, tb, B, b0, ALMT, lay, GN,
                     GS);
}

// Channel groups of 4 (FP32) or 2 (FP64), then 2 and 1 for the rest: the
// recurrence is shared by a group, the groups' channels are never padding.
template <typename T>
hipError_t launch_legendre_inv_valu(const Tables &tb, int B, const cplx<T> *ALMT, SynLayout lay, cplx<T> *GN,
                                    cplx<T> *GS, hipStream_t st) {
  constexpr int BGMAX = sizeof(T) == 8 ? 2 : 4;
  int b0 = 0;
  for (; b0 + BGMAX <= B; b0 += BGMAX) launch_inv_cfg<T, BGMAX>(tb, B, b0, ALMT, lay, GN, GS, st);
  if (BGMAX == 4 && b0 + 2 <= B) {
    launch_inv_cfg<T, 2>(tb, B, b0, ALMT, lay, GN, GS, st);
    b0 += 2;
  }
  if (b0 < B) launch_inv_cfg<T, 1>(tb, B, b0, ALMT, lay, GN, GS, st);
  return hipGetLastError();
}

template hipError_t launch_legendre_fwd_valu<double>(const Tables &, int, const double2 *, const double2 *, double2 *,
                                                     hipStream_t);
template hipError_t launch_legendre_fwd_valu<float>(const Tables &, int, const float2 *, const float2 *, float2 *,
                                                    hipStream_t);
template hipError_t launch_legendre_inv_valu<double>(const Tables &, int, const double2 *, SynLayout, double2 *,
                                                     double2 *, hipStream_t);
template hipError_t launch_legendre_inv_valu<float>(const Tables &, int, const float2 *, SynLayout, float2 *,
                                                    float2 *, hipStream_t);

}  // namespace shtx
