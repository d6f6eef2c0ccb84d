// Conversions between the caller's coefficient layout alm[b][idx(l,m)] and
// the transposed internal layout ALMT[idx(l,m)][b] of the Legendre kernels,
// with the per-coefficient scale factors of each entry point.
//
//   to caller:   alm = f_m * ALMT           (Im of m = 0 set to 0),
//                or alm += f_m * ALMT       (accumulating, iterative refinement)
//   from caller: ALMT = s * f_m * c_lm * alm (Im of m = 0 ignored)
//
// f_m is f0 for m = 0 and fm for m > 0; c_lm is the normalisation of the
// scaled recurrence (tables.hip) that the synthesis kernels expect folded in.
#include "common.h"

namespace shtx {

// One workgroup per (m, tile of l); LDS tile transposes [l][b] <-> [b][l].
constexpr int kTileL = 64;

template <typename T, typename TO>
__global__ void __launch_bounds__(256)
    k_alm_out(int L, int B, const cplx<T> *__restrict__ ALMT, cplx<TO> *__restrict__ alm, T f0, T fm, int acc) {
  using C = cplx<T>;
  using CO = cplx<TO>;
  __shared__ C tile[kTileL][17];
  const int m = blockIdx.y;
  const int l0 = m + blockIdx.x * kTileL;
  if (l0 > L) return;
  const int nl = min(kTileL, L + 1 - l0);
  const size_t base = alm_idx(l0, m, L);
  const size_t nalm = nalm_of(L);
  const T f = (m == 0) ? f0 : fm;
  for (int b0 = 0; b0 < B; b0 += 16) {
    const int nb = min(16, B - b0);
    for (int t = threadIdx.x; t < nl * nb; t += 256) {
      const int l = t / nb, b = t - l * nb;
      tile[l][b] = ALMT[(base + l) * B + b0 + b];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nl * nb; t += 256) {
      const int b = t / nl, l = t - b * nl;
      const C v = tile[l][b];
      CO o;
      o.x = (TO)(f * v.x);
      o.y = (m == 0) ? (TO)0 : (TO)(f * v.y);
      CO *dst = alm + (size_t)(b0 + b) * nalm + base + l;
      if (acc) {
        const CO prev = *dst;
        o.x += prev.x;
        o.y += prev.y;
      }
      *dst = o;
    }
    __syncthreads();
  }
}

template <typename T, typename TI>
__global__ void __launch_bounds__(256)
    k_alm_in(int L, int B, const cplx<TI> *__restrict__ alm, const double *__restrict__ coefC,
             cplx<T> *__restrict__ ALMT, double s, double f0, double fm) {
  using C = cplx<T>;
  __shared__ C tile[kTileL][17];
  const int m = blockIdx.y;
  const int l0 = m + blockIdx.x * kTileL;
  if (l0 > L) return;
  const int nl = min(kTileL, L + 1 - l0);
  const size_t base = alm_idx(l0, m, L);
  const size_t nalm = nalm_of(L);
  const double f = s * ((m == 0) ? f0 : fm);
  for (int b0 = 0; b0 < B; b0 += 16) {
    const int nb = min(16, B - b0);
    for (int t = threadIdx.x; t < nl * nb; t += 256) {
      const int b = t / nl, l = t - b * nl;
      const cplx<TI> v = alm[(size_t)(b0 + b) * nalm + base + l];
      const double g = f * coefC[base + l];
      C o;
      o.x = (T)(g * (double)v.x);
      o.y = (m == 0) ? (T)0 : (T)(g * (double)v.y);
      tile[l][b] = o;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nl * nb; t += 256) {
      const int l = t / nb, b = t - l * nb;
      ALMT[(base + l) * B + b0 + b] = tile[l][b];
    }
    __syncthreads();
  }
}

template <typename T, typename TO>
hipError_t launch_alm_out(int L, int B, const cplx<T> *ALMT, cplx<TO> *alm, double f0, double fm, int acc,
                          hipStream_t st) {
  const dim3 grid((L + 1 + kTileL - 1) / kTileL, L + 1);
  hipLaunchKernelGGL((k_alm_out<T, TO>), grid, dim3(256), 0, st, L, B, ALMT, alm, (T)f0, (T)fm, acc);
  return hipGetLastError();
}

template <typename T, typename TI>
hipError_t launch_alm_in(int L, int B, const cplx<TI> *alm, const double *coefC, cplx<T> *ALMT, double s,
                         double f0, double fm, hipStream_t st) {
  const dim3 grid((L + 1 + kTileL - 1) / kTileL, L + 1);
  hipLaunchKernelGGL((k_alm_in<T, TI>), grid, dim3(256), 0, st, L, B, alm, coefC, ALMT, s, f0, fm);
  return hipGetLastError();
}

template hipError_t launch_alm_out<double, double>(int, int, const double2 *, double2 *, double, double, int,
                                                   hipStream_t);
template hipError_t launch_alm_out<float, float>(int, int, const float2 *, float2 *, double, double, int,
                                                 hipStream_t);
template hipError_t launch_alm_in<double, double>(int, int, const double2 *, const double *, double2 *, double,
                                                  double, double, hipStream_t);
template hipError_t launch_alm_in<float, float>(int, int, const float2 *, const double *, float2 *, double, double,
                                                double, hipStream_t);

}  // namespace shtx
