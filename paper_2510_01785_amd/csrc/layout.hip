// Conversion of the caller's coefficient layout alm[b][idx(l,m)] into the
// transposed internal layout of the synthesis Legendre kernels, ALMT[idx][b]
// per channel group (chan_group), with the per-coefficient scale factors of
// each entry point:
//
//   ALMT = s * f_m * c_lm * alm   (Im of m = 0 ignored)
//
// f_m is f0 for m = 0 and fm for m > 0; c_lm is the normalisation of the
// scaled recurrence (tables.hip) that the synthesis kernels expect folded in.
// (The analysis kernels write the caller's layout themselves.)
#include "common.h"

namespace shtx {

// A workgroup takes kLayoutThreads consecutive coefficient indices idx(l, m)
// (m = 0 exactly for idx <= lmax) and 16 channels at a time, through an LDS
// tile: the caller side alm[b][idx] is read along idx and the internal side
// written as contiguous runs of each channel group, both coalesced.
constexpr int kLayoutThreads = 256;

template <typename T, typename TI>
__global__ void __launch_bounds__(kLayoutThreads)
    k_alm_in(int L, int B, int gmax, const cplx<TI> *__restrict__ alm, const double *__restrict__ coefC,
             cplx<T> *__restrict__ ALMT, double s, double f0, double fm) {
  using C = cplx<T>;
  __shared__ C tile[kLayoutThreads][17];
  const size_t nalm = nalm_of(L);
  const size_t i0 = (size_t)blockIdx.x * kLayoutThreads;
  const int ni = (int)min((size_t)kLayoutThreads, nalm - i0);
  const int t = threadIdx.x;
  const size_t idx = i0 + t;
  const bool m0 = idx <= (size_t)L;
  const double g = t < ni ? s * (m0 ? f0 : fm) * coefC[idx] : 0.0;
  for (int b0 = 0; b0 < B; b0 += 16) {
    const int nb = min(16, B - b0);
    if (t < ni) {
      for (int b = 0; b < nb; ++b) {
        const cplx<TI> v = alm[(size_t)(b0 + b) * nalm + idx];
        C o;
        o.x = (T)(g * (double)v.x);
        o.y = m0 ? (T)0 : (T)(g * (double)v.y);
        tile[t][b] = o;
      }
    }
    __syncthreads();
    if (gmax == B && nb == 16) {
      // one group of all channels, a full slice of 16: row i0 + r of the
      // [idx][B] layout gets channels b0 .. b0 + 15 (shifts, no division)
      C *dst = ALMT + i0 * (size_t)B + b0;
      for (int q = t; q < ni * 16; q += kLayoutThreads) dst[(size_t)(q >> 4) * B + (q & 15)] = tile[q >> 4][q & 15];
    } else {
      for (int q = t; q < ni * nb; q += kLayoutThreads) {
        const int r = q / nb, b = q - r * nb;
        const ChanGroup gr = chan_group(b0 + b, B, gmax);
        ALMT[(size_t)gr.g0 * (nalm + kCoefPad) + (i0 + r) * gr.w + (b0 + b - gr.g0)] = tile[r][b];
      }
    }
    __syncthreads();
  }
}

template <typename T, typename TI>
hipError_t launch_alm_in(int L, int B, int gmax, const cplx<TI> *alm, const double *coefC, cplx<T> *ALMT,
                         double s, double f0, double fm, hipStream_t st) {
  const dim3 grid((unsigned)((nalm_of(L) + kLayoutThreads - 1) / kLayoutThreads));
  hipLaunchKernelGGL((k_alm_in<T, TI>), grid, dim3(kLayoutThreads), 0, st, L, B, gmax, alm, coefC, ALMT, s, f0,
                     fm);
  return hipGetLastError();
}

template hipError_t launch_alm_in<double, double>(int, int, int, const double2 *, const double *, double2 *,
                                                  double, double, double, hipStream_t);
template hipError_t launch_alm_in<float, float>(int, int, int, const float2 *, const double *, float2 *, double,
                                                double, double, hipStream_t);

}  // namespace shtx
