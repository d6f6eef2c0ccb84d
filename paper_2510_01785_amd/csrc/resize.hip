// Spectral resize: coefficients of band limit lmax_in re-expressed at band
// limit lmax_out, a_lm kept for l <= min(lmax_in, lmax_out) and zero for
// lmax_in < l <= lmax_out.  With the transforms this changes the resolution
// of a band-limited field (analysis at one nside, resize, synthesis at
// another) without leaving the device.
//
// The caller's layout alm[b][idx(l, m)], idx = m (2 lmax + 1 - m) / 2 + l,
// stores each m as one contiguous column l = m .. lmax, so a workgroup copies
// one (m, channel) column from the input to the output layout: both sides are
// contiguous runs.  Complex elements are copied bit for bit.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/shtx.h"

namespace shtx {
namespace {

template <typename E>
__global__ void __launch_bounds__(256) k_alm_resize(int lin, int lout, int B, const E *__restrict__ in,
                                                    E *__restrict__ out) {
  const int m = blockIdx.x;  // 0 .. lout
  const size_t nin = (size_t)(lin + 1) * (lin + 2) / 2, nout = (size_t)(lout + 1) * (lout + 2) / 2;
  // column starts (an input column exists only for m <= lin)
  const size_t cin = m <= lin ? (size_t)m * (2 * lin + 1 - m) / 2 : 0, cout = (size_t)m * (2 * lout + 1 - m) / 2;
  const int lkeep = lin < lout ? lin : lout;  // rows copied; the rest of the column is zero
  for (int b = blockIdx.y; b < B; b += gridDim.y) {
    const E *src = in + (size_t)b * nin + cin;
    E *dst = out + (size_t)b * nout + cout;
    for (int l = m + (int)threadIdx.x; l <= lout; l += 256) dst[l] = l <= lkeep ? src[l] : E{};
  }
}

}  // namespace
}  // namespace shtx

extern "C" int shtx_alm_resize(int lmax_in, int lmax_out, int batch, int dtype, const void *alm_in, void *alm_out,
                               void *stream) {
  if (lmax_in < 0 || lmax_out < 0 || lmax_in > 8191 || lmax_out > 8191 || batch < 1) return SHTX_ERR_ARG;
  if (dtype != SHTX_F64 && dtype != SHTX_F32) return SHTX_ERR_ARG;
  if (!alm_in || !alm_out) return SHTX_ERR_ARG;
  const uint64_t eb = dtype == SHTX_F64 ? 16 : 8;  // complex element
  const uintptr_t a = (uintptr_t)alm_in, c = (uintptr_t)alm_out;
  if ((a | c) % eb) return SHTX_ERR_ARG;
  const uint64_t bin = (uint64_t)(lmax_in + 1) * (lmax_in + 2) / 2 * batch * eb;
  const uint64_t bout = (uint64_t)(lmax_out + 1) * (lmax_out + 2) / 2 * batch * eb;
  if (a < c + bout && c < a + bin) return SHTX_ERR_ARG;  // input and output overlap
  const dim3 grid(lmax_out + 1, batch < 65535 ? batch : 65535);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (eb == 16)
    hipLaunchKernelGGL(shtx::k_alm_resize<uint4>, grid, dim3(256), 0, st, lmax_in, lmax_out, batch,
                       static_cast<const uint4 *>(alm_in), static_cast<uint4 *>(alm_out));
  else
    hipLaunchKernelGGL(shtx::k_alm_resize<uint2>, grid, dim3(256), 0, st, lmax_in, lmax_out, batch,
                       static_cast<const uint2 *>(alm_in), static_cast<uint2 *>(alm_out));
  return hipGetLastError() == hipSuccess ? SHTX_OK : SHTX_ERR_HIP;
}
