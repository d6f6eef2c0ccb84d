// Conversion of maps between the RING pixel order the transforms use and the
// NESTED order of HEALPix (the hierarchical numbering of the definition the
// paper builds on, Sec. III-A; the paper benchmarks this remapping).
//
// NESTED index p = f N^2 + interleave(x, y): base pixel (face) f = 0..11,
// face coordinates 0 <= x, y < N with x in the even and y in the odd bit
// positions.  The face fixes the ring of the pixel and its slot in the ring:
//   ring  i = rf N - x - y - 1                    (rf = 2, 3, 4 for the north,
//                                                  equatorial and south faces)
//   slot  j = (qf n + x - y + 1 + s) / 2, 1-based, cyclic in 1 .. 4n
//         (qf = 1, 3, 5, 7 for polar faces and 0, 2, 4, 6 for equatorial
//          ones; n = i, 4N - i or N pixels per quadrant in the north cap,
//          south cap and belt; s = (i - N) mod 2 on the belt, 0 in the caps)
// and the RING index is the ring's first pixel plus j - 1.  nside is a power
// of two, so every step is a shift, a mask or an add: no division.
//
// One thread per NESTED pixel computes its RING index once and moves that
// pixel for every channel: the NESTED side of each channel is read or written
// by consecutive lanes (coalesced), the RING side is a gather (RING -> NESTED)
// or a scatter (NESTED -> RING) whose 64 lanes touch short runs of about 15
// rings.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/shtx.h"

namespace shtx {
namespace {

// bits 0, 2, 4, ... of v packed into bits 0, 1, 2, ...
__device__ __forceinline__ uint32_t compact_even_bits(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0f0f0f0fu;
  v = (v | (v >> 4)) & 0x00ff00ffu;
  v = (v | (v >> 8)) & 0x0000ffffu;
  return v;
}

__device__ __forceinline__ uint32_t nest_to_ring(uint32_t p, int lgn) {
  const int N = 1 << lgn;
  const uint32_t f = p >> (2 * lgn);
  const uint32_t ipf = p & ((1u << (2 * lgn)) - 1u);
  const int x = (int)compact_even_bits(ipf);
  const int y = (int)compact_even_bits(ipf >> 1);
  const int row = (int)(f >> 2);                 // 0 north, 1 equatorial, 2 south
  const int rf = row + 2;                        // ring of the face's northern corner / N
  const int qf = 2 * (int)(f & 3u) + (row != 1);  // longitude of the face centre / (pi/4)
  const int i = rf * N - x - y - 1;              // ring, 1 .. 4N-1
  const uint32_t npix = 12u << (2 * lgn);
  int n, shift;
  uint32_t start;
  if (i < N) {  // north cap
    n = i;
    shift = 0;
    start = 2u * (uint32_t)i * (uint32_t)(i - 1);
  } else if (i > 3 * N) {  // south cap
    n = 4 * N - i;
    shift = 0;
    start = npix - 2u * (uint32_t)n * (uint32_t)(n + 1);
  } else {  // belt
    n = N;
    shift = (i - N) & 1;
    start = 2u * (uint32_t)N * (uint32_t)(N - 1) + 4u * (uint32_t)N * (uint32_t)(i - N);
  }
  int j = (qf * n + x - y + 1 + shift) >> 1;
  if (j > 4 * n) j -= 4 * n;
  if (j < 1) j += 4 * n;
  return start + (uint32_t)(j - 1);
}

// to_ring: out[b][ring(p)] = in[b][p];  otherwise out[b][p] = in[b][ring(p)]
template <typename E, bool ToRing>
__global__ void __launch_bounds__(256) k_reorder(int lgn, int B, const E *__restrict__ in, E *__restrict__ out) {
  const uint32_t npix = 12u << (2 * lgn);
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= npix) return;
  const uint32_t r = nest_to_ring(p, lgn);
  const size_t src = ToRing ? p : r, dst = ToRing ? r : p;
  for (int b = 0; b < B; ++b) {
    const size_t o = (size_t)b * npix;
    out[o + dst] = in[o + src];
  }
}

int elem_bytes(int dtype) {
  return dtype == SHTX_F64 ? 8 : dtype == SHTX_F32 ? 4 : dtype == SHTX_BF16 ? 2 : 0;
}

template <bool ToRing>
int reorder(int nside, int batch, int dtype, const void *in, void *out, void *stream) {
  if (nside < 1 || nside > 8192 || (nside & (nside - 1)) || batch < 1) return SHTX_ERR_ARG;
  const int eb = elem_bytes(dtype);
  if (eb == 0 || !in || !out) return SHTX_ERR_ARG;
  if (((uintptr_t)in | (uintptr_t)out) % (uintptr_t)eb) return SHTX_ERR_ARG;
  const int lgn = __builtin_ctz((unsigned)nside);
  const uint64_t npix = 12ull << (2 * lgn);
  const uint64_t bytes = npix * (uint64_t)batch * (uint64_t)eb;
  const uintptr_t a = (uintptr_t)in, c = (uintptr_t)out;
  if (a < c + bytes && c < a + bytes) return SHTX_ERR_ARG;  // a permutation cannot run in place
  const dim3 grid((unsigned)((npix + 255) / 256));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (eb == 8)
    hipLaunchKernelGGL((k_reorder<uint64_t, ToRing>), grid, dim3(256), 0, st, lgn, batch,
                       static_cast<const uint64_t *>(in), static_cast<uint64_t *>(out));
  else if (eb == 4)
    hipLaunchKernelGGL((k_reorder<uint32_t, ToRing>), grid, dim3(256), 0, st, lgn, batch,
                       static_cast<const uint32_t *>(in), static_cast<uint32_t *>(out));
  else
    hipLaunchKernelGGL((k_reorder<uint16_t, ToRing>), grid, dim3(256), 0, st, lgn, batch,
                       static_cast<const uint16_t *>(in), static_cast<uint16_t *>(out));
  return hipGetLastError() == hipSuccess ? SHTX_OK : SHTX_ERR_HIP;
}

}  // namespace
}  // namespace shtx

extern "C" {

int shtx_nest2ring(int nside, int batch, int dtype, const void *map_nest, void *map_ring, void *stream) {
  return shtx::reorder<true>(nside, batch, dtype, map_nest, map_ring, stream);
}

int shtx_ring2nest(int nside, int batch, int dtype, const void *map_ring, void *map_nest, void *stream) {
  return shtx::reorder<false>(nside, batch, dtype, map_ring, map_nest, stream);
}

}  // extern "C"
