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
// A workgroup takes a T x T square of one face (T = min(nside, 64)): its
// NESTED indices are one contiguous range, and each of its 2T - 1 diagonals
// x + y = const is one contiguous run of one ring in RING order (slot j grows
// by one as x - y grows by two; a run wraps at most once, at the ring's
// start).  A workgroup moves one (square, channel) through LDS: the NESTED
// side is copied as one contiguous block, the RING side by whole diagonals,
// lanes along the runs (two diagonals per wave step where they fit), so both
// sides are read and written in runs.
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

// bits 0, 1, 2, ... of v (v < 2^16) spread to bits 0, 2, 4, ...
__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {
  v &= 0x0000ffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

constexpr int kTileLog = 6;  // squares of up to 64 x 64 pixels

// ToRing: out (RING) <- in (NESTED); otherwise out (NESTED) <- in (RING)
// vec16: the NESTED side of every square is copied in 16-byte pieces (the
// host checks that the squares and both maps allow it)
template <typename E, bool ToRing>
__global__ void __launch_bounds__(256) k_reorder(int lgn, int lgt, int B, int vec16, const E *__restrict__ in,
                                                 E *__restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  E *tile = reinterpret_cast<E *>(smem_raw);  // T*T values in local NESTED order
  const int N = 1 << lgn, T = 1 << lgt, TT = T * T;
  const uint32_t npix = 12u << (2 * lgn);
  const int lq = 2 * (lgn - lgt);  // log2 of the squares per face
  const uint32_t blk = blockIdx.x;
  const uint32_t f = blk >> lq, q = blk & ((1u << lq) - 1u);
  const int X0 = (int)(compact_even_bits(q) << lgt), Y0 = (int)(compact_even_bits(q >> 1) << lgt);
  const uint32_t nest0 = (f << (2 * lgn)) + (q << (2 * lgt));
  const int row = (int)(f >> 2);
  const int rf = row + 2;                         // ring of the face's northern corner / N
  const int qf = 2 * (int)(f & 3u) + (row != 1);  // longitude of the face centre / (pi/4)
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  for (int b = blockIdx.y; b < B; b += gridDim.y) {  // one channel per workgroup (row of the grid)
    const size_t o = (size_t)b * npix;
    if (ToRing) {
      if (vec16) {
        const uint4 *src = reinterpret_cast<const uint4 *>(in + o + nest0);
        uint4 *t4 = reinterpret_cast<uint4 *>(tile);
        for (int e = tid; e < TT * (int)sizeof(E) / 16; e += 256) t4[e] = src[e];
      } else {
        for (int e = tid; e < TT; e += 256) tile[e] = in[o + nest0 + e];
      }
      __syncthreads();
    }
    // diagonals d = x + y of the square, lane k taking x = xmin(d) + k.  For
    // T = 64 the diagonals go in pairs of 64 pixels in all (d, 62 - d) and
    // (d, 190 - d), plus 31, 63 and 95 alone: 65 steps of one wave each;
    // smaller squares take one diagonal per step.
    const int nsteps = T == 64 ? 65 : 2 * T - 1;
    for (int st = w; st < nsteps; st += 4) {
      int da = st, db = -1;
      if (T == 64) {
        if (st < 31) {
          db = 62 - st;
        } else if (st == 32) {
          da = 63;
        } else if (st > 32 && st < 64) {
          da = st + 31;
          db = 159 - st;
        } else if (st == 64) {
          da = 95;
        }
      }
      const int la = da < T ? da + 1 : 2 * T - 1 - da;
      const int lb = db < 0 ? 0 : (db < T ? db + 1 : 2 * T - 1 - db);
      if (lane >= la + lb) continue;
      const int d = lane < la ? da : db;
      const int k = lane < la ? lane : lane - la;
      const int xmin = d < T ? 0 : d - T + 1;
      const int i = rf * N - (X0 + Y0 + d) - 1;  // ring, 1 .. 4N-1
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
      const int x = xmin + k, y = d - x;
      int j = ((qf * n + (X0 + xmin) - (Y0 + d - xmin) + 1 + shift) >> 1) + k;
      if (j > 4 * n) j -= 4 * n;
      if (j < 1) j += 4 * n;
      const size_t r = o + start + (uint32_t)(j - 1);
      const uint32_t li = spread_bits((uint32_t)x) | (spread_bits((uint32_t)y) << 1);
      if (ToRing)
        out[r] = tile[li];
      else
        tile[li] = in[r];
    }
    __syncthreads();
    if (!ToRing) {
      if (vec16) {
        uint4 *dst = reinterpret_cast<uint4 *>(out + o + nest0);
        const uint4 *t4 = reinterpret_cast<const uint4 *>(tile);
        for (int e = tid; e < TT * (int)sizeof(E) / 16; e += 256) dst[e] = t4[e];
      } else {
        for (int e = tid; e < TT; e += 256) out[o + nest0 + e] = tile[e];
      }
      __syncthreads();
    }
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
  const int lgt = lgn < kTileLog ? lgn : kTileLog;
  const dim3 grid(12u << (2 * (lgn - lgt)), batch < 65535 ? batch : 65535);  // (square, channel)
  const size_t lds = ((size_t)1 << (2 * lgt)) * (size_t)eb;
  // 16-byte pieces: squares of a multiple of 16 bytes (then every square and
  // channel starts on a 16-byte boundary of a 16-byte aligned map)
  const int vec16 = (lds % 16 == 0) && (((a | c) & 15u) == 0);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (eb == 8)
    hipLaunchKernelGGL((k_reorder<uint64_t, ToRing>), grid, dim3(256), lds, st, lgn, lgt, batch, vec16,
                       static_cast<const uint64_t *>(in), static_cast<uint64_t *>(out));
  else if (eb == 4)
    hipLaunchKernelGGL((k_reorder<uint32_t, ToRing>), grid, dim3(256), lds, st, lgn, lgt, batch, vec16,
                       static_cast<const uint32_t *>(in), static_cast<uint32_t *>(out));
  else
    hipLaunchKernelGGL((k_reorder<uint16_t, ToRing>), grid, dim3(256), lds, st, lgn, lgt, batch, vec16,
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
