// Conversion of maps between the pixel layouts of HEALPix (Sec. III-B): RING
// (the order of the transforms), NESTED and FLAT, through the face
// coordinates (x, y, f) of each pixel, as the paper's two-step conversion
// source -> (x, y, f) -> target.  The paper benchmarks this remapping.
//
// NESTED index p = f N^2 + interleave(x, y): base pixel (face) f = 0..11,
// face coordinates 0 <= x, y < N with x in the even and y in the odd bit
// positions.  FLAT index p = f N^2 + r N + c: each face an N x N image whose
// column axis c and row axis r run from an origin corner of the face (S, E,
// N or W) counter-clockwise or clockwise (face corners S = (0, 0),
// E = (N-1, 0), N = (N-1, N-1), W = (0, N-1); origin S counter-clockwise is
// c = x, r = y; clockwise exchanges c and r).  The face fixes the ring of a
// pixel and its slot in the ring:
//   ring  i = rf N - x - y - 1                    (rf = 2, 3, 4 for the north,
//                                                  equatorial and south faces)
//   slot  j = (qf n + x - y + 1 + s) / 2, 1-based, cyclic in 1 .. 4n
//         (qf = 1, 3, 5, 7 for polar faces and 0, 2, 4, 6 for equatorial
//          ones; n = i, 4N - i or N pixels per quadrant in the north cap,
//          south cap and belt; s = (i - N) mod 2 on the belt, 0 in the caps)
// and the RING index is the ring's first pixel plus j - 1.  nside is a power
// of two, so every step is a shift, a mask or an add: no division.
//
// A workgroup takes a T x T square of one face (T = min(nside, 64)) and one
// channel, held in LDS in local NESTED order.  Each side of a conversion
// reads or writes the square in runs: its NESTED indices are one contiguous
// range; in a FLAT layout it is T rows of T contiguous pixels (a rotation or
// reflection of an aligned square is an aligned square); each of its 2T - 1
// diagonals x + y = const is one contiguous run of one ring in RING order
// (slot j grows by one as x - y grows by two; a run wraps at most once, at
// the ring's start), lanes along the runs, two diagonals per wave step where
// they fit.
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

enum Kind { kRing = 0, kNest = 1, kFlat = 2 };

// Orientation of a FLAT layout: origin corner k (0..3 = S, E, N, W) and
// clockwise flag.  Face coordinates (x, y) -> (c, r) and back.
struct FlatOrient {
  int k, cw, n1;  // n1 = N - 1
  __device__ __forceinline__ void cr(int x, int y, int &c, int &r) const {
    int a, b;
    if (k == 0) {
      a = x;
      b = y;
    } else if (k == 1) {
      a = y;
      b = n1 - x;
    } else if (k == 2) {
      a = n1 - x;
      b = n1 - y;
    } else {
      a = n1 - y;
      b = x;
    }
    c = cw ? b : a;
    r = cw ? a : b;
  }
  __device__ __forceinline__ void xy(int c, int r, int &x, int &y) const {
    const int a = cw ? r : c, b = cw ? c : r;
    if (k == 0) {
      x = a;
      y = b;
    } else if (k == 1) {
      x = n1 - b;
      y = a;
    } else if (k == 2) {
      x = n1 - a;
      y = n1 - b;
    } else {
      x = b;
      y = n1 - a;
    }
  }
};

// The square of workgroup `blk`: face f, square origin (X0, Y0) in face
// coordinates, first NESTED index.
struct Square {
  uint32_t f, nest0;
  int X0, Y0, rf, qf;
};
__device__ __forceinline__ Square square_of(uint32_t blk, int lgn, int lgt) {
  const int lq = 2 * (lgn - lgt);  // log2 of the squares per face
  Square s;
  s.f = blk >> lq;
  const uint32_t q = blk & ((1u << lq) - 1u);
  s.X0 = (int)(compact_even_bits(q) << lgt);
  s.Y0 = (int)(compact_even_bits(q >> 1) << lgt);
  s.nest0 = (s.f << (2 * lgn)) + (q << (2 * lgt));
  const int row = (int)(s.f >> 2);
  s.rf = row + 2;                           // ring of the face's northern corner / N
  s.qf = 2 * (int)(s.f & 3u) + (row != 1);  // longitude of the face centre / (pi/4)
  return s;
}

// Visit every pixel of the square along its ring diagonals: fn(ring index in
// the channel's map, local NESTED index).  The 256 threads take one diagonal
// (or a pair of diagonals of 64 pixels in all) per wave step.
template <typename Fn>
__device__ __forceinline__ void ring_diagonals(const Square &sq, int lgn, int lgt, Fn fn) {
  const int N = 1 << lgn, T = 1 << lgt;
  const uint32_t npix = 12u << (2 * lgn);
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
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
    const int i = sq.rf * N - (sq.X0 + sq.Y0 + d) - 1;  // ring, 1 .. 4N-1
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
    int j = ((sq.qf * n + (sq.X0 + xmin) - (sq.Y0 + d - xmin) + 1 + shift) >> 1) + k;
    if (j > 4 * n) j -= 4 * n;
    if (j < 1) j += 4 * n;
    fn(start + (uint32_t)(j - 1), spread_bits((uint32_t)x) | (spread_bits((uint32_t)y) << 1));
  }
}

// Visit every pixel of the square in the rows of a FLAT layout: fn(flat index
// in the channel's map, local NESTED index); lanes along the rows.
template <typename Fn>
__device__ __forceinline__ void flat_rows(const Square &sq, int lgn, int lgt, const FlatOrient &fo, Fn fn) {
  const int N = 1 << lgn, T = 1 << lgt;
  int ca, ra, cb, rb;
  fo.cr(sq.X0, sq.Y0, ca, ra);
  fo.cr(sq.X0 + T - 1, sq.Y0 + T - 1, cb, rb);
  const int c0 = min(ca, cb), r0 = min(ra, rb);
  const uint32_t base = sq.f << (2 * lgn);
  for (int e = threadIdx.x; e < T * T; e += 256) {
    const int c = c0 + (e & (T - 1)), r = r0 + (e >> lgt);
    int x, y;
    fo.xy(c, r, x, y);
    const uint32_t li = spread_bits((uint32_t)(x - sq.X0)) | (spread_bits((uint32_t)(y - sq.Y0)) << 1);
    fn(base + (uint32_t)r * (uint32_t)N + (uint32_t)c, li);
  }
}

// One (square, channel) per workgroup: the square read from `in` (layout
// Src) into LDS, then written to `out` (layout Dst).  vec16: NESTED sides are
// copied in 16-byte pieces (the host checks that the squares and both maps
// allow it).
template <typename E, int Src, int Dst>
__global__ void __launch_bounds__(256) k_reorder(int lgn, int lgt, int B, int vec16, FlatOrient fsrc, FlatOrient fdst,
                                                 const E *__restrict__ in, E *__restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  E *tile = reinterpret_cast<E *>(smem_raw);  // T*T values in local NESTED order
  const int TT = 1 << (2 * lgt);
  const uint32_t npix = 12u << (2 * lgn);
  const Square sq = square_of(blockIdx.x, lgn, lgt);
  const int tid = threadIdx.x;
  for (int b = blockIdx.y; b < B; b += gridDim.y) {  // one channel per workgroup (row of the grid)
    const size_t o = (size_t)b * npix;
    const E *src = in + o;
    E *dst = out + o;
    if (Src == kNest) {
      if (vec16) {
        const uint4 *s4 = reinterpret_cast<const uint4 *>(src + sq.nest0);
        uint4 *t4 = reinterpret_cast<uint4 *>(tile);
        for (int e = tid; e < TT * (int)sizeof(E) / 16; e += 256) t4[e] = s4[e];
      } else {
        for (int e = tid; e < TT; e += 256) tile[e] = src[sq.nest0 + e];
      }
    } else if (Src == kFlat) {
      flat_rows(sq, lgn, lgt, fsrc, [&](uint32_t g, uint32_t li) { tile[li] = src[g]; });
    } else {
      ring_diagonals(sq, lgn, lgt, [&](uint32_t g, uint32_t li) { tile[li] = src[g]; });
    }
    __syncthreads();
    if (Dst == kNest) {
      if (vec16) {
        uint4 *d4 = reinterpret_cast<uint4 *>(dst + sq.nest0);
        const uint4 *t4 = reinterpret_cast<const uint4 *>(tile);
        for (int e = tid; e < TT * (int)sizeof(E) / 16; e += 256) d4[e] = t4[e];
      } else {
        for (int e = tid; e < TT; e += 256) dst[sq.nest0 + e] = tile[e];
      }
    } else if (Dst == kFlat) {
      flat_rows(sq, lgn, lgt, fdst, [&](uint32_t g, uint32_t li) { dst[g] = tile[li]; });
    } else {
      ring_diagonals(sq, lgn, lgt, [&](uint32_t g, uint32_t li) { dst[g] = tile[li]; });
    }
    __syncthreads();
  }
}

int elem_bytes(int dtype) {
  return dtype == SHTX_F64 ? 8 : dtype == SHTX_F32 ? 4 : dtype == SHTX_BF16 ? 2 : 0;
}

// layout code -> kind and FLAT orientation
bool decode_layout(int code, int nside, int *kind, FlatOrient *fo) {
  *fo = FlatOrient{0, 0, nside - 1};
  if (code == SHTX_LAYOUT_RING) {
    *kind = kRing;
  } else if (code == SHTX_LAYOUT_NESTED) {
    *kind = kNest;
  } else if (code >= SHTX_LAYOUT_FLAT && code < SHTX_LAYOUT_FLAT + 8) {
    *kind = kFlat;
    fo->k = (code - SHTX_LAYOUT_FLAT) >> 1;
    fo->cw = (code - SHTX_LAYOUT_FLAT) & 1;
  } else {
    return false;
  }
  return true;
}

template <typename E, int S, int D>
void launch_pair(dim3 grid, size_t lds, hipStream_t st, int lgn, int lgt, int B, int vec16, FlatOrient fs,
                 FlatOrient fd, const void *in, void *out) {
  hipLaunchKernelGGL((k_reorder<E, S, D>), grid, dim3(256), lds, st, lgn, lgt, B, vec16, fs, fd,
                     static_cast<const E *>(in), static_cast<E *>(out));
}

template <typename E>
void launch_kinds(int ks, int kd, dim3 grid, size_t lds, hipStream_t st, int lgn, int lgt, int B, int vec16,
                  FlatOrient fs, FlatOrient fd, const void *in, void *out) {
#define SHTX_REORDER_CASE(S, D) \
  if (ks == S && kd == D) return launch_pair<E, S, D>(grid, lds, st, lgn, lgt, B, vec16, fs, fd, in, out);
  SHTX_REORDER_CASE(kRing, kRing)
  SHTX_REORDER_CASE(kRing, kNest)
  SHTX_REORDER_CASE(kRing, kFlat)
  SHTX_REORDER_CASE(kNest, kRing)
  SHTX_REORDER_CASE(kNest, kNest)
  SHTX_REORDER_CASE(kNest, kFlat)
  SHTX_REORDER_CASE(kFlat, kRing)
  SHTX_REORDER_CASE(kFlat, kNest)
  SHTX_REORDER_CASE(kFlat, kFlat)
#undef SHTX_REORDER_CASE
}

int reorder(int nside, int batch, int dtype, int src_layout, int dst_layout, const void *in, void *out,
            void *stream) {
  if (nside < 1 || nside > 8192 || (nside & (nside - 1)) || batch < 1) return SHTX_ERR_ARG;
  const int eb = elem_bytes(dtype);
  if (eb == 0 || !in || !out) return SHTX_ERR_ARG;
  int ks, kd;
  FlatOrient fs, fd;
  if (!decode_layout(src_layout, nside, &ks, &fs) || !decode_layout(dst_layout, nside, &kd, &fd)) return SHTX_ERR_ARG;
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
    launch_kinds<uint64_t>(ks, kd, grid, lds, st, lgn, lgt, batch, vec16, fs, fd, in, out);
  else if (eb == 4)
    launch_kinds<uint32_t>(ks, kd, grid, lds, st, lgn, lgt, batch, vec16, fs, fd, in, out);
  else
    launch_kinds<uint16_t>(ks, kd, grid, lds, st, lgn, lgt, batch, vec16, fs, fd, in, out);
  return hipGetLastError() == hipSuccess ? SHTX_OK : SHTX_ERR_HIP;
}

}  // namespace
}  // namespace shtx

extern "C" {

int shtx_reorder(int nside, int batch, int dtype, int src_layout, int dst_layout, const void *in, void *out,
                 void *stream) {
  return shtx::reorder(nside, batch, dtype, src_layout, dst_layout, in, out, stream);
}

int shtx_nest2ring(int nside, int batch, int dtype, const void *map_nest, void *map_ring, void *stream) {
  return shtx::reorder(nside, batch, dtype, SHTX_LAYOUT_NESTED, SHTX_LAYOUT_RING, map_nest, map_ring, stream);
}

int shtx_ring2nest(int nside, int batch, int dtype, const void *map_ring, void *map_nest, void *stream) {
  return shtx::reorder(nside, batch, dtype, SHTX_LAYOUT_RING, SHTX_LAYOUT_NESTED, map_ring, map_nest, stream);
}

}  // extern "C"
