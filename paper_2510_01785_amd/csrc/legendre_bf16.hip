// Legendre step of the analysis with BF16 operands on the matrix cores:
// a[l, col] = sum_p lambda_lm(z_p) X_{E/O}[p, col] (Eq. (14)/(26), parity
// folded) for groups of 16 channels, as v_mfma_f32_32x32x16_bf16 products
// with FP32 accumulation.  The ring spectra X arrive in BF16 from the ring
// FFT; lambda comes from the FP64 recurrence of Eq. (16) (on mu = lambda/c,
// tables.hip) and is rounded to BF16 for the product.  This is the BF16 map
// path: its spectra and Legendre values carry BF16 rounding (relative 2^-9
// per value), the sums and the recurrence do not.
//
// Operand layouts of v_mfma_f32_32x32x16_bf16 (A 32 x 16, B 16 x 32, D 32 x
// 32): lane j holds A[j % 32][8 (j / 32) + e] and B[8 (j / 32) + e][j % 32]
// for e = 0..7 (eight BF16 in four registers); the accumulator holds D[i][j]
// in lane j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.  Rows are l of
// one parity, K are ring pairs, columns (channel, re/im).
//
// Work split: a workgroup takes one (m, l0) item of the XCD-grouped block
// list (blocks of kBlockL l restarted from stored recurrence checkpoints);
// its kBfWaves waves (one: measured faster than two or four, Nside 1024 B 16
// 0.81 ms against 0.83 and 0.88) take 128-ring slices of every chunk, two
// adjacent rings per lane (two independent FP64 recurrences per lane).  A lane packs
// its two rings' BF16 lambda of one l into one 32-bit word, so K slot 2q,
// 2q + 1 of a slice are its rings 2q, 2q + 1.  The spectra arrive in that
// K order from k_pack_spectra_bf16 (below): one 16-byte load per lane and K
// step is a B operand, all of a slice issued before the recurrence that
// precedes their first use and kept in registers for the block.
//
// Stored-lambda mode (the paper's precomputed Legendre tensor, Sec. III-G,
// Eq. (28), kept resident in HBM for a hot (nside, lmax) instead of streamed
// from the host): the same kernel, in MODE kLamBuild, writes every 64 x 128
// BF16 lambda tile it would compute to a table in device memory (only the
// tiles the pruned triangle executes; a per-(item, slice) offset table in front
// of them), and in MODE kLamStored reads the tiles from that table as its A
// operands instead of running the recurrence.  The operands and the order of
// the products are the same, so the coefficients are bit-identical.
#include <algorithm>
#include <vector>

#include "common.h"

namespace shtx {

size_t lam_header_words(int nside, int nitems);

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x16_t mfma_bf16(u32x4_t a, u32x4_t b, f32x16_t c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                  0, 0, 0);
}


// FP64 -> FP32 kept as its own rounding step (left visible, the compiler
// folds the two conversions FP64 -> FP32 -> BF16 into one direct FP64 -> BF16
// rounding, a sequence of about ten instructions per value on this target).
__device__ __forceinline__ float f64_to_f32(double d) {
  float f = (float)d;
  asm("" : "+v"(f));
  return f;
}

constexpr int kBfWaves = 1;
constexpr int kBfSlice = 128;                  // rings per wave slice
constexpr int kBfChunk = kBfWaves * kBfSlice;  // rings per chunk
constexpr int kBfSub = 64;                     // l per lambda tile (half a block)
constexpr int kBfRS = 64 + 4;                  // tile row stride in words (64 ring pairs)
constexpr int kBfTileW = kBfSub * kBfRS;       // words per wave tile
constexpr int kBfRedRS = 32 + 1;               // row stride of the cross-wave reduction (floats)
static_assert(32 * kBfRS <= kBfTileW, "spectrum staging fits the tile");
static_assert(kBfWaves * kBlockL * kBfRedRS <= kBfWaves * kBfTileW + 512, "reduction fits the LDS");

enum LamMode { kLamCompute = 0, kLamBuild = 1, kLamStored = 2 };
constexpr int kLamTileW = kBfSub * 64;  // words of one stored tile (64 l x 64 ring pairs)
constexpr int kLamTileBytes = kLamTileW * 4;

template <int MODE>
__global__ void __launch_bounds__(64 * kBfWaves)
    k_legendre_fwd_bf16(Tables tb, int B, const double *__restrict__ coefA, const u32x4_t *__restrict__ XT,
                        size_t xt_par, float2 *__restrict__ alm, float f0, float fm, int accum,
                        const uint32_t *__restrict__ lam_off, uint32_t *__restrict__ lam_tiles) {
  const int b0 = 16 * blockIdx.y;  // channel group of this row of the grid
  __shared__ __attribute__((aligned(16))) uint32_t tile[kBfWaves * kBfTileW + 512];
  __shared__ double sA[kBlockL];
  const int g = blockIdx.x;
  const int x = g & 7, kx = g >> 3;
  const int i0 = tb.ck_xoff[x];
  if (kx >= tb.ck_xoff[x + 1] - i0) return;  // uniform across the workgroup
  const int item = i0 + kx;
  const int2 it = tb.ck_items[item];
  const int m = it.x, l0 = it.y;
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), j = tid & 63;
  const int h = j >> 5, col = j & 31;
  {
    const double *Ag = coefA + alm_idx(m, m, L) - m;
    for (int t = tid; t < kBlockL; t += 64 * kBfWaves) sA[t] = Ag[min(l0 + t, L)];
  }
  __syncthreads();
  uint32_t *tw = tile + w * kBfTileW;
  const int nrb = (Rp + 7) / 8;
  // B operands of this lane in the packed spectra: (parity, m) rows of the
  // channel group, 16 bytes per (ring block, column)
  const u32x4_t *xt = MODE == kLamBuild ? nullptr : XT + ((size_t)blockIdx.y * M + m) * nrb * 32 + col;

  f32x16_t acc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.f;

  // this lane's two rings of a chunk: recurrence start (kBlockL: idle in this
  // block), checkpoint, z; fetched one chunk ahead
  struct Ring {
    int t0;
    double2 v;
    double z;
  };
  auto fetch_ring = [&](int q) {
    Ring r;
    const bool ok = q < Rp;
    r.t0 = ok ? (int)tb.ck_t[(size_t)item * Rp + q] : kBlockL;
    r.v = ok ? tb.ck_v[(size_t)item * Rp + q] : make_double2(0.0, 0.0);
    r.z = ok ? tb.rp_z[q] : 0.0;
    return r;
  };
  Ring na = fetch_ring(w * kBfSlice + 2 * j), nb = fetch_ring(w * kBfSlice + 2 * j + 1);
  for (int c0 = 0; c0 < Rp; c0 += kBfChunk) {
    const Ring ra = na, rb = nb;
    asm volatile("" ::"v"(ra.t0), "v"(rb.t0), "v"(ra.v.x), "v"(ra.v.y), "v"(rb.v.x), "v"(rb.v.y), "v"(ra.z),
                 "v"(rb.z));
    na = fetch_ring(c0 + kBfChunk + w * kBfSlice + 2 * j);
    nb = fetch_ring(c0 + kBfChunk + w * kBfSlice + 2 * j + 1);
    const int q0 = c0 + w * kBfSlice;  // first ring of this wave's slice (uniform)
    if (__all(ra.t0 >= kBlockL && rb.t0 >= kBlockL)) continue;  // no ring of the slice is active here
    // last start offset of the slice (later groups need no injection
    // selects) and first (a half block before it holds only zero lambdas)
    int tx = max(ra.t0 < kBlockL ? ra.t0 : -1, rb.t0 < kBlockL ? rb.t0 : -1), tn = min(ra.t0, rb.t0);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      tx = max(tx, __shfl_xor(tx, o));
      tn = min(tn, __shfl_xor(tn, o));
    }
    const int tlast = __builtin_amdgcn_readfirstlane(tx);
    const int tfirst = __builtin_amdgcn_readfirstlane(tn);
    // stored tiles of this (item, slice): hb 0 (if active) then hb 1
    uint32_t toff = 0;
    if constexpr (MODE != kLamCompute) {
      const int nslices = (Rp + kBfSlice - 1) / kBfSlice;
      toff = __builtin_amdgcn_readfirstlane(lam_off[(size_t)item * nslices + q0 / kBfSlice]);
    }

    // B operands of the slice: K step k of lane half h is ring block
    // q0 / 8 + 2 k + h (clamped: blocks past the last ring pair meet zero
    // lambdas); issued here, first needed after the recurrence of the first
    // half block
    u32x4_t xop[2][8];
    if constexpr (MODE != kLamBuild) {
#pragma unroll
      for (int par = 0; par < 2; ++par)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int rb = min((q0 >> 3) + 2 * k + h, nrb - 1);
          xop[par][k] = xt[par * xt_par + (size_t)rb * 32];
        }
    }

    double pa_ = 0.0, ca = 0.0, pb_ = 0.0, cb = 0.0;  // (mu_{l-1}, mu_l) of the two rings
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      // half blocks with no lambda: every ring of the slice starts after it
      // (the state stays zero until its start), or every l of it is beyond
      // lmax (output rows that are never stored)
      if (hb == 0 && tfirst >= kBfSub) continue;
      if (hb == 1 && l0 + kBfSub > L) continue;
      uint32_t *gt = lam_tiles + (size_t)(toff + (hb == 1 && tfirst < kBfSub ? 1u : 0u)) * kLamTileW;
#pragma unroll 1
      for (int t8 = 0; t8 < kBfSub / 8; ++t8) {
        if constexpr (MODE == kLamStored) break;  // lambda comes from the table
        const int tb8 = hb * kBfSub + t8 * 8;
        int aaddr = tb8;
        asm volatile("" : "+v"(aaddr));
        const double2 *sA2 = reinterpret_cast<const double2 *>(sA + aaddr);
        double Ac[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double2 a2 = sA2[u];
          Ac[2 * u] = a2.x;
          Ac[2 * u + 1] = a2.y;
        }
        // the tile row of l = tb8 + u: this wave's LDS tile, or the table
        uint32_t *trow = MODE == kLamBuild ? gt + (t8 * 8) * 64 + j : tw + (t8 * 8) * kBfRS + j;
        const int rs = MODE == kLamBuild ? 64 : kBfRS;
        if (tb8 <= tlast) {  // uniform: some ring starts in this group
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double xa = fma(Ac[u] * ra.z, ca, -pa_);
            const double xb = fma(Ac[u] * rb.z, cb, -pb_);
            if (u == 0) {
              const bool ia = (tb8 == ra.t0), ib = (tb8 == rb.t0);
              pa_ = ia ? ra.v.x : ca;
              ca = ia ? ra.v.y : xa;
              pb_ = ib ? rb.v.x : cb;
              cb = ib ? rb.v.y : xb;
            } else {
              pa_ = ca;
              ca = xa;
              pb_ = cb;
              cb = xb;
            }
            trow[u * rs] = pack_bf16x2(f64_to_f32(ca), f64_to_f32(cb));
          }
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double xa = fma(Ac[u] * ra.z, ca, -pa_);
            const double xb = fma(Ac[u] * rb.z, cb, -pb_);
            pa_ = ca;
            ca = xa;
            pb_ = cb;
            cb = xb;
            trow[u * rs] = pack_bf16x2(f64_to_f32(ca), f64_to_f32(cb));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if constexpr (MODE == kLamBuild) continue;
      // contraction: even rows l0 + hb*64 + 2i, odd rows + 1; K = 8 steps of
      // 16 rings (8 ring pairs = 4 words per lane); A from the LDS tile, or
      // (stored mode) from the table
      const uint32_t *at = MODE == kLamStored ? gt : tw;
      const int ars = MODE == kLamStored ? 64 : kBfRS;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const u32x4_t ae = *reinterpret_cast<const u32x4_t *>(at + (2 * col) * ars + 8 * k + 4 * h);
        const u32x4_t ao = *reinterpret_cast<const u32x4_t *>(at + (2 * col + 1) * ars + 8 * k + 4 * h);
        acc[hb * 2 + 0] = mfma_bf16(ae, xop[0][k], acc[hb * 2 + 0]);
        acc[hb * 2 + 1] = mfma_bf16(ao, xop[1][k], acc[hb * 2 + 1]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if constexpr (MODE == kLamBuild) return;
  // sum the waves' partial tiles, red[w][l - l0][col], and write the
  // caller's layout alm[b][idx(l, m)] = f_m c_lm a (Im = 0 for m = 0), or add
  __syncthreads();
  float *red = reinterpret_cast<float *>(tile);
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int hb = a >> 1, par = a & 1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * h + (r & 3);
      const int lrel = hb * kBfSub + 2 * i + par;
      red[(w * kBlockL + lrel) * kBfRedRS + col] = acc[a][r];
    }
  }
  __syncthreads();
  const double *Cn = tb.coefC + alm_idx(m, m, L) - m;
  const size_t nalm = nalm_of(L);
  const size_t base = alm_idx(l0, m, L);
  const float f = (m == 0) ? f0 : fm;
  for (int e = tid; e < 16 * kBlockL; e += 64 * kBfWaves) {
    const int c = e / kBlockL, lrel = e % kBlockL;
    const int l = l0 + lrel;
    if (l > L || b0 + c >= B) continue;
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int ww = 0; ww < kBfWaves; ++ww) {
      re += red[(ww * kBlockL + lrel) * kBfRedRS + 2 * c];
      im += red[(ww * kBlockL + lrel) * kBfRedRS + 2 * c + 1];
    }
    const float gg = f * (float)Cn[l];
    float2 v = make_float2(gg * re, (m == 0) ? 0.f : gg * im);
    float2 *dst = alm + (size_t)(b0 + c) * nalm + base + lrel;
    if (accum) {
      const float2 o = *dst;
      v.x += o.x;
      v.y += o.y;
    }
    *dst = v;
  }
}

static int longest_xcd_items(int L) {
  int longest = 0;
  for (int xg = 0; xg < 8; ++xg) {
    int c = 0;
    for (int m = xg; m <= L; m += 8) c += (L - m + kBlockL) / kBlockL;
    longest = c > longest ? c : longest;
  }
  return longest;
}

// The BF16 ring spectra X_{E/O}[p][m][b] (one 32-bit word per value, Re in
// the low half) rewritten in the B-operand order of the contraction:
// XT[parity][g][m][rb][col] holds, for channel 16 g + col / 2 (Re for even
// col, Im for odd), the BF16 values of ring pairs 8 rb .. 8 rb + 7 in 16
// bytes (zero past the last ring pair and the batch).  A wave covers two m
// rows of 32 columns: 128 contiguous bytes per ring pair read (16 channels),
// 512 per row written.
__global__ void __launch_bounds__(256)
    k_pack_spectra_bf16(const uint32_t *__restrict__ XE, const uint32_t *__restrict__ XO, u32x4_t *__restrict__ XT,
                        int B, int M, int Rp, int nrb, int ng) {
  const int col = threadIdx.x & 31;
  const int m = blockIdx.x * 8 + (threadIdx.x >> 5);
  const int rb = blockIdx.y, g = blockIdx.z % ng, par = blockIdx.z / ng;
  if (m >= M) return;
  const uint32_t *X = par ? XO : XE;
  const int c = 16 * g + (col >> 1), sh = 16 * (col & 1);
  uint32_t v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int p = 8 * rb + e;
    const uint32_t wd = (p < Rp && c < B) ? X[((size_t)p * M + m) * B + c] : 0u;
    v[e] = (wd >> sh) & 0xffffu;
  }
  u32x4_t o;
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = v[2 * i] | (v[2 * i + 1] << 16);
  XT[((((size_t)par * ng + g) * M + m) * nrb + rb) * 32 + col] = o;
}

size_t bf16_packed_spectra_bytes(int lmax, int npairs, int B) {
  return 2 * (size_t)((B + 15) / 16) * (size_t)(lmax + 1) * (size_t)((npairs + 7) / 8) * 512;
}

hipError_t launch_pack_spectra_bf16(const Tables &tb, int B, const uint32_t *XE, const uint32_t *XO, void *xt,
                                    hipStream_t st) {
  const int M = tb.lmax + 1, Rp = tb.npairs, nrb = (Rp + 7) / 8, ng = (B + 15) / 16;
  if (2 * ng > 65535 || nrb > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pack_spectra_bf16, dim3((M + 7) / 8, nrb, 2 * ng), dim3(256), 0, st, XE, XO,
                     static_cast<u32x4_t *>(xt), B, M, Rp, nrb, ng);
  return hipGetLastError();
}

// Legendre step on the packed spectra xt (k_pack_spectra_bf16's output).
hipError_t launch_legendre_fwd_bf16(const Tables &tb, int B, const void *xt, float2 *alm, double f0, double fm,
                                    int accum, hipStream_t st, const uint32_t *lam) {
  if (tb.nitems == 0) return hipErrorInvalidValue;
  const int M = tb.lmax + 1, Rp = tb.npairs, nrb = (Rp + 7) / 8, ng = (B + 15) / 16;
  if (ng > 65535) return hipErrorInvalidValue;
  const u32x4_t *XT = static_cast<const u32x4_t *>(xt);
  const size_t xt_par = (size_t)ng * M * nrb * 32;
  const dim3 grid(8 * longest_xcd_items(tb.lmax), ng);
  if (lam) {
    const uint32_t *tiles = lam + lam_header_words(tb.nside, tb.nitems);
    hipLaunchKernelGGL(k_legendre_fwd_bf16<kLamStored>, grid, dim3(64 * kBfWaves), 0, st, tb, B, tb.coefA, XT, xt_par, alm,
                       (float)f0, (float)fm, accum, lam, const_cast<uint32_t *>(tiles));
  } else {
    hipLaunchKernelGGL(k_legendre_fwd_bf16<kLamCompute>, grid, dim3(64 * kBfWaves), 0, st, tb, B, tb.coefA, XT, xt_par, alm,
                       (float)f0, (float)fm, accum, nullptr, nullptr);
  }
  return hipGetLastError();
}

// The stored-lambda table: per (item, 128-ring slice) the index of its first
// tile (header, lam_header_words words), then the tiles.  A slice has a tile
// for each of its active half blocks, by the rule the kernel applies (any
// ring active in the block; the first half block if some ring starts in it,
// the second if it holds l <= lmax).
size_t lam_header_words(int nside, int nitems) {
  const size_t ns = (2 * (size_t)nside + kBfSlice - 1) / kBfSlice;
  return align_up((size_t)nitems * ns, 1024);
}

std::vector<uint32_t> lam_tile_offsets(int nside, int lmax, int nitems, const uint8_t *ck_t, const int2 *items,
                                       size_t *ntiles) {
  const int Rp = 2 * nside, ns = (Rp + kBfSlice - 1) / kBfSlice;
  std::vector<uint32_t> off((size_t)nitems * ns);
  size_t run = 0;
  for (int it = 0; it < nitems; ++it) {
    const int l0 = items[it].y;
    for (int s = 0; s < ns; ++s) {
      int tmin = kBlockL;
      for (int q = s * kBfSlice; q < std::min(Rp, (s + 1) * kBfSlice); ++q)
        tmin = std::min(tmin, (int)ck_t[(size_t)it * Rp + q]);
      off[(size_t)it * ns + s] = (uint32_t)run;
      if (tmin < kBlockL) run += (size_t)(tmin < kBfSub) + (size_t)(l0 + kBfSub <= lmax);
    }
  }
  *ntiles = run;
  return off;
}

hipError_t launch_lambda_table_build(const Tables &tb, uint32_t *lam, hipStream_t st) {
  if (tb.nitems == 0) return hipErrorInvalidValue;
  const dim3 grid(8 * longest_xcd_items(tb.lmax), 1);
  hipLaunchKernelGGL(k_legendre_fwd_bf16<kLamBuild>, grid, dim3(64 * kBfWaves), 0, st, tb, 16, tb.coefA, nullptr, (size_t)0,
                     nullptr, 1.f, 1.f, 0, lam, lam + lam_header_words(tb.nside, tb.nitems));
  return hipGetLastError();
}

}  // namespace shtx
