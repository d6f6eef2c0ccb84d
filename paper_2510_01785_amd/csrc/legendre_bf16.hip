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
// its four waves take 128-ring slices of every 512-ring chunk, two adjacent
// rings per lane (two independent FP64 recurrences per lane).  A lane packs
// its two rings' BF16 lambda of one l into one 32-bit word, so K slot 2q,
// 2q + 1 of a slice are its rings 2q, 2q + 1.  The spectra of a slice are
// transposed into that K order through the same LDS tile (B operands kept in
// registers for the whole block).
#include "common.h"

namespace shtx {

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

constexpr int kBfWaves = 4;
constexpr int kBfSlice = 128;                  // rings per wave slice
constexpr int kBfChunk = kBfWaves * kBfSlice;  // rings per chunk
constexpr int kBfSub = 64;                     // l per lambda tile (half a block)
constexpr int kBfRS = 64 + 4;                  // tile row stride in words (64 ring pairs)
constexpr int kBfTileW = kBfSub * kBfRS;       // words per wave tile
constexpr int kBfRedRS = 32 + 1;               // row stride of the cross-wave reduction (floats)
static_assert(32 * kBfRS <= kBfTileW, "spectrum staging fits the tile");
static_assert(kBfWaves * kBlockL * kBfRedRS <= kBfWaves * kBfTileW + 512, "reduction fits the LDS");

__global__ void __launch_bounds__(256)
    k_legendre_fwd_bf16(Tables tb, int B, const double *__restrict__ coefA, const uint32_t *__restrict__ XE,
                        const uint32_t *__restrict__ XO, float2 *__restrict__ alm, float f0, float fm, int accum) {
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
    if (tid < kBlockL) sA[tid] = Ag[min(l0 + tid, L)];
  }
  __syncthreads();
  uint32_t *tw = tile + w * kBfTileW;
  const bool fast_x = (B & 3) == 0;  // 16-byte spectrum pieces are aligned

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

    // spectra of the slice -> B operands: staging [col][ring pair] words
    // (row stride kBfRS), each word the two rings of one pair; a lane loads
    // 16-byte pieces (4 channels) of rings 2q and 2q + 1, q = lane % 32 +
    // 32 t, piece lane / 32 + 2 u
    u32x4_t xop[2][8];
#pragma unroll
    for (int par = 0; par < 2; ++par) {
      const uint32_t *X = par ? XO : XE;
      uint32_t pa[2][2][4], pb[2][2][4];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int q = (j & 31) + 32 * t, c4 = (j >> 5) + 2 * u;
          const int ra_ = min(q0 + 2 * q, Rp - 1), rb_ = min(q0 + 2 * q + 1, Rp - 1);
          const size_t oa = ((size_t)ra_ * M + m) * B, ob = ((size_t)rb_ * M + m) * B;
          const int cb = b0 + 4 * c4;
          if (fast_x && cb + 3 < B) {
            const uint4 va = *reinterpret_cast<const uint4 *>(X + oa + cb);
            const uint4 vb = *reinterpret_cast<const uint4 *>(X + ob + cb);
            pa[t][u][0] = va.x; pa[t][u][1] = va.y; pa[t][u][2] = va.z; pa[t][u][3] = va.w;
            pb[t][u][0] = vb.x; pb[t][u][1] = vb.y; pb[t][u][2] = vb.z; pb[t][u][3] = vb.w;
          } else {
            // channels beyond the batch read channel B-1 (finite data; those
            // columns are never stored)
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              const int c = min(cb + d, B - 1);
              pa[t][u][d] = X[oa + c];
              pb[t][u][d] = X[ob + c];
            }
          }
        }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int q = (j & 31) + 32 * t, c4 = (j >> 5) + 2 * u;
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const uint32_t a = pa[t][u][d], b = pb[t][u][d];
            const int n = 8 * c4 + 2 * d;  // column of the real part
            tw[n * kBfRS + q] = (a & 0xffffu) | (b << 16);
            tw[(n + 1) * kBfRS + q] = (a >> 16) | (b & 0xffff0000u);
          }
        }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int k = 0; k < 8; ++k) xop[par][k] = *reinterpret_cast<const u32x4_t *>(tw + col * kBfRS + 8 * k + 4 * h);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    double pa_ = 0.0, ca = 0.0, pb_ = 0.0, cb = 0.0;  // (mu_{l-1}, mu_l) of the two rings
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      // half blocks with no lambda: every ring of the slice starts after it
      // (the state stays zero until its start), or every l of it is beyond
      // lmax (output rows that are never stored)
      if (hb == 0 && tfirst >= kBfSub) continue;
      if (hb == 1 && l0 + kBfSub > L) continue;
#pragma unroll 1
      for (int t8 = 0; t8 < kBfSub / 8; ++t8) {
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
        uint32_t *trow = tw + (t8 * 8) * kBfRS + j;
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
            trow[u * kBfRS] = pack_bf16x2(f64_to_f32(ca), f64_to_f32(cb));
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
            trow[u * kBfRS] = pack_bf16x2(f64_to_f32(ca), f64_to_f32(cb));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // contraction: even rows l0 + hb*64 + 2i, odd rows + 1; K = 8 steps of
      // 16 rings (8 ring pairs = 4 words per lane)
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const u32x4_t ae = *reinterpret_cast<const u32x4_t *>(tw + (2 * col) * kBfRS + 8 * k + 4 * h);
        const u32x4_t ao = *reinterpret_cast<const u32x4_t *>(tw + (2 * col + 1) * kBfRS + 8 * k + 4 * h);
        acc[hb * 2 + 0] = mfma_bf16(ae, xop[0][k], acc[hb * 2 + 0]);
        acc[hb * 2 + 1] = mfma_bf16(ao, xop[1][k], acc[hb * 2 + 1]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // sum the four waves' partial tiles, red[w][l - l0][col], and write the
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
  for (int e = tid; e < 16 * kBlockL; e += 256) {
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

hipError_t launch_legendre_fwd_bf16(const Tables &tb, int B, const uint32_t *XE, const uint32_t *XO, float2 *alm,
                                    double f0, double fm, int accum, hipStream_t st) {
  if (tb.nitems == 0) return hipErrorInvalidValue;
  int longest = 0;
  {
    const int L = tb.lmax;
    for (int xg = 0; xg < 8; ++xg) {
      int c = 0;
      for (int m = xg; m <= L; m += 8) c += (L - m + kBlockL) / kBlockL;
      longest = c > longest ? c : longest;
    }
  }
  hipLaunchKernelGGL(k_legendre_fwd_bf16, dim3(8 * longest, (B + 15) / 16), dim3(256), 0, st, tb, B, tb.coefA, XE,
                     XO, alm, (float)f0, (float)fm, accum);
  return hipGetLastError();
}

}  // namespace shtx
