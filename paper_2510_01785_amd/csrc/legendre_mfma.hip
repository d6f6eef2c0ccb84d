// Legendre step on the matrix cores (FP32 contraction, FP64 recurrence) for
// groups of 16 channels: per m the parity-folded sums of Eq. (14)/(26) and
// Eq. (24) are dense products
//   analysis:  a[l, col]   = sum_p lambda_lm(z_p) X_{E/O}[p, col]   (K = ring pairs)
//   synthesis: S[p, col]   = sum_l lambda_lm(z_p) a[l, col]         (K = l)
// with col = (channel, re/im), 32 columns.  Both use v_mfma_f32_32x32x2_f32:
// A is 32 x 2 (lane j holds A[j % 32][j / 32]), B is 2 x 32 (lane j holds
// B[j / 32][j % 32]) and the 32 x 32 accumulator holds D[i][j] in lane
// j + 32 ((i / 4) % 2), register 4 (i / 8) + i % 4.
//
// lambda is produced by the FP64 recurrence of Eq. (16) on mu = lambda / c
// (tables.hip) with lanes running rings; in the synthesis that is already the
// A layout (rows = rings, K = l), in the analysis the values go through a
// wave-private LDS tile to become rows = l, K = rings.
#include "common.h"

namespace shtx {

typedef float f32x16 __attribute__((ext_vector_type(16)));
__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

constexpr int kFwdWaves = 4;
constexpr int kSubL = 64;       // l's per LDS sub-tile (two per block)
constexpr int kTileRS = 64 + 4; // row stride of the LDS tile in floats

// Analysis.  Workgroup = one (m, l0) item of the XCD-grouped block list;
// 4 waves take 64-ring slices of every 256-ring chunk; each lane restarts its
// ring's recurrence from the block checkpoint, writes 64 lambdas per sub-tile
// into its wave's LDS tile [l][ring], and the wave multiplies the tile (rows =
// even or odd l) with the ring spectra E or O held in registers.  The four
// waves' partial sums are added through LDS at the end.
__global__ void __launch_bounds__(256)
    k_legendre_fwd_mfma(Tables tb, int B, int b0, const double *__restrict__ coefA, const float2 *__restrict__ XE,
                        const float2 *__restrict__ XO, float2 *__restrict__ ALMT) {
  __shared__ float tile[kFwdWaves * kSubL * kTileRS];
  __shared__ double sA[kBlockL];
  const int g = blockIdx.x;
  const int x = g & 7, k = g >> 3;
  const int i0 = tb.ck_xoff[x];
  if (k >= tb.ck_xoff[x + 1] - i0) return;  // uniform across the workgroup
  const int item = i0 + k;
  const int2 it = tb.ck_items[item];
  const int m = it.x, l0 = it.y;
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int tid = threadIdx.x, w = tid >> 6, j = tid & 63;
  const int h = j >> 5, col = j & 31;
  const bool colok = (b0 + (col >> 1)) < B;
  {
    const double *Ag = coefA + alm_idx(m, m, L) - m;
    if (tid < kBlockL) sA[tid] = Ag[min(l0 + tid, L)];
  }
  __syncthreads();
  float *tw = tile + w * kSubL * kTileRS;
  const float *xe_f = reinterpret_cast<const float *>(XE);
  const float *xo_f = reinterpret_cast<const float *>(XO);

  f32x16 acc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.f;

  for (int c0 = 0; c0 < Rp; c0 += 64 * kFwdWaves) {
    const int q = c0 + w * 64 + j;  // this lane's ring for the recurrence
    const bool qok = q < Rp;
    const int t0 = qok ? (int)tb.ck_t[(size_t)item * Rp + q] : kBlockL;
    if (__all(t0 >= kBlockL)) continue;  // no ring of this slice is active here
    const double2 v = qok ? tb.ck_v[(size_t)item * Rp + q] : make_double2(0.0, 0.0);
    const double z = qok ? tb.rp_z[q] : 0.0;
    // B operands: K-step s pairs ring c0+64w+s (lanes < 32) with ring +32 (lanes >= 32)
    float xe[32], xo[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const int r = c0 + w * 64 + h * 32 + s;
      const bool ok = colok && r < Rp;
      const size_t o = (((size_t)r * M + m) * B + b0) * 2 + col;
      xe[s] = ok ? xe_f[o] : 0.f;
      xo[s] = ok ? xo_f[o] : 0.f;
    }
    double prv = 0.0, cur = 0.0;
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      // recurrence: 64 steps, one lambda per lane per step into the tile.
      // Coefficients are uniform (scalar loads, index clamped to lmax);
      // steps past lmax produce values that are masked to zero.
#pragma unroll 1
      for (int t8 = 0; t8 < kSubL / 8; ++t8) {
        const int tb8 = hb * kSubL + t8 * 8;
        const int lb8 = l0 + tb8;
        double Ac[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) Ac[u] = sA[tb8 + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double nx = fma(Ac[u] * z, cur, -prv);
          if (u == 0) {
            const bool inj = (tb8 == t0);
            prv = inj ? v.x : cur;
            cur = inj ? v.y : nx;
          } else {
            prv = cur;
            cur = nx;
          }
          tw[(t8 * 8 + u) * kTileRS + j] = (lb8 + u <= L) ? (float)cur : 0.f;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // contraction: even rows l0+hb*64+2i, odd rows +1; K = 32 steps of 2 rings
      const int i = col;
      const float *re = tw + (2 * i) * kTileRS + h * 32;
      const float *ro = tw + (2 * i + 1) * kTileRS + h * 32;
#pragma unroll
      for (int s4 = 0; s4 < 8; ++s4) {
        const float4 ae = *reinterpret_cast<const float4 *>(re + 4 * s4);
        const float4 ao = *reinterpret_cast<const float4 *>(ro + 4 * s4);
        acc[hb * 2 + 0] = mfma32(ae.x, xe[4 * s4 + 0], acc[hb * 2 + 0]);
        acc[hb * 2 + 1] = mfma32(ao.x, xo[4 * s4 + 0], acc[hb * 2 + 1]);
        acc[hb * 2 + 0] = mfma32(ae.y, xe[4 * s4 + 1], acc[hb * 2 + 0]);
        acc[hb * 2 + 1] = mfma32(ao.y, xo[4 * s4 + 1], acc[hb * 2 + 1]);
        acc[hb * 2 + 0] = mfma32(ae.z, xe[4 * s4 + 2], acc[hb * 2 + 0]);
        acc[hb * 2 + 1] = mfma32(ao.z, xo[4 * s4 + 2], acc[hb * 2 + 1]);
        acc[hb * 2 + 0] = mfma32(ae.w, xe[4 * s4 + 3], acc[hb * 2 + 0]);
        acc[hb * 2 + 1] = mfma32(ao.w, xo[4 * s4 + 3], acc[hb * 2 + 1]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // sum the four waves' partial tiles: red[w][l - l0][col]
  __syncthreads();
  float *red = tile;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int hb = a >> 1, par = a & 1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * h + (r & 3);
      const int lrel = hb * kSubL + 2 * i + par;
      red[(w * kBlockL + lrel) * 32 + col] = acc[a][r];
    }
  }
  __syncthreads();
  const double *Cn = tb.coefC + alm_idx(m, m, L) - m;
  float *out = reinterpret_cast<float *>(ALMT);
  for (int e = tid; e < kBlockL * 32; e += 256) {
    const int lrel = e >> 5, cc = e & 31;
    const int l = l0 + lrel;
    if (l > L || b0 + (cc >> 1) >= B) continue;
    float s = 0.f;
#pragma unroll
    for (int ww = 0; ww < kFwdWaves; ++ww) s += red[(ww * kBlockL + lrel) * 32 + cc];
    out[(alm_idx(l, m, L) * B + b0) * 2 + cc] = (float)Cn[l] * s;
  }
}

// Synthesis.  Workgroup = (m, chunk of 128 ring pairs), 4 waves of 32 rings;
// lanes j and j+32 both run ring j's recurrence (the two K slots of a row) and
// feed lambda_l / lambda_{l+2} (even MFMA) and lambda_{l+1} / lambda_{l+3} (odd
// MFMA) against a_{l..l+3} of 16 channels.  Workgroups are dealt so that all
// chunks of one m run on one XCD (consecutive workgroups go to consecutive
// XCDs), sharing the a_m slab in L2.
constexpr int kInvRings = 128;
constexpr int kInvBlk = 64;  // l's staged per block

__global__ void __launch_bounds__(256)
    k_legendre_inv_mfma(Tables tb, int B, int b0, const double *__restrict__ coefA, const float2 *__restrict__ ALMT,
                        float2 *__restrict__ GN, float2 *__restrict__ GS) {
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int nch = (Rp + kInvRings - 1) / kInvRings;
  const int g = blockIdx.x;
  const int x = g & 7, q = g >> 3;
  const int m = x + 8 * (q / nch);
  const int chunk = q % nch;
  if (m > L) return;  // uniform
  const int tid = threadIdx.x, w = tid >> 6, j = tid & 63;
  const int h = j >> 5, col = j & 31;
  const int p = chunk * kInvRings + w * 32 + col;
  const bool pok = p < Rp;
  const bool colok = (b0 + (col >> 1)) < B;
  const double z = pok ? tb.rp_z[p] : 0.0;
  const int ls = pok ? tb.seed_l[(size_t)m * Rp + p] : L + 1;
  const double2 sd = pok ? tb.seed_v[(size_t)m * Rp + p] : make_double2(0.0, 0.0);
  // first l any ring of the workgroup needs
  __shared__ int s_lb;
  __shared__ float sB[2][kInvBlk][32];
  __shared__ double sA[2][kInvBlk];
  if (tid == 0) s_lb = L + 1;
  __syncthreads();
  atomicMin(&s_lb, ls);
  int wl = ls;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) wl = min(wl, __shfl_xor(wl, o));
  __syncthreads();
  const int lb = s_lb;
  const double *Ag = coefA + alm_idx(m, m, L) - m;
  const float *ag = reinterpret_cast<const float *>(ALMT) + ((alm_idx(m, m, L) - m) * B + b0) * 2;
  const size_t arow = (size_t)B * 2;
  // staging of one block: rows l0..l0+kInvBlk-1 of a (32 floats each, 8 per
  // thread) and their recurrence coefficients
  const int srow = tid >> 2, scol = (tid & 3) * 8;
  float stg[8];
  double stgA = 0.0;
  auto fetch = [&](int l0) {
    const int l = l0 + srow;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int cc = scol + e;
      const bool ok = l <= L && (b0 + (cc >> 1)) < B;
      stg[e] = ok ? ag[(size_t)l * arow + cc] : 0.f;
    }
    if (tid < kInvBlk) stgA = Ag[min(l0 + tid, L)];
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) sB[buf][srow][scol + e] = stg[e];
    if (tid < kInvBlk) sA[buf][tid] = stgA;
  };
  f32x16 acc_e, acc_o;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc_e[r] = acc_o[r] = 0.f;
  double prv = 0.0, cur = 0.0;
  if (lb <= L) {
    fetch(lb);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int l0 = lb; l0 <= L; l0 += kInvBlk) {
    const bool more = l0 + kInvBlk <= L;
    if (more) fetch(l0 + kInvBlk);
    if (wl <= l0 + kInvBlk - 1) {  // some ring of this wave is active in the block
#pragma unroll 1
      for (int u8 = 0; u8 < kInvBlk / 8; ++u8) {
        const int lq = l0 + 8 * u8;
        float lam[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double nx = fma(sA[buf][8 * u8 + u] * z, cur, -prv);
          if (u == 0) {
            const bool inj = (lq == ls);
            prv = inj ? sd.x : cur;
            cur = inj ? sd.y : nx;
          } else {
            prv = cur;
            cur = nx;
          }
          lam[u] = (lq + u <= L) ? (float)cur : 0.f;
        }
        const float *rb = &sB[buf][8 * u8 + 2 * h][col];
        acc_e = mfma32(h ? lam[2] : lam[0], rb[0], acc_e);
        acc_o = mfma32(h ? lam[3] : lam[1], rb[32], acc_o);
        acc_e = mfma32(h ? lam[6] : lam[4], rb[4 * 32], acc_e);
        acc_o = mfma32(h ? lam[7] : lam[5], rb[5 * 32], acc_o);
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (!colok) return;
  float *gn = reinterpret_cast<float *>(GN);
  float *gs = reinterpret_cast<float *>(GS);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + 4 * h + (r & 3);
    const int pr = chunk * kInvRings + w * 32 + i;
    if (pr >= Rp) continue;
    const size_t o = (((size_t)pr * M + m) * B + b0) * 2 + col;
    gn[o] = acc_e[r] + acc_o[r];
    gs[o] = acc_e[r] - acc_o[r];
  }
}

bool mfma_fwd_supported(const Tables &tb) { return tb.nitems > 0; }

hipError_t launch_legendre_fwd_mfma(const Tables &tb, int B, const float2 *XE, const float2 *XO, float2 *ALMT,
                                    hipStream_t st) {
  // grid: 8 XCD groups x the longest group
  int longest = 0;
  {
    // item counts per XCD group follow from the same enumeration as k_items
    const int L = tb.lmax;
    for (int xg = 0; xg < 8; ++xg) {
      int c = 0;
      for (int m = xg; m <= L; m += 8) c += (L - m + kBlockL) / kBlockL;
      longest = c > longest ? c : longest;
    }
  }
  for (int b0 = 0; b0 < B; b0 += 16)
    hipLaunchKernelGGL(k_legendre_fwd_mfma, dim3(8 * longest), dim3(256), 0, st, tb, B, b0, tb.coefA, XE, XO,
                       ALMT);
  return hipGetLastError();
}

hipError_t launch_legendre_inv_mfma(const Tables &tb, int B, const float2 *ALMT, float2 *GN, float2 *GS,
                                    hipStream_t st) {
  const int nch = (tb.npairs + kInvRings - 1) / kInvRings;
  const int nm = (tb.lmax + 1 + 7) / 8;
  for (int b0 = 0; b0 < B; b0 += 16)
    hipLaunchKernelGGL(k_legendre_inv_mfma, dim3(8 * nm * nch), dim3(256), 0, st, tb, B, b0, tb.coefA, ALMT, GN,
                       GS);
  return hipGetLastError();
}

}  // namespace shtx
