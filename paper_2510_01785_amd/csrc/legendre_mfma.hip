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

// Word 3 of a raw buffer resource on gfx9-family GPUs (untyped 32-bit
// loads, no swizzle).
constexpr int kBufferWord3 = 0x00020000;
constexpr int kSubL = 64;       // l's per LDS sub-tile (two per block)
constexpr int kTileRS = 64 + 4; // row stride of the LDS tile in floats
constexpr int kRedRS = 32 + 1;  // row stride of the cross-wave reduction (reuses the tile)
static_assert(kBlockL * kRedRS <= kSubL * kTileRS, "reduction fits the tile");

// Analysis.  Workgroup = one (m, l0) item of the XCD-grouped block list;
// NW waves take 64-ring slices of every 64 NW-ring chunk; each lane restarts its
// ring's recurrence from the block checkpoint, writes 64 lambdas per sub-tile
// into its wave's LDS tile [l][ring], and the wave multiplies the tile (rows =
// even or odd l) with the ring spectra E or O held in registers.  The NW
// waves' partial sums are added through LDS at the end.  NW = 1 or 2 (launch
// choice): smaller workgroups than four waves measured faster at every size
// (more of them, a shorter cross-wave reduction and barriers over fewer
// waves).
template <int NW>
__global__ void __launch_bounds__(64 * NW)
    k_legendre_fwd_mfma(Tables tb, int B, const double *__restrict__ coefA, const float2 *__restrict__ XE,
                        const float2 *__restrict__ XO, float2 *__restrict__ alm, float f0, float fm, int accum) {
  const int b0 = 16 * blockIdx.y;  // channel group of this row of the grid
  __shared__ float tile[NW * kSubL * kTileRS];
  __shared__ double sA[kBlockL];
  const int g = blockIdx.x;
  const int x = g & 7, k = g >> 3;
  const int i0 = tb.ck_xoff[x];
  if (k >= tb.ck_xoff[x + 1] - i0) return;  // uniform across the workgroup
  const int item = i0 + k;
  const int2 it = tb.ck_items[item];
  const int m = it.x, l0 = it.y;
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), j = tid & 63;
  const int h = j >> 5, col = j & 31;
  // columns beyond the batch read channel B-1 (finite data; their outputs are not stored)
  const int colc = (b0 + (col >> 1)) < B ? col : 2 * (B - 1 - b0) + (col & 1);
  // floats per ring pair in X; the fast load path needs 32 of them in 32 bits
  const size_t rowf = (size_t)M * B * 2;
  const bool fast_rows = rowf * 32 * sizeof(float) < (size_t)0x7fffffff;
  {
    const double *Ag = coefA + alm_idx(m, m, L) - m;
    for (int t = tid; t < kBlockL; t += 64 * NW) sA[t] = Ag[min(l0 + t, L)];
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

  // this lane's ring per chunk: recurrence start (kBlockL: not
  // active in this block), checkpoint and z, fetched one chunk ahead
  auto fetch_ring = [&](int q, int &t0, double2 &v, double &z) {
    const bool qok = q < Rp;
    t0 = qok ? (int)tb.ck_t[(size_t)item * Rp + q] : kBlockL;
    v = qok ? tb.ck_v[(size_t)item * Rp + q] : make_double2(0.0, 0.0);
    z = qok ? tb.rp_z[q] : 0.0;
  };
  int t0n;
  double2 vn;
  double zn;
  fetch_ring(w * 64 + j, t0n, vn, zn);
  for (int c0 = 0; c0 < Rp; c0 += 64 * NW) {
    const int t0 = t0n;
    const double2 v = vn;
    const double z = zn;
    // wait for this chunk's values here: the recurrence below then waits for
    // no load, while the spectrum loads issued before it are in flight
    asm volatile("" ::"v"(t0), "v"(v.x), "v"(v.y), "v"(z));
    fetch_ring(c0 + 64 * NW + w * 64 + j, t0n, vn, zn);
    if (__all(t0 >= kBlockL)) continue;  // no ring of this slice is active here
    // last start offset of the wave: later groups need no injection selects;
    // first start offset: a half block before it holds only zero lambdas
    int tx = t0 < kBlockL ? t0 : -1, tn = t0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      tx = max(tx, __shfl_xor(tx, o));
      tn = min(tn, __shfl_xor(tn, o));
    }
    const int tlast = __builtin_amdgcn_readfirstlane(tx);
    const int tfirst = __builtin_amdgcn_readfirstlane(tn);
    // B operands: K-step s pairs ring c0+64w+s (lanes < 32) with ring +32 (lanes >= 32)
    float xe[32], xo[32];
    const int rw = c0 + w * 64;  // first ring of this wave's slice (uniform)
    if (fast_rows && rw + 64 <= Rp) {
      // uniform row address per step, one 32-bit lane offset (half, column)
      // buffer loads: one resource per slice (uniform base), the lane's byte
      // offset in a VGPR and the step's row offset in an SGPR, so no per-load
      // vector address arithmetic (offsets < 2^32 by fast_rows)
      const unsigned voff = (unsigned)(h * 32 * rowf + colc) * 4u;
      const size_t o0 = ((size_t)rw * M + m) * B * 2 + (size_t)b0 * 2;
      const __amdgpu_buffer_rsrc_t re = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(xe_f + o0), 0, 0xffffffff, kBufferWord3);
      const __amdgpu_buffer_rsrc_t ro = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float *>(xo_f + o0), 0, 0xffffffff, kBufferWord3);
#pragma unroll
      for (int s = 0; s < 32; ++s) {
        const unsigned so = (unsigned)(s * rowf) * 4u;
        xe[s] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(re, voff, so, 0));
        xo[s] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ro, voff, so, 0));
      }
    } else {
      // rings beyond the last pair read the last pair (their lambda is zero)
#pragma unroll
      for (int s = 0; s < 32; ++s) {
        const int r = min(rw + h * 32 + s, Rp - 1);
        const size_t o = (((size_t)r * M + m) * B + b0) * 2 + colc;
        xe[s] = xe_f[o];
        xo[s] = xo_f[o];
      }
    }
    // issue the loads here, ahead of the recurrence (left alone, the compiler
    // sinks them to their first use after it and their latency is exposed)
    asm volatile("" ::: "memory");
    double prv = 0.0, cur = 0.0;
#pragma unroll
    for (int hb = 0; hb < 2; ++hb) {
      // half blocks with no lambda: every ring of the wave starts after it
      // (the recurrence state stays zero until its start), or every l of it
      // is beyond lmax (output rows that are never stored)
      if (hb == 0 && tfirst >= kSubL) continue;
      if (hb == 1 && l0 + kSubL > L) continue;
      // recurrence: 64 steps, one lambda per lane per step into the tile
#pragma unroll 1
      for (int t8 = 0; t8 < kSubL / 8; ++t8) {
        const int tb8 = hb * kSubL + t8 * 8;
        // the group's coefficients: one lane-uniform LDS address, four
        // 16-byte reads at immediate offsets
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
        // rows l > lmax only feed output rows that are never stored
        if (tb8 <= tlast) {  // uniform: some ring starts in this group
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
            tw[(t8 * 8 + u) * kTileRS + j] = (float)cur;
          }
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double nx = fma(Ac[u] * z, cur, -prv);
            prv = cur;
            cur = nx;
            tw[(t8 * 8 + u) * kTileRS + j] = (float)cur;
          }
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
  // sum the waves' partial tiles, red[w][l - l0][col] (row stride
  // kRedRS: the reads below walk l, conflict-free), and write the caller's
  // layout alm[b][idx(l, m)] = f_m c_lm a (Im = 0 for m = 0), or add to it
  __syncthreads();
  float *red = tile;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int hb = a >> 1, par = a & 1;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * h + (r & 3);
      const int lrel = hb * kSubL + 2 * i + par;
      red[(w * kBlockL + lrel) * kRedRS + col] = acc[a][r];
    }
  }
  __syncthreads();
  const double *Cn = tb.coefC + alm_idx(m, m, L) - m;
  const size_t nalm = nalm_of(L);
  const size_t base = alm_idx(l0, m, L);
  const float f = (m == 0) ? f0 : fm;
  for (int e = tid; e < 16 * kBlockL; e += 64 * NW) {
    const int c = e / kBlockL, lrel = e % kBlockL;  // a wave walks 64 consecutive l of one channel
    const int l = l0 + lrel;
    if (l > L || b0 + c >= B) continue;
    float re = 0.f, im = 0.f;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      re += red[(ww * kBlockL + lrel) * kRedRS + 2 * c];
      im += red[(ww * kBlockL + lrel) * kRedRS + 2 * c + 1];
    }
    const float g = f * (float)Cn[l];
    float2 v = make_float2(g * re, (m == 0) ? 0.f : g * im);
    float2 *dst = alm + (size_t)(b0 + c) * nalm + base + lrel;
    if (accum) {
      const float2 o = *dst;
      v.x += o.x;
      v.y += o.y;
    }
    *dst = v;
  }
}

// Synthesis.  Workgroup = one wave = (m, chunk of 64 ring pairs), one ring
// per lane.  Per 8 steps of l every lane advances its ring's recurrence by 8
// values; v_permlane32_swap pairs them into the A operands of the 32-ring
// halves (lanes 0-31: lambda_l, lanes 32-63: lambda_{l+2} of the same 32
// rings), so that with B = a_{l}, a_{l+2} (even MFMA) and a_{l+1}, a_{l+3}
// (odd MFMA) of 16 channels each half takes 4 MFMAs per 8 steps and no ring's
// recurrence is computed twice.  The recurrence coefficients are wave-uniform
// scalar loads and the B operands come straight from the coefficient slab
// (L1/L2), one group ahead: no LDS, no barriers, and every wave starts at its
// own rings' first non-negligible l.  Workgroups are dealt so that all chunks
// of eight consecutive m run on one XCD (consecutive workgroups go to
// consecutive XCDs): they share the a_m slabs in L2.  A wave writes, per ring
// pair, whole [m][batch] rows of the synthesis spectra (32 consecutive floats
// per ring: one 128-byte line at 16 channels).
constexpr int kInvRings = 64;

// (lanes 0-31 of x | lanes 0-31 of y) and (lanes 32-63 of x | lanes 32-63 of y)
__device__ __forceinline__ void pair_halves(float x, float y, float &lo, float &hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}

__global__ void __launch_bounds__(64)
    k_legendre_inv_mfma(Tables tb, int B, const double *__restrict__ coefA, const float2 *__restrict__ ALMT,
                        SynLayout lay, float2 *__restrict__ GN, float2 *__restrict__ GS) {
  const int b0 = 16 * blockIdx.y;  // channel group of this row of the grid
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int nch = (Rp + kInvRings - 1) / kInvRings;
  const int g = blockIdx.x;
  const int x = g & 7, q = g >> 3;
  // XCD x takes the octets x, x+8, ... of m; within an octet, m-major then chunk
  const int oct = x + 8 * (q / (8 * nch));
  const int r8 = q % (8 * nch);
  const int m = 8 * oct + r8 / nch;
  const int chunk = r8 % nch;
  if (m > L) return;  // uniform
  const int j = threadIdx.x;
  const int h = j >> 5, col = j & 31;
  const int p = chunk * kInvRings + j;
  const bool pok = p < Rp;
  const bool colok = (b0 + (col >> 1)) < B;
  const double z = pok ? tb.rp_z[p] : 0.0;
  const int ls = pok ? tb.seed_l[(size_t)m * Rp + p] : L + 1;
  const double2 sd = pok ? tb.seed_v[(size_t)m * Rp + p] : make_double2(0.0, 0.0);
  // first l any ring of each 32-ring half needs (aligned to m + 8j like every
  // seed), and the last seed of the wave (after it no ring starts: steps
  // without the injection selects)
  int wh = ls, wx = pok && ls <= L ? ls : -1;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) wh = min(wh, __shfl_xor(wh, o));
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) wx = max(wx, __shfl_xor(wx, o));
  const int wl0 = __builtin_amdgcn_readfirstlane(wh);
  const int wl1 = __builtin_amdgcn_readfirstlane(__shfl(wh, 32));
  const int wl = min(wl0, wl1);
  const int wlast = __builtin_amdgcn_readfirstlane(wx);
  f32x16 acc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[a][r] = 0.f;
  // A[l] of this m through the constant address space: wave-uniform indices
  // become scalar loads into SGPRs
  // (32-bit index arithmetic keeps the address on the scalar unit; nalm < 2^31)
  typedef __attribute__((address_space(4))) const double cdouble;
  const int aoff = m * (2 * L + 1 - m) / 2;  // alm_idx(m, m, L) - m
  const cdouble *Ag = (const cdouble *)coefA + aoff;
  // this lane's column of the coefficient slab a[l][col] (channels beyond the
  // batch read channel B-1: finite data, outputs not stored)
  const int colc = colok ? col : 2 * (B - 1 - b0) + (col & 1);
  // slab of column m (uniform) and this lane's fixed offsets in it: B operands
  // of the group starting at lq are rows lq + 2h + {0, 1, 4, 5}.  Rows past
  // lmax (at most 7, inside the padded coefficient workspace) are read and
  // then zeroed with their lambda in the last group.
  // Buffer loads: the slab's base in the resource, the lane's offsets in
  // VGPRs and the group's row offset in an SGPR (no per-load vector address
  // arithmetic); the slab of one m is below 2^32 bytes for any supported
  // (lmax, batch) that fits the device.
  const float *ag = reinterpret_cast<const float *>(ALMT) + ((size_t)aoff * B + b0) * 2;
  const unsigned arow = 2u * (unsigned)B;
  const unsigned vo0 = (2u * h * arow + colc) * 4u, vo1 = vo0 + arow * 4u, vo4 = vo0 + 16u * arow,
                 vo5 = vo0 + 20u * arow;
  const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(ag), 0, 0xffffffff,
                                                                       kBufferWord3);
  auto fetchB = [&](int lq, float (&bv)[4]) {
    const unsigned so = (unsigned)lq * arow * 4u;
    bv[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ar, vo0, so, 0));
    bv[1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ar, vo1, so, 0));
    bv[2] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ar, vo4, so, 0));
    bv[3] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ar, vo5, so, 0));
  };
  double prv = 0.0, cur = 0.0;
  // one group of 8 steps from l = lq with its operands bc (B) and ac (A_l);
  // the next group's operands go to bn, an (the last group re-reads its own
  // rows: every group issues the same loads, so the waits count exactly).
  // Two register sets alternate: no copies, and a group waits only for the
  // loads issued one group earlier (scalar loads complete out of order, so a
  // wait for one is a wait for all: the next ones go after this group's).
  auto group = [&](int lq, const float (&bc)[4], const double (&ac)[8], float (&bn)[4], double (&an)[8]) {
    const int ln = lq + 8 <= L ? lq + 8 : lq;
    fetchB(ln, bn);
    // the next group's scalar loads take an address that is known only
    // once this group's A_l have arrived, so they are issued after that wait
    // (and a group ahead of their own)
    int la = ln;
    asm volatile("" : "+s"(la) : "s"(ac[7]));
#pragma unroll
    for (int u = 0; u < 8; ++u) an[u] = Ag[la + u];
    float lam[8];
    // a ring's state is exactly zero before its seed, so the seed enters as a
    // 0/1 factor on two fused multiply-adds (no selects, no branch)
    const double f = (lq == ls) ? 1.0 : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double nx = fma(ac[u] * z, cur, -prv);
      if (u == 0) {
        prv = fma(f, sd.x, cur);
        cur = fma(f, sd.y, nx);
      } else {
        prv = cur;
        cur = nx;
      }
      lam[u] = (float)cur;
    }
    float bb[4] = {bc[0], bc[1], bc[2], bc[3]};
    if (lq + 7 > L) {  // last group: l beyond lmax contributes nothing
#pragma unroll
      for (int u = 0; u < 8; ++u) lam[u] = (lq + u <= L) ? lam[u] : 0.f;
      const int r0 = lq + 2 * h;
      bb[0] = r0 <= L ? bb[0] : 0.f;
      bb[1] = r0 + 1 <= L ? bb[1] : 0.f;
      bb[2] = r0 + 4 <= L ? bb[2] : 0.f;
      bb[3] = r0 + 5 <= L ? bb[3] : 0.f;
    }
    float e0lo, e0hi, o0lo, o0hi, e1lo, e1hi, o1lo, o1hi;
    pair_halves(lam[0], lam[2], e0lo, e0hi);
    pair_halves(lam[1], lam[3], o0lo, o0hi);
    pair_halves(lam[4], lam[6], e1lo, e1hi);
    pair_halves(lam[5], lam[7], o1lo, o1hi);
    if (lq + 7 >= wl0) {
      acc[0] = mfma32(e0lo, bb[0], acc[0]);
      acc[1] = mfma32(o0lo, bb[1], acc[1]);
      acc[0] = mfma32(e1lo, bb[2], acc[0]);
      acc[1] = mfma32(o1lo, bb[3], acc[1]);
    }
    if (lq + 7 >= wl1) {
      acc[2] = mfma32(e0hi, bb[0], acc[2]);
      acc[3] = mfma32(o0hi, bb[1], acc[3]);
      acc[2] = mfma32(e1hi, bb[2], acc[2]);
      acc[3] = mfma32(o1hi, bb[3], acc[3]);
    }
  };
  float bA[4], bB[4];
  double aA[8], aB[8];  // A_l of the groups (scalar registers)
  if (wl <= L) {
    fetchB(wl, bA);
#pragma unroll
    for (int u = 0; u < 8; ++u) aA[u] = Ag[wl + u];
  }
#pragma unroll 1
  for (int lq = wl; lq <= L; lq += 16) {
    group(lq, bA, aA, bB, aB);
    if (lq + 8 > L) break;
    group(lq + 8, bB, aB, bA, aA);
  }
  if (!colok) return;
  float *gn = reinterpret_cast<float *>(GN);
  float *gs = reinterpret_cast<float *>(GS);
  const int c = b0 + (col >> 1);
  const size_t ringf = (size_t)lay.ns * lay.M * lay.G * 2;  // floats per ring pair
  const size_t cofs = lay.idx(0, c, m) * 2 + (col & 1);
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = 8 * (r >> 2) + 4 * h + (r & 3);
      const int pr = chunk * kInvRings + hh * 32 + i;
      if (pr >= Rp) continue;
      const size_t o = (size_t)pr * ringf + cofs;
      gn[o] = acc[2 * hh][r] + acc[2 * hh + 1][r];
      gs[o] = acc[2 * hh][r] - acc[2 * hh + 1][r];
    }
  }
}

bool mfma_fwd_supported(const Tables &tb) { return tb.nitems > 0; }

hipError_t launch_legendre_fwd_mfma(const Tables &tb, int B, const float2 *XE, const float2 *XO, float2 *alm, double f0,
                                    double fm, int accum, hipStream_t st) {
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
  // all 16-channel groups in one launch (one tail instead of one per group);
  // one wave per workgroup from 2048 ring pairs (Nside 1024 B 16: 2.30 ms
  // against 2.33 with two waves and 2.43 with four), two below (Nside 512
  // B 16: 0.401 ms against 0.414 with one and 0.411 with four)
  const dim3 grid(8 * longest, (B + 15) / 16);
  if (tb.npairs >= 2048)
    hipLaunchKernelGGL(k_legendre_fwd_mfma<1>, grid, dim3(64), 0, st, tb, B, tb.coefA, XE, XO, alm, (float)f0,
                       (float)fm, accum);
  else
    hipLaunchKernelGGL(k_legendre_fwd_mfma<2>, grid, dim3(128), 0, st, tb, B, tb.coefA, XE, XO, alm, (float)f0,
                       (float)fm, accum);
  return hipGetLastError();
}

hipError_t launch_legendre_inv_mfma(const Tables &tb, int B, const float2 *ALMT, SynLayout lay, float2 *GN,
                                    float2 *GS, hipStream_t st) {
  const int nch = (tb.npairs + kInvRings - 1) / kInvRings;
  const int noct = (tb.lmax + 1 + 7) / 8;
  const int per_xcd = ((noct + 7) / 8) * 8 * nch;  // octets per XCD x 8 m x chunks
  hipLaunchKernelGGL(k_legendre_inv_mfma, dim3(8 * per_xcd, (B + 15) / 16), dim3(64), 0, st, tb, B, tb.coefA,
                     ALMT, lay, GN, GS);
  return hipGetLastError();
}

}  // namespace shtx
