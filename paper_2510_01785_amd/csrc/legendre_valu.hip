// Legendre step on the vector ALUs: the FP64 recurrence of Eq. (16) (run on
// mu_l = lambda_l / c_l, see tables.hip) fused with the contraction of
// Eq. (14)/(26) (analysis) or Eq. (24) (synthesis), using the north/south
// parity fold: a ring pair contributes lambda_lm(z) E_m for even l-m and
// lambda_lm(z) O_m for odd l-m to a_lm; conversely the synthesis sums
// S_e = sum_{l-m even} lambda a, S_o = sum_{l-m odd} lambda a give
// g_N = S_e + S_o and g_S = S_e - S_o.
//
// These kernels serve any batch size and both FP64 and FP32 contraction.
// Each ring starts at its stored seed l_s (a multiple of 8 above m, below
// which |lambda_lm| < 2^-64) and runs to lmax.
#include <algorithm>

#include "common.h"

namespace shtx {

// Analysis: a workgroup takes one (m, 128-l block) item of the XCD-grouped
// item list and starts every ring from its stored recurrence checkpoint at
// the block start (as the matrix-core kernel does).  Each lane owns R ring
// pairs of its wave's slice (rings j, j + 64, ...), runs their recurrences
// and, per step l, sums lambda_lm(z) X over them for BG channels (X = E for
// even l - m, O for odd: item starts are m + 128 k).  Every SL steps the wave
// transposes these per-lane sums through a wave-private LDS tile [slot][lane]
// (slot = (step, channel)); lane (slot, h) then adds the values of 64/H ring
// lanes into its accumulator of that slot.  At the end the 4 waves x H
// partial sums of every (l, channel) are added through LDS, scaled by c_lm
// and the entry point's factor, and written (or added) to the caller's layout
// alm[b][idx(l, m)], Im = 0 for m = 0.
template <typename T, int BG> struct FwdValuShape {
  // (step, channel) slots per transpose: 16, or 32 for FP32 groups of 4
  // channels (whose final reduction needs the larger tile)
  static constexpr int kSlots = (sizeof(T) == 4 && BG == 4) ? 32 : 16;
  static constexpr int kRS = 65;  // tile row stride in complex elements
  // waves per SIMD the registers are sized for: a 66.5 KB tile (FP64, or
  // FP32 with 32 slots) allows two workgroups per CU, the 33 KB FP32 one three
  static constexpr int kWaves = (sizeof(T) == 4 && kSlots == 16) ? 3 : 2;
};

template <typename T, int BG, int R>
__global__ void __launch_bounds__(256)
    __attribute__((amdgpu_waves_per_eu(FwdValuShape<T, BG>::kWaves, FwdValuShape<T, BG>::kWaves)))
    k_legendre_fwd_valu(Tables tb, int B, int bbase, const cplx<T> *__restrict__ XE, const cplx<T> *__restrict__ XO,
                        cplx<T> *__restrict__ alm, T f0, T fm, int accum) {
  const int b0 = bbase + BG * (int)blockIdx.y;  // channel group of this row of the grid
  using C = cplx<T>;
  constexpr int NW = 4;
  constexpr int SLOTS = FwdValuShape<T, BG>::kSlots, RS = FwdValuShape<T, BG>::kRS;
  constexpr int SL = SLOTS / BG;     // steps per transpose
  constexpr int H = 64 / SLOTS;      // lane groups that share a slot
  constexpr int NG = kBlockL / SL;   // transposes per block
  constexpr int LPH = 64 / H;        // ring lanes summed by one lane
  static_assert(SL % 2 == 0 && kBlockL % SL == 0, "steps per transpose");
  static_assert(NW * H * kBlockL * BG <= NW * SLOTS * RS, "final reduction fits the tile");
  __shared__ C tile[NW * SLOTS * RS];
  __shared__ double sA[kBlockL];  // the block's recurrence coefficients

  const int g = blockIdx.x;
  const int x = g & 7, k = g >> 3;
  const int i0 = tb.ck_xoff[x];
  if (k >= tb.ck_xoff[x + 1] - i0) return;  // uniform across the workgroup
  const int item = i0 + k;
  const int2 it = tb.ck_items[item];
  const int m = it.x, l0 = it.y;
  const int L = tb.lmax, M = L + 1, Rp = tb.npairs;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), j = tid & 63;
  const int slot = j % SLOTS, h = j / SLOTS;
  const int aoff = m * (2 * L + 1 - m) / 2;  // alm_idx(m, m, L) - m
  const int ng_end = min(NG, (L - l0) / SL + 1);  // transposes that hold a row l <= lmax
  C *tw = tile + w * SLOTS * RS;
  // one coalesced read of the block's coefficients (past lmax: the table's
  // zero padding, rows that are never stored)
  if (tid < kBlockL) sA[tid] = tb.coefA[aoff + l0 + tid];
  // Ring slices of 64 R rings go to the waves round-robin from the first
  // active one: rings start earlier toward the equator, so the active slices
  // of a block are (up to the discrete seeds) a suffix, and starting there
  // balances them over the waves.  s0 counts the slices whose last ring is
  // idle; every slice is still visited exactly once.
  const int nsl = (Rp + 64 * R - 1) / (64 * R);
  bool idle = false;
  if (tid < nsl) idle = tb.ck_t[(size_t)item * Rp + min((tid + 1) * 64 * R, Rp) - 1] >= kBlockL;
  const int s0 = __syncthreads_count(idle);

  C acc[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) acc[q] = cmk<C>(0, 0);

  for (int ks = w; ks < nsl; ks += NW) {
    const int c0 = ((s0 + ks) % nsl) * 64 * R;
    int t0[R];
    int tmin = kBlockL;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = c0 + r * 64 + j;
      t0[r] = q < Rp ? (int)tb.ck_t[(size_t)item * Rp + q] : kBlockL;
      tmin = min(tmin, t0[r]);
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) tmin = min(tmin, __shfl_xor(tmin, o));
    const int g_begin = __builtin_amdgcn_readfirstlane(tmin) / SL;  // earlier transposes hold zeros only
    if (g_begin >= ng_end) continue;                                 // uniform: no ring of this slice is active
    double z[R], prv[R], cur[R];
    double2 v[R];
    C xe[R][BG], xo[R][BG];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = c0 + r * 64 + j;
      const bool ok = q < Rp;
      const int qc = ok ? q : Rp - 1;  // idle lanes read finite data; their lambda stays zero
      z[r] = tb.rp_z[qc];
      v[r] = ok ? tb.ck_v[(size_t)item * Rp + q] : make_double2(0.0, 0.0);
      prv[r] = cur[r] = 0.0;
      const size_t o = ((size_t)qc * M + m) * B + b0;
#pragma unroll
      for (int b = 0; b < BG; ++b) {
        xe[r][b] = XE[o + b];
        xo[r][b] = XO[o + b];
      }
    }
    double a8[8];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      if (q < g_begin || q >= ng_end) continue;  // uniform
#pragma unroll
      for (int u = 0; u < SL; ++u) {
        const int t = q * SL + u;
        if (u % 8 == 0) {
#pragma unroll
          for (int i = 0; i < 8; ++i) a8[i] = sA[t + i];  // same address in every lane
        }
        const double a = a8[u % 8];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double nx = fma(a * z[r], cur[r], -prv[r]);
          if (t % kAlign == 0) {
            const bool inj = (t == t0[r]);
            prv[r] = inj ? v[r].x : cur[r];
            cur[r] = inj ? v[r].y : nx;
          } else {
            prv[r] = cur[r];
            cur[r] = nx;
          }
        }
#pragma unroll
        for (int b = 0; b < BG; ++b) {
          T sr = 0, si = 0;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const T lam = (T)cur[r];
            const C xv = (u & 1) ? xo[r][b] : xe[r][b];
            sr = fma(lam, xv.x, sr);
            si = fma(lam, xv.y, si);
          }
          tw[(u * BG + b) * RS + j] = cmk<C>(sr, si);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // all LPH reads in flight at once, then a pairwise sum (short chains)
      const C *src = tw + slot * RS + h * LPH;
      C e[LPH];
#pragma unroll
      for (int i = 0; i < LPH; ++i) e[i] = src[i];
#pragma unroll
      for (int st = 1; st < LPH; st <<= 1)
#pragma unroll
        for (int i = 0; i < LPH; i += 2 * st) {
          e[i].x += e[i + st].x;
          e[i].y += e[i + st].y;
        }
      acc[q].x += e[0].x;
      acc[q].y += e[0].y;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // partials red[w * H + h][l - l0][b]; the reads below walk l
  __syncthreads();
  {
    const int u = slot / BG, b = slot % BG;
#pragma unroll
    for (int q = 0; q < NG; ++q) tile[((w * H + h) * kBlockL + q * SL + u) * BG + b] = acc[q];
  }
  __syncthreads();
  const double *Cn = tb.coefC + aoff;
  const size_t nalm = nalm_of(L);
  const size_t base = alm_idx(l0, m, L);
  const T f = (m == 0) ? f0 : fm;
  for (int e = tid; e < BG * kBlockL; e += 256) {
    const int b = e / kBlockL, lrel = e % kBlockL;
    const int l = l0 + lrel;
    if (l > L) continue;
    T re = 0, im = 0;
#pragma unroll
    for (int pp = 0; pp < NW * H; ++pp) {
      const C v = tile[(pp * kBlockL + lrel) * BG + b];
      re += v.x;
      im += v.y;
    }
    const T gsc = f * (T)Cn[l];
    C val = cmk<C>(gsc * re, (m == 0) ? (T)0 : gsc * im);
    C *dst = alm + (size_t)(b0 + b) * nalm + base + lrel;
    if (accum) {
      const C o = *dst;
      val.x += o.x;
      val.y += o.y;
    }
    *dst = val;
  }
}

// v where keep, else +0 (bit mask: a NaN in unused padding is dropped too,
// and the load stays unconditional).
__device__ __forceinline__ double keep_if(double v, bool keep) {
  return __longlong_as_double(__double_as_longlong(v) & (keep ? -1LL : 0LL));
}
__device__ __forceinline__ float keep_if(float v, bool keep) {
  return __uint_as_float(__float_as_uint(v) & (keep ? 0xffffffffu : 0u));
}

// Synthesis: one wave per workgroup = (m, 64 R ring pairs), R ring pairs
// per lane (p = chunk 64 R + 64 r + lane); every lane runs its rings'
// recurrences and accumulates S_e and S_o for BG channels itself (no
// reduction).  The lanes step through l together from the wave's earliest
// seed, 8 steps per group: seeds sit at l = m + 8j, so within a group l - m is
// even exactly at the even steps.  The recurrence coefficients and the
// coefficients a_l of the BG channels are wave-uniform: one batch of scalar
// loads per group (32-bit offsets into the constant address space) serves
// all R rings.  Workgroups are dealt so that the chunks of one m run on one
// XCD.
template <typename T, int BG, int R>
__global__ void __launch_bounds__(64)
    k_legendre_inv_valu(Tables tb, int B, int bbase, const cplx<T> *__restrict__ ALMT, SynLayout lay,
                        cplx<T> *__restrict__ GN, cplx<T> *__restrict__ GS) {
  const int b0 = bbase + BG * (int)blockIdx.y;  // channel group of this row of the grid
  using C = cplx<T>;
  typedef __attribute__((address_space(4))) const double cdouble;
  typedef __attribute__((address_space(4))) const T creal;
  const int L = tb.lmax, Rp = tb.npairs;
  const int nch = (Rp + 64 * R - 1) / (64 * R);
  const int g = blockIdx.x;
  const int x = g & 7, q = g >> 3;
  const int m = x + 8 * (q / nch);
  const int chunk = q % nch;
  if (m > L) return;  // uniform
  const int j = threadIdx.x;
  double z[R], prv[R], cur[R];
  double2 sd[R];
  int ls[R];
  int wlv = L + 1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = chunk * 64 * R + 64 * r + j;
    const bool valid = p < Rp;
    z[r] = valid ? tb.rp_z[p] : 0.0;
    ls[r] = valid ? tb.seed_l[(size_t)m * Rp + p] : L + 1;
    sd[r] = valid ? tb.seed_v[(size_t)m * Rp + p] : make_double2(0.0, 0.0);
    prv[r] = cur[r] = 0.0;
    wlv = min(wlv, ls[r]);
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) wlv = min(wlv, __shfl_xor(wlv, o));
  const int wl = __builtin_amdgcn_readfirstlane(wlv);
  const int aoff = m * (2 * L + 1 - m) / 2;  // alm_idx(m, m, L) - m
  const cdouble *A = (const cdouble *)tb.coefA + aoff;
  // a[l][b] (re, im) of this channel group, stored [idx][BG] (chan_group):
  // T index 2 ((aoff + l) BG + b) + {0, 1} from the group's base
  const size_t nalm = nalm_of(L);
  const creal *a = (const creal *)ALMT + 2 * ((size_t)b0 * (nalm + kCoefPad) + (size_t)aoff * BG);
  T se[R][BG][2], so[R][BG][2];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int b = 0; b < BG; ++b) se[r][b][0] = se[r][b][1] = so[r][b][0] = so[r][b][1] = (T)0;
#pragma unroll 1
  for (int lq = wl; lq <= L; lq += 8) {
    // all scalar loads of the group first, one wait: 8 recurrence
    // coefficients and 8 contiguous rows of a (the buffer has padding rows
    // past lmax; in the last group their values are replaced by zeros)
    double Ag[8];
    T ar[8][BG], ai[8][BG];
    const creal *gp = a + (size_t)lq * (2 * BG);
#pragma unroll
    for (int u = 0; u < 8; ++u) Ag[u] = A[lq + u];  // coefficients padded past lmax
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int b = 0; b < BG; ++b) {
        ar[u][b] = gp[2 * (u * BG + b)];
        ai[u][b] = gp[2 * (u * BG + b) + 1];
      }
    // all of them in SGPRs here: the loads are issued together and waited for
    // once (left to itself the scheduler loads one row per step, each with
    // its own wait)
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      asm volatile("" : "+s"(Ag[u]));
#pragma unroll
      for (int b = 0; b < BG; ++b) asm volatile("" : "+s"(ar[u][b]), "+s"(ai[u][b]));
    }
    if (lq + 7 > L) {  // uniform: the last group
#pragma unroll
      for (int u = 1; u < 8; ++u)
#pragma unroll
        for (int b = 0; b < BG; ++b) {
          const bool in = lq + u <= L;
          ar[u][b] = keep_if(ar[u][b], in);
          ai[u][b] = keep_if(ai[u][b], in);
        }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double nx = fma(Ag[u] * z[r], cur[r], -prv[r]);
        if (u == 0) {
          const bool inj = (lq == ls[r]);
          prv[r] = inj ? sd[r].x : cur[r];
          cur[r] = inj ? sd[r].y : nx;
        } else {
          prv[r] = cur[r];
          cur[r] = nx;
        }
        const T lam = (T)cur[r];
#pragma unroll
        for (int b = 0; b < BG; ++b) {
          if (u & 1) {
            so[r][b][0] = fma(lam, ar[u][b], so[r][b][0]);
            so[r][b][1] = fma(lam, ai[u][b], so[r][b][1]);
          } else {
            se[r][b][0] = fma(lam, ar[u][b], se[r][b][0]);
            se[r][b][1] = fma(lam, ai[u][b], se[r][b][1]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = chunk * 64 * R + 64 * r + j;
    if (p >= Rp) continue;
#pragma unroll
    for (int b = 0; b < BG; ++b) {
      if (b0 + b >= B) continue;
      const size_t o = lay.idx(p, b0 + b, m);
      GN[o] = cmk<C>(se[r][b][0] + so[r][b][0], se[r][b][1] + so[r][b][1]);
      GS[o] = cmk<C>(se[r][b][0] - so[r][b][0], se[r][b][1] - so[r][b][1]);
    }
  }
}

template <typename T, int BG, int R>
static void launch_fwd_cfg(const Tables &tb, int B, int b0, int ngroups, const cplx<T> *XE, const cplx<T> *XO,
                           cplx<T> *alm, double f0, double fm, int accum, hipStream_t st) {
  int longest = 0;  // items of the largest XCD group (m = x mod 8, blocks of kBlockL l's)
  for (int x = 0; x < 8; ++x) {
    int c = 0;
    for (int m = x; m <= tb.lmax; m += 8) c += (tb.lmax - m + kBlockL) / kBlockL;
    longest = std::max(longest, c);
  }
  hipLaunchKernelGGL((k_legendre_fwd_valu<T, BG, R>), dim3(8 * longest, ngroups), dim3(256), 0, st, tb, B, b0, XE,
                     XO, alm, (T)f0, (T)fm, accum);
}

// Channel groups of 2 (FP64) or 4 (FP32), then 2 and 1 for the rest; writes
// the caller's layout (factors f0 for m = 0 and fm for m > 0, optionally
// added to what alm holds).
template <typename T>
hipError_t launch_legendre_fwd_valu(const Tables &tb, int B, const cplx<T> *XE, const cplx<T> *XO, cplx<T> *alm,
                                    double f0, double fm, int accum, hipStream_t st) {
  if (tb.nitems == 0) return hipErrorInvalidValue;
  // the groups of one width in one launch (one tail per width)
  int b0 = 0;
  if constexpr (sizeof(T) == 4) {
    if (B >= 4) launch_fwd_cfg<T, 4, 2>(tb, B, b0, B / 4, XE, XO, alm, f0, fm, accum, st);
    b0 = B / 4 * 4;
  }
  if (B - b0 >= 2) launch_fwd_cfg<T, 2, 2>(tb, B, b0, (B - b0) / 2, XE, XO, alm, f0, fm, accum, st);
  b0 += (B - b0) / 2 * 2;
  if (b0 < B) launch_fwd_cfg<T, 1, 4>(tb, B, b0, 1, XE, XO, alm, f0, fm, accum, st);
  return hipGetLastError();
}

template <typename T, int BG>
static void launch_inv_cfg(const Tables &tb, int B, int b0, int ngroups, const cplx<T> *ALMT, SynLayout lay,
                           cplx<T> *GN, cplx<T> *GS, hipStream_t st) {
  constexpr int R = BG == 1 ? 4 : 2;  // ring pairs per lane
  const int nch = (tb.npairs + 64 * R - 1) / (64 * R);
  const int nm = (tb.lmax + 1 + 7) / 8;
  hipLaunchKernelGGL((k_legendre_inv_valu<T, BG, R>), dim3(8 * nm * nch, ngroups), dim3(64), 0, st, tb, B, b0,
                     ALMT, lay, GN, GS);
}

// Channel groups of 4 (FP32) or 2 (FP64), then 2 and 1 for the rest: the
// recurrence is shared by a group, the groups' channels are never padding.
template <typename T>
hipError_t launch_legendre_inv_valu(const Tables &tb, int B, const cplx<T> *ALMT, SynLayout lay, cplx<T> *GN,
                                    cplx<T> *GS, hipStream_t st) {
  constexpr int BGMAX = sizeof(T) == 8 ? 2 : 4;
  int b0 = 0;
  if (B >= BGMAX) launch_inv_cfg<T, BGMAX>(tb, B, 0, B / BGMAX, ALMT, lay, GN, GS, st);  // one launch per width
  b0 = B / BGMAX * BGMAX;
  if (BGMAX == 4 && b0 + 2 <= B) {
    launch_inv_cfg<T, 2>(tb, B, b0, 1, ALMT, lay, GN, GS, st);
    b0 += 2;
  }
  if (b0 < B) launch_inv_cfg<T, 1>(tb, B, b0, 1, ALMT, lay, GN, GS, st);
  return hipGetLastError();
}

template hipError_t launch_legendre_fwd_valu<double>(const Tables &, int, const double2 *, const double2 *, double2 *,
                                                     double, double, int, hipStream_t);
template hipError_t launch_legendre_fwd_valu<float>(const Tables &, int, const float2 *, const float2 *, float2 *,
                                                    double, double, int, hipStream_t);
template hipError_t launch_legendre_inv_valu<double>(const Tables &, int, const double2 *, SynLayout, double2 *,
                                                     double2 *, hipStream_t);
template hipError_t launch_legendre_inv_valu<float>(const Tables &, int, const float2 *, SynLayout, float2 *,
                                                    float2 *, hipStream_t);

}  // namespace shtx
