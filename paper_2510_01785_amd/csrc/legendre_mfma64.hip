// Legendre steps in FP64 on the matrix cores.  Analysis: per m the
// parity-folded sums of Eq. (14)/(26),
//   a[l, col] = sum_p lambda_lm(z_p) X_{E/O}[p, col]   (K = ring pairs),
// for groups of 8 channels (col = (channel, re/im), 16 columns), as
// v_mfma_f64_16x16x4_f64 products with FP64 accumulation.  A is 16 x 4 (lane
// j holds A[j % 16][j / 16]), B is 4 x 16 (lane j holds B[j / 16][j % 16]),
// the 16 x 16 accumulator holds D[j / 16 + 4 r][j % 16] in lane j, register
// r (checked on the device: rows step by 4 across the registers).  Rows are
// 16 l of one parity, K four ring pairs, columns the 16 (channel, re/im) of
// the group.
//
// lambda comes from the FP64 recurrence of Eq. (16) on mu = lambda / c
// (tables.hip), restarted at every block of kBlockL l from the stored
// checkpoints; the c_lm factor is applied to the sums.  The FP64 matrix
// instruction does 1024 fused multiply-adds at the FP64 vector rate with its
// operands in registers, where the vector-ALU kernel needs a load or a
// broadcast per product.
//
// Work split: a workgroup takes one (m, l0) item of the XCD-grouped block
// list; its NW waves (one or two, by size) take 64-ring slices of every
// 64 NW-ring chunk, one ring per lane.  Per 32-l sub-tile a lane writes its ring's 32 mu values into
// its wave's LDS tile (rows: the 16 even l, then the 16 odd l; columns: the
// 64 rings), and the wave multiplies the two 16-row parity tiles with the
// slice's spectra E and O, held in registers for the whole block.  K step
// 2 t + e of lane group q (= lane / 16) is ring 8 t + 2 q + e of the slice,
// so one 16-byte LDS read gives a lane the A values of two K steps.  The
// waves' partial sums are added through LDS at the end.
#include "common.h"

namespace shtx {

typedef double f64x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4_t mfma64(double a, double b, f64x4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kSub64 = 32;      // l per LDS sub-tile
constexpr int kRS64 = 64 + 2;   // tile row stride in doubles: 16-byte rows, a
                                // column read of 16 rows hits 16 distinct bank groups
constexpr int kRed64 = 16 + 1;  // row stride of the cross-wave reduction (doubles)
// LDS doubles per wave: the lambda tile, or the wave's share of the
// cross-wave reduction at the end (the larger)
constexpr int kTile64 = kSub64 * kRS64;
constexpr int kRedN64 = kBlockL * kRed64;
constexpr int kLds64 = kTile64 > kRedN64 ? kTile64 : kRedN64;
static_assert(kBlockL == 4 * kSub64, "four sub-tiles per block");

template <int NW>
__global__ void __launch_bounds__(64 * NW)
    k_legendre_fwd_mfma64(Tables tb, int B, const double *__restrict__ coefA, const double2 *__restrict__ XE,
                          const double2 *__restrict__ XO, double2 *__restrict__ alm, double f0, double fm,
                          int accum) {
  const int b0 = 8 * blockIdx.y;  // channel group of this row of the grid
  __shared__ __attribute__((aligned(16))) double lds[NW * kLds64];
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
  const int q = j >> 4, n = j & 15;
  // column n: channel b0 + n / 2, re or im; channels beyond the batch read
  // channel B - 1 (finite data; their sums are not stored)
  const int cch = min(b0 + (n >> 1), B - 1);
  {
    const double *Ag = coefA + alm_idx(m, m, L) - m;
    for (int t = tid; t < kBlockL; t += 64 * NW) sA[t] = Ag[min(l0 + t, L)];
  }
  __syncthreads();
  double *tw = lds + w * kSub64 * kRS64;
  const double *xe = reinterpret_cast<const double *>(XE);
  const double *xo = reinterpret_cast<const double *>(XO);

  f64x4_t acc[8];  // [sub-tile][parity]
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[a][r] = 0.0;

  // this lane's ring per chunk: recurrence start (kBlockL: idle in this
  // block), checkpoint (mu_{l-1}, mu_l) there, z; fetched one chunk ahead
  auto fetch_ring = [&](int p, int &t0, double2 &v, double &z) {
    const bool ok = p < Rp;
    t0 = ok ? (int)tb.ck_t[(size_t)item * Rp + p] : kBlockL;
    v = ok ? tb.ck_v[(size_t)item * Rp + p] : make_double2(0.0, 0.0);
    z = ok ? tb.rp_z[p] : 0.0;
  };
  int t0n;
  double2 vn;
  double zn;
  fetch_ring(w * 64 + j, t0n, vn, zn);
  for (int c0 = 0; c0 < Rp; c0 += 64 * NW) {
    const int t0 = t0n;
    const double2 v = vn;
    const double z = zn;
    asm volatile("" ::"v"(t0), "v"(v.x), "v"(v.y), "v"(z));
    fetch_ring(c0 + 64 * NW + w * 64 + j, t0n, vn, zn);
    if (__all(t0 >= kBlockL)) continue;  // no ring of this slice is active here
    // last start offset of the slice (later groups need no injection
    // selects) and first (sub-tiles before it hold only zero lambdas)
    int tx = t0 < kBlockL ? t0 : -1, tn = t0;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      tx = max(tx, __shfl_xor(tx, o));
      tn = min(tn, __shfl_xor(tn, o));
    }
    const int tlast = __builtin_amdgcn_readfirstlane(tx);
    const int tfirst = __builtin_amdgcn_readfirstlane(tn);
    // B operands of the slice, K step s: ring 8 (s / 2) + 2 q + s % 2 (rings
    // beyond the last pair read the last pair: their lambda is zero)
    const int rw = c0 + w * 64;
    double be[16], bo[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int r = min(rw + 8 * (s >> 1) + 2 * q + (s & 1), Rp - 1);
      const size_t o = 2 * (((size_t)r * M + m) * B + cch) + (n & 1);
      be[s] = xe[o];
      bo[s] = xo[o];
    }
    // issue the loads here, ahead of the recurrence
    asm volatile("" ::: "memory");
    double prv = 0.0, cur = 0.0;
#pragma unroll
    for (int sub = 0; sub < 4; ++sub) {
      // sub-tiles with no lambda: every ring of the slice starts after it, or
      // every l of it is beyond lmax (then so are the later ones)
      if (tfirst >= (sub + 1) * kSub64) continue;
      if (l0 + sub * kSub64 > L) break;
#pragma unroll 1
      for (int t8 = 0; t8 < kSub64 / 8; ++t8) {
        const int tb8 = sub * kSub64 + t8 * 8;
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
        // row of l = l0 + tb8 + u in the tile: parity * 16 + (t8 * 8 + u) / 2
        double *trow = tw + (t8 * 4) * kRS64 + j;
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
            trow[((u & 1) * 16 + (u >> 1)) * kRS64] = cur;
          }
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const double nx = fma(Ac[u] * z, cur, -prv);
            prv = cur;
            cur = nx;
            trow[((u & 1) * 16 + (u >> 1)) * kRS64] = cur;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // contraction: parity tile par (rows l0 + 32 sub + 2 i + par), 16 K
      // steps of 4 rings
      const double *ae = tw + n * kRS64 + 2 * q;
      const double *ao = tw + (16 + n) * kRS64 + 2 * q;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const double2 e2 = *reinterpret_cast<const double2 *>(ae + 8 * t);
        const double2 o2 = *reinterpret_cast<const double2 *>(ao + 8 * t);
        acc[2 * sub + 0] = mfma64(e2.x, be[2 * t], acc[2 * sub + 0]);
        acc[2 * sub + 1] = mfma64(o2.x, bo[2 * t], acc[2 * sub + 1]);
        acc[2 * sub + 0] = mfma64(e2.y, be[2 * t + 1], acc[2 * sub + 0]);
        acc[2 * sub + 1] = mfma64(o2.y, bo[2 * t + 1], acc[2 * sub + 1]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // sum the waves' partial tiles, red[w][l - l0][col], and write the
  // caller's layout alm[b][idx(l, m)] = f_m c_lm a (Im = 0 for m = 0), or add
  __syncthreads();
  double *red = lds;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int sub = a >> 1, par = a & 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lrel = sub * kSub64 + 2 * (q + 4 * r) + par;
      red[(w * kBlockL + lrel) * kRed64 + n] = acc[a][r];
    }
  }
  __syncthreads();
  const double *Cn = tb.coefC + alm_idx(m, m, L) - m;
  const size_t nalm = nalm_of(L);
  const size_t base = alm_idx(l0, m, L);
  const double f = (m == 0) ? f0 : fm;
  for (int e = tid; e < 8 * kBlockL; e += 64 * NW) {
    const int c = e / kBlockL, lrel = e % kBlockL;
    const int l = l0 + lrel;
    if (l > L || b0 + c >= B) continue;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      re += red[(ww * kBlockL + lrel) * kRed64 + 2 * c];
      im += red[(ww * kBlockL + lrel) * kRed64 + 2 * c + 1];
    }
    const double gg = f * Cn[l];
    double2 val = make_double2(gg * re, (m == 0) ? 0.0 : gg * im);
    double2 *dst = alm + (size_t)(b0 + c) * nalm + base + lrel;
    if (accum) {
      const double2 o = *dst;
      val.x += o.x;
      val.y += o.y;
    }
    *dst = val;
  }
}

// Synthesis, Eq. (24): S_{N/S}[p, col] = sum_l lambda_lm(z_p) a[l, col] with
// the even-l (E) and odd-l (O) sums combined as E + O (north) and E - O
// (south).  Workgroup = one wave = (m, chunk of 64 ring pairs), one ring per
// lane, CT 16-column tiles of 8 channels (CT = 2: 16 channels; CT = 1 for
// groups of at most 8, where a second tile would be padding).  Rows are rings, K is l: per 8
// steps of l every lane advances its ring's recurrence by 8 values; the four
// even-l values (l, l+2, l+4, l+6) of all 64 rings then form the A operands
// of the four 16-ring tiles by one 4 x 4 transpose of (register, 16-lane row)
// blocks (two v_permlane32_swap and two v_permlane16_swap per 32 bits), and
// likewise the odd-l values: K index q of a tile is l + 2 q (+ 1).  The B
// operands (a[l + 2 q (+ 1)][col]) come from the coefficient slab of m, one
// group ahead.  Workgroups are dealt so that the chunks of eight consecutive
// m run on one XCD (they share the coefficient slabs in L2).
constexpr int kInv64Rings = 64;

// out[t] row q = in[q] row t for the four 16-lane rows q, t of a wave
__device__ __forceinline__ void row_transpose4(const double (&in)[4], double (&out)[4]) {
  unsigned lo[4], hi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned long long u = __double_as_longlong(in[k]);
    lo[k] = (unsigned)u;
    hi[k] = (unsigned)(u >> 32);
  }
  auto tr = [](unsigned (&x)[4]) {
    const auto a = __builtin_amdgcn_permlane32_swap(x[0], x[2], false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(x[1], x[3], false, false);
    const auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
    const auto d = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
    x[0] = c[0];
    x[1] = c[1];
    x[2] = d[0];
    x[3] = d[1];
  };
  tr(lo);
  tr(hi);
#pragma unroll
  for (int k = 0; k < 4; ++k)
    out[k] = __longlong_as_double((long long)(((unsigned long long)hi[k] << 32) | lo[k]));
}

template <int CT>
__global__ void __launch_bounds__(64)
    k_legendre_inv_mfma64(Tables tb, int B, int bg, const double *__restrict__ coefA,
                          const double2 *__restrict__ ALMT, SynLayout lay, double2 *__restrict__ GN,
                          double2 *__restrict__ GS) {
  const int b0 = bg + 8 * CT * blockIdx.y;  // channel group of this row of the grid
  const int L = tb.lmax, Rp = tb.npairs;
  const int nch = (Rp + kInv64Rings - 1) / kInv64Rings;
  const int g = blockIdx.x;
  const int x = g & 7, gq = g >> 3;
  // XCD x takes the octets x, x+8, ... of m; within an octet, m-major then chunk
  const int oct = x + 8 * (gq / (8 * nch));
  const int r8 = gq % (8 * nch);
  const int m = 8 * oct + r8 / nch;
  const int chunk = r8 % nch;
  if (m > L) return;  // uniform
  const int j = threadIdx.x;
  const int q = j >> 4, n = j & 15;
  const int p = chunk * kInv64Rings + j;
  const bool pok = p < Rp;
  const double z = pok ? tb.rp_z[p] : 0.0;
  const int ls = pok ? tb.seed_l[(size_t)m * Rp + p] : L + 1;
  const double2 sd = pok ? tb.seed_v[(size_t)m * Rp + p] : make_double2(0.0, 0.0);
  // first l any ring of each 16-ring tile needs (seeds are aligned to m + 8 k)
  int wh = ls;
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) wh = min(wh, __shfl_xor(wh, o));
  int wl_t[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) wl_t[t] = __builtin_amdgcn_readfirstlane(__shfl(wh, 16 * t));
  const int wl = min(min(wl_t[0], wl_t[1]), min(wl_t[2], wl_t[3]));
  f64x4_t acc[4][2][CT];  // [tile][parity][column tile]
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[t][e][c][r] = 0.0;
  // A[l] of this m through the constant address space: wave-uniform indices
  // become scalar loads (32-bit index arithmetic; nalm < 2^31)
  typedef __attribute__((address_space(4))) const double cdouble;
  const int aoff = m * (2 * L + 1 - m) / 2;  // alm_idx(m, m, L) - m
  const cdouble *Ag = (const cdouble *)coefA + aoff;
  // this lane's columns of the coefficient slab a[l][col] (channels beyond the
  // batch read channel B-1: finite data, outputs not stored); rows past lmax
  // (at most 7, inside the padded coefficient workspace) are read and then
  // zeroed with their lambda in the last group
  const double *ag = reinterpret_cast<const double *>(ALMT) + (size_t)aoff * B * 2;
  int cofs[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) cofs[c] = 2 * min(b0 + 8 * c + (n >> 1), B - 1) + (n & 1);
  const size_t arow = 2 * (size_t)B;  // doubles per row l
  auto fetchB = [&](int lq, double (&bv)[2][CT]) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int c = 0; c < CT; ++c) bv[e][c] = ag[(size_t)(lq + 2 * q + e) * arow + cofs[c]];
  };
  double prv = 0.0, cur = 0.0;
  // one group of 8 steps from l = lq with its operands bc (B) and ac (A_l);
  // the next group's go to bn, an (two register sets alternate)
  auto group = [&](int lq, const double (&bc)[2][CT], const double (&ac)[8], double (&bn)[2][CT],
                   double (&an)[8]) {
    const int ln = lq + 8 <= L ? lq + 8 : lq;
    fetchB(ln, bn);
    int la = ln;
    asm volatile("" : "+s"(la) : "s"(ac[7]));
#pragma unroll
    for (int u = 0; u < 8; ++u) an[u] = Ag[la + u];
    double lam[8];
    // a ring's state is exactly zero before its seed, so the seed enters as a
    // 0/1 factor on two fused multiply-adds
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
      lam[u] = cur;
    }
    double bb[2][CT];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int c = 0; c < CT; ++c) bb[e][c] = bc[e][c];
    if (lq + 7 > L) {  // last group: l beyond lmax contributes nothing
#pragma unroll
      for (int u = 0; u < 8; ++u) lam[u] = (lq + u <= L) ? lam[u] : 0.0;
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int c = 0; c < CT; ++c) bb[e][c] = (lq + 2 * q + e <= L) ? bb[e][c] : 0.0;
    }
    double te[4], to[4];
    row_transpose4({lam[0], lam[2], lam[4], lam[6]}, te);
    row_transpose4({lam[1], lam[3], lam[5], lam[7]}, to);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (lq + 7 < wl_t[t]) continue;  // uniform: no ring of the tile has started
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        acc[t][0][c] = mfma64(te[t], bb[0][c], acc[t][0][c]);
        acc[t][1][c] = mfma64(to[t], bb[1][c], acc[t][1][c]);
      }
    }
  };
  double bA[2][CT], bB[2][CT];
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
  // ring 16 t + q + 4 r of the chunk, column n of tile c
  double *gn = reinterpret_cast<double *>(GN);
  double *gs = reinterpret_cast<double *>(GS);
  const size_t ringd = (size_t)lay.ns * lay.M * lay.G * 2;  // doubles per ring pair
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int ch = b0 + 8 * c + (n >> 1);
    if (ch >= B) continue;
    const size_t co = lay.idx(0, ch, m) * 2 + (n & 1);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pr = chunk * kInv64Rings + 16 * t + q + 4 * r;
        if (pr >= Rp) continue;
        const size_t o = (size_t)pr * ringd + co;
        gn[o] = acc[t][0][c][r] + acc[t][1][c][r];
        gs[o] = acc[t][0][c][r] - acc[t][1][c][r];
      }
  }
}

hipError_t launch_legendre_fwd_mfma64(const Tables &tb, int B, const double2 *XE, const double2 *XO, double2 *alm,
                                      double f0, double fm, int accum, hipStream_t st) {
  if (tb.nitems == 0 || (B + 7) / 8 > 65535) return hipErrorInvalidValue;
  // grid: 8 XCD groups x the longest group (item counts per group follow the
  // enumeration of the item table)
  int longest = 0;
  for (int xg = 0; xg < 8; ++xg) {
    int c = 0;
    for (int m = xg; m <= tb.lmax; m += 8) c += (tb.lmax - m + kBlockL) / kBlockL;
    longest = c > longest ? c : longest;
  }
  // one wave per workgroup from 2048 ring pairs, two below (as the FP32
  // analysis; Nside 1024 B 16: 4.82 ms against 4.91 with two waves and 5.01
  // with four; Nside 512 B 8: 0.390 ms with two, 0.399 with one)
  const dim3 grid(8 * longest, (B + 7) / 8);
  if (tb.npairs >= 2048)
    hipLaunchKernelGGL(k_legendre_fwd_mfma64<1>, grid, dim3(64), 0, st, tb, B, tb.coefA, XE, XO, alm, f0, fm, accum);
  else
    hipLaunchKernelGGL(k_legendre_fwd_mfma64<2>, grid, dim3(128), 0, st, tb, B, tb.coefA, XE, XO, alm, f0, fm,
                       accum);
  return hipGetLastError();
}

hipError_t launch_legendre_inv_mfma64(const Tables &tb, int B, const double2 *ALMT, SynLayout lay, double2 *GN,
                                      double2 *GS, hipStream_t st) {
  if ((B + 15) / 16 > 65535) return hipErrorInvalidValue;
  const int nch = (tb.npairs + kInv64Rings - 1) / kInv64Rings;
  const int noct = (tb.lmax + 1 + 7) / 8;
  const int per_xcd = ((noct + 7) / 8) * 8 * nch;  // octets per XCD x 8 m x chunks
  // groups of 16 channels, and a last group of at most 8 on one column tile
  const int n16 = (B % 16 != 0 && B % 16 <= 8) ? B / 16 : (B + 15) / 16;
  if (n16 > 0)
    hipLaunchKernelGGL(k_legendre_inv_mfma64<2>, dim3(8 * per_xcd, n16), dim3(64), 0, st, tb, B, 0, tb.coefA, ALMT,
                       lay, GN, GS);
  if (16 * n16 < B)
    hipLaunchKernelGGL(k_legendre_inv_mfma64<1>, dim3(8 * per_xcd, 1), dim3(64), 0, st, tb, B, 16 * n16, tb.coefA,
                       ALMT, lay, GN, GS);
  return hipGetLastError();
}

}  // namespace shtx
