// Resident tables for one (nside, lmax): ring-pair geometry, recurrence
// coefficients, Legendre seeds at each ring's first non-negligible l, and the
// roots of unity of every ring length.  All of it is computed on the device in
// FP64 by the kernels below; nothing is copied from the host.
//
// Legendre normalisation.  The orthonormal lambda_lm of Eq. (8) (with the
// (-1)^m of Eq. (15)) obeys the three-term recurrence of Eq. (16):
//   lambda_l = alpha_l z lambda_{l-1} - alpha_l beta_l lambda_{l-2},
//   alpha_l = sqrt((4l^2-1)/(l^2-m^2)), beta_l = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
// The kernels run it on mu_l = lambda_l / c_l with c_m = c_{m+1} = 1 and
// c_l = alpha_l beta_l c_{l-2}, which turns it into
//   mu_l = A_l z mu_{l-1} - mu_{l-2},   A_l = alpha_l c_{l-1} / c_l,
// one multiply and one fused multiply-add per step; c_l (0.17 .. 1.13 for
// l <= 4095) is applied once per coefficient, outside the ring sums.
#include "common.h"

namespace shtx {

__global__ void k_ring_pairs(int N, int *rp_n, int *rp_sN, int *rp_sS, int *p0n, int *p0d, int *rp_M,
                             int *rp_bsoff, double *z_out, double *sth_out, double *w_out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= 2 * N) return;
  const int i = p + 1;  // north ring number, 1 .. 2N
  const long long npix = 12LL * N * N;
  int n, sN, num, den;
  double z;
  if (i < N) {  // north polar cap
    n = 4 * i;
    z = 1.0 - (double)((long long)i * i) / (3.0 * (double)N * (double)N);
    sN = 2 * i * (i - 1);
    num = 1;
    den = 4 * i;
  } else {  // belt, north half (incl. equator)
    n = 4 * N;
    z = (double)(4 * N - 2 * i) / (3.0 * (double)N);
    sN = 2 * N * (N - 1) + 4 * N * (i - N);
    if (((i - N) & 1) == 0) {
      num = 1;
      den = 4 * N;
    } else {
      num = 0;
      den = 1;
    }
  }
  // south partner 4N - i: same length and phi0; RING start by symmetry
  const int sS = (i == 2 * N) ? sN : (int)(npix - (long long)sN - n);
  // Bluestein length and offset of this ring length in the chirp-transform table
  int M = 0, off = 0;
  if (i < N) {
    M = bluestein_len(i);
    for (int j = 1; j < i; ++j) off += bluestein_len(j);
  }
  rp_M[p] = M;
  rp_bsoff[p] = off;
  rp_n[p] = n;
  rp_sN[p] = sN;
  rp_sS[p] = sS;
  p0n[p] = num;
  p0d[p] = den;
  z_out[p] = z;
  sth_out[p] = sqrt((1.0 - z) * (1.0 + z));
  w_out[p] = 4.0 * M_PI / (double)npix;
}

// One thread per m: c_lm and A_lm for l = m..L (m-major packed index).
__global__ void k_coefs(int L, double *coefA, double *coefC) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m > L) return;
  if (m == L) {
    const size_t n = nalm_of(L);
    for (size_t i = 0; i < kCoefPadTable; ++i) coefA[n + i] = coefC[n + i] = 0.0;
  }
  const double dm = m;
  double c2 = 1.0, c1 = 1.0;  // c_{l-2}, c_{l-1}
  size_t base = alm_idx(m, m, L);
  coefC[base] = 1.0;
  coefA[base] = 0.0;
  for (int l = m + 1; l <= L; ++l) {
    const double dl = l;
    const double alpha = sqrt((4.0 * dl * dl - 1.0) / (dl * dl - dm * dm));
    double c;
    if (l == m + 1) {
      c = 1.0;
    } else {
      const double beta = sqrt(((dl - 1.0) * (dl - 1.0) - dm * dm) / (4.0 * (dl - 1.0) * (dl - 1.0) - 1.0));
      c = alpha * beta * c2;
    }
    coefC[base + (l - m)] = c;
    coefA[base + (l - m)] = alpha * c1 / c;
    c2 = c1;
    c1 = c;
  }
}

// One thread per ring pair: lambda_mm for m = 0..L as (mantissa, exponent),
// lambda_mm = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}, lambda_00 = 1/sqrt(4 pi).
// Stashed in seed_v[m*Rp + p] = (mantissa, exponent) for k_seeds.
__global__ void k_lambda_mm(int L, int Rp, const double *sth, double2 *stash) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= Rp) return;
  const double s = sth[p];
  double x = 1.0 / sqrt(4.0 * M_PI);
  int e = 0;
  stash[p] = make_double2(x, 0.0);
  for (int m = 1; m <= L; ++m) {
    x *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
    int de;
    x = frexp(x, &de);
    e += de;
    stash[(size_t)m * Rp + p] = make_double2(x, (double)e);
  }
}

// One thread per (m, p): walk mu_l from l = m (value x * 2^e, rescaled to keep
// the mantissas in range) to the first l with |mu_l| >= 2^kSkipExp, align that
// start down to m + kAlign*j, and store the plain doubles (mu_{ls-1}, mu_ls)
// there.  Rings that never reach the threshold get ls = L+1.
__global__ void k_seeds(int L, int Rp, const double *zarr, const double *coefA, int *seed_l,
                        double2 *seed_v) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (p >= Rp) return;
  const size_t slot = (size_t)m * Rp + p;
  const double2 st = seed_v[slot];
  const double z = zarr[p];
  const double *A = coefA + alm_idx(m, m, L) - m;  // A[l]
  const int e0 = (int)st.y;
  // pass 1: find the first l whose value reaches the threshold
  int lstar = L + 1;
  {
    double a = 0.0, b = st.x;  // mu_{l-1}, mu_l mantissas
    int e = e0;
    for (int l = m; l <= L; ++l) {
      if (l > m) {
        const double nb = A[l] * z * b - a;
        a = b;
        b = nb;
      }
      if (b != 0.0 && ilogb(b) + e >= kSkipExp) {
        lstar = l;
        break;
      }
      if (fabs(b) > 0x1p300) {
        a = ldexp(a, -300);
        b = ldexp(b, -300);
        e += 300;
      }
    }
  }
  if (lstar > L) {
    seed_l[slot] = L + 1;
    seed_v[slot] = make_double2(0.0, 0.0);
    return;
  }
  const int ls = m + ((lstar - m) / kAlign) * kAlign;
  // pass 2: rerun up to ls and convert to plain doubles
  double a = 0.0, b = st.x;
  int e = e0;
  for (int l = m + 1; l <= ls; ++l) {
    const double nb = A[l] * z * b - a;
    a = b;
    b = nb;
    if (fabs(b) > 0x1p300) {
      a = ldexp(a, -300);
      b = ldexp(b, -300);
      e += 300;
    }
  }
  seed_l[slot] = ls;
  seed_v[slot] = make_double2(ldexp(a, e), ldexp(b, e));
}

// Roots exp(-2 pi i k / n) for n = 4i, i = blockIdx.y + 1.
__global__ void k_roots(int N, double2 *r64, float2 *r32) {
  const int i = blockIdx.y + 1;
  const int n = 4 * i;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s, c;
  sincospi((double)k / (2.0 * (double)i), &s, &c);
  const size_t o = roots_offset(i) + k;
  r64[o] = make_double2(c, -s);
  r32[o] = make_float2((float)c, (float)-s);
}

// Bluestein chirp c_j = exp(-i pi j^2 / i) for j < i (Eq. (19) for the
// length-i DFTs of a ring of length 4i), with j^2 reduced modulo 2i exactly;
// stored at the ring's offset in the root-table layout.
__global__ void k_chirp(int N, double2 *c64, float2 *c32) {
  const int i = blockIdx.y + 1;
  if (bluestein_len(i) == 0) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= i) return;
  const int r = (int)(((long long)j * j) % (2 * i));
  double s, c;
  sincospi((double)r / (double)i, &s, &c);
  const size_t o = roots_offset(i) + j;
  c64[o] = make_double2(c, -s);
  c32[o] = make_float2((float)c, (float)-s);
}

// b_j = conj(c_{|j|}) for |j| < i, wrapped onto length M, zero elsewhere.
__global__ void k_bhat_init(int N, const int *rp_bsoff, const double2 *c64, double2 *buf) {
  const int i = blockIdx.y + 1;
  const int M = bluestein_len(i);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (M == 0 || j >= M) return;
  const double2 *c = c64 + roots_offset(i);
  double2 v = make_double2(0.0, 0.0);
  if (j < i)
    v = make_double2(c[j].x, -c[j].y);
  else if (j > M - i)
    v = make_double2(c[M - j].x, -c[M - j].y);
  buf[rp_bsoff[i - 1] + j] = v;
}

// One radix-2 Stockham stage (span p = 2^s) of the length-M forward FFT of
// every Bluestein ring, FP64, global memory ping-pong; rings whose FFT has
// fewer stages copy through so that all results end in the same buffer.
__global__ void k_bhat_fft_stage(int N, int s, const int *rp_bsoff, const double2 *src, double2 *dst) {
  const int i = blockIdx.y + 1;
  const int M = bluestein_len(i);
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (M == 0 || b >= M / 2) return;
  const int off = rp_bsoff[i - 1];
  const int h = M / 2;
  if ((1 << s) >= M) {
    dst[off + b] = src[off + b];
    dst[off + b + h] = src[off + b + h];
    return;
  }
  const int p = 1 << s;
  const int k = b & (p - 1);
  double sn, cs;
  sincospi((double)k / (double)p, &sn, &cs);  // exp(-2 pi i k / (2p))
  const double2 u0 = src[off + b];
  const double2 x1 = src[off + b + h];
  const double2 u1 = make_double2(x1.x * cs + x1.y * sn, x1.y * cs - x1.x * sn);
  const int o = ((b - k) << 1) + k;
  dst[off + o] = make_double2(u0.x + u1.x, u0.y + u1.y);
  dst[off + o + p] = make_double2(u0.x - u1.x, u0.y - u1.y);
}

__global__ void k_bhat_finish(size_t nb, const double2 *src, double2 *b64, float2 *b32) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb) return;
  const double2 v = src[j];
  b64[j] = v;
  b32[j] = make_float2((float)v.x, (float)v.y);
}

// Roots exp(-2 pi i k / M) of the largest Bluestein length.
__global__ void k_rootsP(int M, double2 *r64, float2 *r32) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)M, &s, &c);
  r64[k] = make_double2(c, -s);
  r32[k] = make_float2((float)c, (float)-s);
}

// Analysis block list: items (m, l0 = m + kBlockL*b), grouped by XCD (m mod 8
// goes to XCD m mod 8, since consecutive workgroups are dealt round-robin to
// the 8 XCDs) and ordered by m inside each group, so that all blocks of one
// m share one L2.  Single thread.
__global__ void k_items(int L, int2 *items, int *xoff, int *pos) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int k = 0;
  for (int x = 0; x < 8; ++x) {
    xoff[x] = k;
    for (int m = x; m <= L; m += 8) {
      pos[m] = k;
      for (int l0 = m; l0 <= L; l0 += kBlockL) items[k++] = make_int2(m, l0);
    }
  }
  xoff[8] = k;
}

// Checkpoints of the recurrence at every analysis block start: one thread per
// (m, p) runs mu from its seed l_s to lmax with the same operation sequence as
// the transform kernels and records, per block, where the ring starts inside
// the block and the pair (mu_{l-1}, mu_l) there.
__global__ void k_checkpoints(int L, int Rp, const double *zarr, const double *coefA, const int *seed_l,
                              const double2 *seed_v, const int *pos, uint8_t *ck_t, double2 *ck_v) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (p >= Rp) return;
  const size_t slot = (size_t)m * Rp + p;
  const int ls = seed_l[slot];
  const double2 sd = seed_v[slot];
  const double z = zarr[p];
  const double *A = coefA + alm_idx(m, m, L) - m;
  double prv = sd.x, cur = sd.y;
  int lc = ls;  // l of the state (prv, cur)
  const int base = pos[m];
  for (int b = 0, l0 = m; l0 <= L; ++b, l0 += kBlockL) {
    const size_t o = (size_t)(base + b) * Rp + p;
    if (ls > L || ls >= l0 + kBlockL) {
      ck_t[o] = (uint8_t)kBlockL;
      ck_v[o] = make_double2(0.0, 0.0);
    } else if (ls >= l0) {
      ck_t[o] = (uint8_t)(ls - l0);
      ck_v[o] = sd;
    } else {
      while (lc < l0) {
        ++lc;
        const double nx = fma(A[lc] * z, cur, -prv);
        prv = cur;
        cur = nx;
      }
      ck_t[o] = 0;
      ck_v[o] = make_double2(prv, cur);
    }
  }
}

// One thread per NESTED pixel p = f N^2 + interleave(x, y) (x in the even
// bits): its RING index from the face's corner ring rf and longitude position
// qf (HEALPix grid definition, Sec. III-A/III-B): ring i = rf N - x - y - 1,
// 1-based slot j = (qf n + x - y + 1 + s) / 2 cyclic in 1..4n, with n = i,
// 4N - i or N pixels per quadrant (north cap, south cap, belt) and belt shift
// s = (i - N) mod 2; r2n[RING index] = p.
__global__ void k_ring2nest_table(int lgn, uint32_t *r2n) {
  const uint32_t N = 1u << lgn, npix = 12u << (2 * lgn);
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const uint32_t f = p >> (2 * lgn), q = p & ((1u << (2 * lgn)) - 1u);
  uint32_t x = q & 0x55555555u, y = (q >> 1) & 0x55555555u;
  for (int k = 1; k < 16; k <<= 1) {  // compact the even bits
    const uint32_t m = k == 1 ? 0x33333333u : k == 2 ? 0x0f0f0f0fu : k == 4 ? 0x00ff00ffu : 0x0000ffffu;
    x = (x | (x >> k)) & m;
    y = (y | (y >> k)) & m;
  }
  const int row = (int)(f >> 2), rf = row + 2, qf = 2 * (int)(f & 3u) + (row != 1);
  const int i = rf * (int)N - (int)x - (int)y - 1;
  int n, s;
  uint32_t start;
  if (i < (int)N) {
    n = i;
    s = 0;
    start = 2u * (uint32_t)i * (uint32_t)(i - 1);
  } else if (i > 3 * (int)N) {
    n = 4 * (int)N - i;
    s = 0;
    start = npix - 2u * (uint32_t)n * (uint32_t)(n + 1);
  } else {
    n = (int)N;
    s = (i - (int)N) & 1;
    start = 2u * N * (N - 1u) + 4u * N * (uint32_t)(i - (int)N);
  }
  int j = (qf * n + (int)x - (int)y + 1 + s) >> 1;
  if (j > 4 * n) j -= 4 * n;
  if (j < 1) j += 4 * n;
  r2n[start + (uint32_t)(j - 1)] = p;
}

hipError_t launch_tables_build(int nside, int lmax, void *base, hipStream_t st) {
  const TableOffsets o = table_offsets(nside, lmax);
  char *b = static_cast<char *>(base);
  const int Rp = 2 * nside;
  auto I = [&](size_t off) { return reinterpret_cast<int *>(b + off); };
  auto D = [&](size_t off) { return reinterpret_cast<double *>(b + off); };
  hipLaunchKernelGGL(k_ring_pairs, dim3((Rp + 255) / 256), dim3(256), 0, st, nside, I(o.rp_n), I(o.rp_sN),
                     I(o.rp_sS), I(o.rp_p0n), I(o.rp_p0d), I(o.rp_M), I(o.rp_bsoff), D(o.rp_z), D(o.rp_sth),
                     D(o.rp_w));
  hipLaunchKernelGGL(k_coefs, dim3((lmax + 1 + 63) / 64), dim3(64), 0, st, lmax, D(o.coefA), D(o.coefC));
  {
    const uint32_t npix = 12u * (uint32_t)nside * (uint32_t)nside;
    hipLaunchKernelGGL(k_ring2nest_table, dim3((npix + 255) / 256), dim3(256), 0, st, __builtin_ctz((unsigned)nside),
                       reinterpret_cast<uint32_t *>(b + o.r2n));
  }
  double2 *sv = reinterpret_cast<double2 *>(b + o.seed_v);
  hipLaunchKernelGGL(k_lambda_mm, dim3((Rp + 63) / 64), dim3(64), 0, st, lmax, Rp, D(o.rp_sth), sv);
  hipLaunchKernelGGL(k_seeds, dim3((Rp + 63) / 64, lmax + 1), dim3(64), 0, st, lmax, Rp, D(o.rp_z),
                     D(o.coefA), I(o.seed_l), sv);
  hipLaunchKernelGGL(k_roots, dim3((4 * nside + 255) / 256, nside), dim3(256), 0, st, nside,
                     reinterpret_cast<double2 *>(b + o.roots64), reinterpret_cast<float2 *>(b + o.roots32));
  if (o.nitems > 0) {
    hipLaunchKernelGGL(k_items, dim3(1), dim3(64), 0, st, lmax, reinterpret_cast<int2 *>(b + o.ck_items),
                       I(o.ck_xoff), I(o.ck_pos));
    hipLaunchKernelGGL(k_checkpoints, dim3((Rp + 63) / 64, lmax + 1), dim3(64), 0, st, lmax, Rp, D(o.rp_z),
                       D(o.coefA), I(o.seed_l), sv, I(o.ck_pos), reinterpret_cast<uint8_t *>(b + o.ck_t),
                       reinterpret_cast<double2 *>(b + o.ck_v));
  }
  if (o.mmax_bs > 0) {
    auto D2 = [&](size_t off) { return reinterpret_cast<double2 *>(b + off); };
    auto F2 = [&](size_t off) { return reinterpret_cast<float2 *>(b + off); };
    const int ncap = nside - 1;
    hipLaunchKernelGGL(k_chirp, dim3((nside + 255) / 256, ncap), dim3(256), 0, st, nside, D2(o.chirp64),
                       F2(o.chirp32));
    hipLaunchKernelGGL(k_bhat_init, dim3((o.mmax_bs + 255) / 256, ncap), dim3(256), 0, st, nside, I(o.rp_bsoff),
                       D2(o.chirp64), D2(o.bhat_tmp));
    int S = 0;
    while ((1 << S) < o.mmax_bs) ++S;
    double2 *bufs[2] = {D2(o.bhat_tmp), D2(o.bhat64)};
    for (int s = 0; s < S; ++s)
      hipLaunchKernelGGL(k_bhat_fft_stage, dim3((o.mmax_bs / 2 + 255) / 256, ncap), dim3(256), 0, st, nside, s,
                         I(o.rp_bsoff), bufs[s & 1], bufs[(s + 1) & 1]);
    const double2 *res = bufs[S & 1];
    hipLaunchKernelGGL(k_bhat_finish, dim3((unsigned)((o.nbhat + 255) / 256)), dim3(256), 0, st, o.nbhat, res,
                       D2(o.bhat64), F2(o.bhat32));
    hipLaunchKernelGGL(k_rootsP, dim3((o.mmax_bs + 255) / 256), dim3(256), 0, st, o.mmax_bs, D2(o.rootsP64),
                       F2(o.rootsP32));
  }
  return hipGetLastError();
}

}  // namespace shtx
