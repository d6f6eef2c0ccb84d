// C ABI of libshtx.so (declared in include/shtx.h): host-side validation,
// table registry, workspace carving and kernel dispatch.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/shtx.h"
#include "common.h"

namespace shtx {

hipError_t launch_tables_build(int nside, int lmax, void *base, hipStream_t st);
template <typename TIn, typename T, typename TS>
hipError_t launch_ring_fft_fwd(Tables, int, const TIn *, const double *, double, const double *, TS *, TS *,
                               hipStream_t, bool);
hipError_t launch_pack_spectra_bf16(const Tables &, int, const uint32_t *, const uint32_t *, void *, hipStream_t);
hipError_t launch_legendre_fwd_bf16(const Tables &, int, const void *, float2 *, double, double, int, hipStream_t,
                                    const uint32_t *);
size_t bf16_packed_spectra_bytes(int lmax, int npairs, int B);
size_t lam_header_words(int nside, int nitems);
std::vector<uint32_t> lam_tile_offsets(int nside, int lmax, int nitems, const uint8_t *ck_t, const int2 *items,
                                       size_t *ntiles);
hipError_t launch_lambda_table_build(const Tables &tb, uint32_t *lam, hipStream_t st);
constexpr size_t kLamTileBytesHost = 64 * 64 * 4;  // one stored BF16 lambda tile
template <typename TOut, typename T>
hipError_t launch_ring_fft_inv(Tables, int, const cplx<T> *, const cplx<T> *, const TOut *, TOut *, hipStream_t);
template <typename T>
hipError_t launch_legendre_fwd_valu(const Tables &, int, const cplx<T> *, const cplx<T> *, cplx<T> *, double, double,
                                    int, hipStream_t);
template <typename T>
hipError_t launch_legendre_inv_valu(const Tables &, int, const cplx<T> *, SynLayout, cplx<T> *, cplx<T> *,
                                    hipStream_t);
bool mfma_fwd_supported(const Tables &tb);
hipError_t launch_legendre_fwd_mfma(const Tables &, int, const float2 *, const float2 *, float2 *, double, double, int,
                                    hipStream_t);
hipError_t launch_legendre_inv_mfma(const Tables &, int, const float2 *, SynLayout, float2 *, float2 *, hipStream_t);
hipError_t launch_legendre_fwd_mfma64(const Tables &, int, const double2 *, const double2 *, double2 *, double, double,
                                      int, hipStream_t);
hipError_t launch_legendre_inv_mfma64(const Tables &, int, const double2 *, SynLayout, double2 *, double2 *,
                                      hipStream_t);
template <typename T, typename TI>
hipError_t launch_alm_in(int, int, int, const cplx<TI> *, const double *, cplx<T> *, double, double, double,
                         hipStream_t);

namespace {

// ------------------------------------------------------------ stage timing
enum Stage { kStFftFwd = 0, kStLegFwd, kStAlmIn, kStLegInv, kStFftInv, kStPackBf16, kNumStages };
const char *kStageNames[kNumStages] = {"ring_fft_fwd", "legendre_fwd", "alm_in", "legendre_inv",
                                       "ring_fft_inv", "pack_bf16"};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[kNumStages];
  double ms[kNumStages] = {};
  long long n[kNumStages] = {};
} g_prof;

// Records start/stop events around one stage when profiling is on.
struct StageTimer {
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(int s, hipStream_t stream) : stage(s), st(stream) {
    if (!g_prof.on) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    hipEventRecord(a, st);
  }
  ~StageTimer() {
    if (!a) return;
    hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.ev[stage].emplace_back(a, b);
  }
};

void profile_collect() {
  for (int s = 0; s < kNumStages; ++s) {
    for (auto &e : g_prof.ev[s]) {
      float t = 0.f;
      hipEventSynchronize(e.second);
      if (hipEventElapsedTime(&t, e.first, e.second) == hipSuccess) {
        g_prof.ms[s] += t;
        g_prof.n[s] += 1;
      }
      hipEventDestroy(e.first);
      hipEventDestroy(e.second);
    }
    g_prof.ev[s].clear();
  }
}

std::mutex g_mu;
struct Registered {
  int nside, lmax;
  Tables view;
};
std::unordered_map<const void *, Registered> g_tables;
// stored-lambda tables: buffer -> (tables buffer, bytes it needs)
struct LamRegistered {
  const void *tables;
  size_t bytes;
};
std::unordered_map<const void *, LamRegistered> g_lams;

bool valid_geom(int nside, int lmax) {
  if (nside < 1 || (nside & (nside - 1)) != 0) return false;
  if (lmax < 0 || lmax > 8191) return false;
  return true;
}

// map and alm are `in` / `out` or `out` / `in` depending on the direction
int check_common(int nside, int lmax, int batch, int dtype, const void *in, const void *out, const void *tables,
                 const void *work, size_t work_bytes, Tables *view, bool map_in) {
  if (!valid_geom(nside, lmax) || batch < 1) return SHTX_ERR_ARG;
  if (dtype != SHTX_F64 && dtype != SHTX_F32 && dtype != SHTX_BF16) return SHTX_ERR_ARG;
  if (!in || !out || !tables || !work) return SHTX_ERR_ARG;
  if (nside > kMaxNside) return SHTX_ERR_UNSUPPORTED;
  if (reinterpret_cast<uintptr_t>(work) % 256 != 0) return SHTX_ERR_ARG;
  {
    const uintptr_t mp = reinterpret_cast<uintptr_t>(map_in ? in : out);
    const uintptr_t ap = reinterpret_cast<uintptr_t>(map_in ? out : in);
    if (mp % (dtype == SHTX_BF16 ? 8 : 16) != 0) return SHTX_ERR_ARG;
    if (ap % (dtype == SHTX_F64 ? 16 : 8) != 0) return SHTX_ERR_ARG;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tables.find(tables);
    if (it == g_tables.end() || it->second.nside != nside || it->second.lmax != lmax) return SHTX_ERR_TABLES;
    *view = it->second.view;
  }
  if (work_bytes < shtx_workspace_bytes(nside, lmax, batch, dtype)) return SHTX_ERR_WORKSPACE;
  return SHTX_OK;
}

template <typename T> struct Work {
  cplx<T> *specA, *specB, *almt;
};

// Channels of one spectrum buffer: the batch, rounded up to whole channel
// slices of the synthesis layout.
size_t spec_channels(int nside, int lmax, int mmax_bs, int batch, size_t cs) {
  const SynLayout l = syn_layout(nside, lmax, mmax_bs, batch, cs);
  return (size_t)l.ns * (size_t)l.G;
}

size_t spec_bytes(int nside, int lmax, int mmax_bs, int batch, size_t cs) {
  return (size_t)(lmax + 1) * (size_t)(2 * nside) * spec_channels(nside, lmax, mmax_bs, batch, cs) * cs;
}

template <typename T> Work<T> carve(void *work, const Tables &tb, int batch) {
  const size_t spec = spec_bytes(tb.nside, tb.lmax, tb.mmax_bs, batch, sizeof(cplx<T>));
  char *b = static_cast<char *>(work);
  Work<T> w;
  w.specA = reinterpret_cast<cplx<T> *>(b);
  w.specB = reinterpret_cast<cplx<T> *>(b + align_up(spec, 256));
  w.almt = reinterpret_cast<cplx<T> *>(b + 2 * align_up(spec, 256));
  return w;
}

constexpr int kMaxIter = 64;  // refinement iterations accepted by shtx_map2alm_iter

// ---------------------------------------------- allocation-free analysis
// Fixed device scratch of shtx_map2alm_noalloc: the two analysis spectrum
// buffers live here instead of in a caller workspace.  One copy per device,
// held until the process ends; calls on one device share it.  Host code
// never uses the array's name as an address: the device address of each
// device's copy is looked up once (hipGetSymbolAddress, that device current)
// and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = (size_t)SHTX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per device

// Device address of the current device's scratch array (looked up on the
// first call on that device); nullptr and *status set on failure.
void *scratch_ptr(int *status) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *status = SHTX_ERR_HIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      *status = SHTX_ERR_HIP;
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  *status = SHTX_OK;
  return g_scratch_ptr[dev];
}

int status_of(hipError_t e) { return e == hipSuccess ? SHTX_OK : SHTX_ERR_HIP; }

// Matrix-core Legendre kernels serve FP32 contraction from mfma_min_batch()
// channels up: 5 for the analysis, 8 for the synthesis by default (below
// that the 32-column matrix tiles are mostly padding and the vector-ALU
// kernels are faster); SHTX_MFMA_MIN_BATCH sets both.  SHTX_FORCE_VALU=1 in
// the environment selects the vector-ALU kernels everywhere.  Both are read
// per call.
int mfma_min_batch(bool synthesis) {
  const char *e = getenv("SHTX_MFMA_MIN_BATCH");
  return e ? atoi(e) : synthesis ? 8 : 5;
}
// FP64 transforms take the FP64 matrix cores from 3 channels for the
// analysis and 5 for the synthesis (measured at Nside 1024: analysis 2.42 ms
// against 3.84 ms on the vector ALUs at 4 channels, 2.40 against 1.94 at 2;
// synthesis 2.30 against 2.36 at 5, 2.29 against 1.69 at 4; the 16-column
// tiles hold 8 channels); SHTX_MFMA_MIN_BATCH sets both.
int mfma64_min_batch(bool synthesis) {
  const char *e = getenv("SHTX_MFMA_MIN_BATCH");
  return e ? atoi(e) : synthesis ? 5 : 3;
}
bool force_valu() {
  const char *e = getenv("SHTX_FORCE_VALU");
  return e && e[0] == '1';
}

// Legendre step of the analysis; both kernels write the caller's layout
// themselves (factors f0 / fm, optional accumulation).
template <typename T> hipError_t legendre_fwd(const Tables &tb, int B, const cplx<T> *XE, const cplx<T> *XO,
                                              cplx<T> *alm, double f0, double fm, int accum, hipStream_t st) {
  return launch_legendre_fwd_valu<T>(tb, B, XE, XO, alm, f0, fm, accum, st);
}
template <> hipError_t legendre_fwd<double>(const Tables &tb, int B, const double2 *XE, const double2 *XO,
                                            double2 *alm, double f0, double fm, int accum, hipStream_t st) {
  if (B >= mfma64_min_batch(false) && mfma_fwd_supported(tb) && !force_valu())
    return launch_legendre_fwd_mfma64(tb, B, XE, XO, alm, f0, fm, accum, st);
  return launch_legendre_fwd_valu<double>(tb, B, XE, XO, alm, f0, fm, accum, st);
}
template <> hipError_t legendre_fwd<float>(const Tables &tb, int B, const float2 *XE, const float2 *XO, float2 *alm,
                                           double f0, double fm, int accum, hipStream_t st) {
  if (B >= mfma_min_batch(false) && mfma_fwd_supported(tb) && !force_valu())
    return launch_legendre_fwd_mfma(tb, B, XE, XO, alm, f0, fm, accum, st);
  return launch_legendre_fwd_valu<float>(tb, B, XE, XO, alm, f0, fm, accum, st);
}
// Synthesis Legendre kernel of a call: matrix cores (enough channels) or
// vector ALUs; the choice also fixes the channel groups of the coefficient
// buffer (chan_group): one group of all channels for the matrix cores, the
// vector-ALU kernels' groups otherwise.
template <typename T> bool inv_on_mfma(int B) {
  if (force_valu()) return false;
  return sizeof(T) == 4 ? B >= mfma_min_batch(true) : B >= mfma64_min_batch(true);
}

template <typename T> hipError_t legendre_inv(const Tables &tb, int B, const cplx<T> *ALMT, SynLayout lay,
                                              cplx<T> *GN, cplx<T> *GS, bool mfma, hipStream_t st) {
  return launch_legendre_inv_valu<T>(tb, B, ALMT, lay, GN, GS, st);
}
template <> hipError_t legendre_inv<double>(const Tables &tb, int B, const double2 *ALMT, SynLayout lay,
                                            double2 *GN, double2 *GS, bool mfma, hipStream_t st) {
  if (mfma) return launch_legendre_inv_mfma64(tb, B, ALMT, lay, GN, GS, st);
  return launch_legendre_inv_valu<double>(tb, B, ALMT, lay, GN, GS, st);
}
template <> hipError_t legendre_inv<float>(const Tables &tb, int B, const float2 *ALMT, SynLayout lay, float2 *GN,
                                           float2 *GS, bool mfma, hipStream_t st) {
  if (mfma) return launch_legendre_inv_mfma(tb, B, ALMT, lay, GN, GS, st);
  return launch_legendre_inv_valu<float>(tb, B, ALMT, lay, GN, GS, st);
}

// BF16 maps take the BF16 matrix-core contraction (BF16 spectra and
// Legendre operands, FP32 accumulation) where the FP32 analysis would take
// the matrix cores; SHTX_BF16_CONTRACT=f32 in the environment (read per
// call) keeps them on the FP32 contraction.
template <typename TIn> bool bf16_contraction(const Tables &tb, int B) {
  if constexpr (!std::is_same<TIn, bf16_t>::value) {
    return false;
  } else {
    const char *e = getenv("SHTX_BF16_CONTRACT");
    if (e && e[0] == 'f') return false;
    return B >= mfma_min_batch(false) && mfma_fwd_supported(tb) && !force_valu();
  }
}

// analysis chain: ring FFT -> Legendre -> caller layout with factors
template <typename TIn, typename T>
int run_analysis(const Tables &tb, int B, const TIn *map, cplx<T> *alm, const double *wtab, double wscale,
                 double f0, double fm, void *work, hipStream_t st, int accumulate = 0, bool nested = false,
                 const double *pixw = nullptr, const uint32_t *lam = nullptr) {
  Work<T> w = carve<T>(work, tb, B);
  hipError_t e;
  if constexpr (std::is_same<T, float>::value) {
    if (lam || bf16_contraction<TIn>(tb, B)) {
      uint32_t *sa = reinterpret_cast<uint32_t *>(w.specA), *sb = reinterpret_cast<uint32_t *>(w.specB);
      {
        StageTimer t(kStFftFwd, st);
        e = launch_ring_fft_fwd<TIn, T, uint32_t>(tb, B, map, wtab, wscale, pixw, sa, sb, st, nested);
      }
      if (e != hipSuccess) return SHTX_ERR_HIP;
      // the spectra in operand order go where the synthesis keeps its
      // coefficients (unused by the analysis)
      {
        StageTimer t(kStPackBf16, st);
        e = launch_pack_spectra_bf16(tb, B, sa, sb, w.almt, st);
      }
      if (e != hipSuccess) return SHTX_ERR_HIP;
      StageTimer t(kStLegFwd, st);
      return status_of(launch_legendre_fwd_bf16(tb, B, w.almt, alm, f0, fm, accumulate, st, lam));
    }
  }
  {
    StageTimer t(kStFftFwd, st);
    e = launch_ring_fft_fwd<TIn, T, cplx<T>>(tb, B, map, wtab, wscale, pixw, w.specA, w.specB, st, nested);
  }
  if (e != hipSuccess) return SHTX_ERR_HIP;
  StageTimer t(kStLegFwd, st);
  return status_of(legendre_fwd<T>(tb, B, w.specA, w.specB, alm, f0, fm, accumulate, st));
}

// synthesis chain: caller layout with factors -> Legendre -> ring FFT
template <typename TOut, typename T>
int run_synthesis(const Tables &tb, int B, const cplx<T> *alm, TOut *map, double s, double f0, double fm, void *work,
                  hipStream_t st, const TOut *sub = nullptr) {
  Work<T> w = carve<T>(work, tb, B);
  const bool mfma = inv_on_mfma<T>(B);  // read once: both kernels follow the same choice
  hipError_t e;
  {
    StageTimer t(kStAlmIn, st);
    const int gmax = mfma ? B : sizeof(T) == 8 ? 2 : 4;
    e = launch_alm_in<T, T>(tb.lmax, B, gmax, alm, tb.coefC, w.almt, s, f0, fm, st);
  }
  if (e != hipSuccess) return SHTX_ERR_HIP;
  {
    StageTimer t(kStLegInv, st);
    e = legendre_inv<T>(tb, B, w.almt, syn_layout(tb.nside, tb.lmax, tb.mmax_bs, B, sizeof(cplx<T>)), w.specA,
                        w.specB, mfma, st);
  }
  if (e != hipSuccess) return SHTX_ERR_HIP;
  StageTimer t(kStFftInv, st);
  return status_of(launch_ring_fft_inv<TOut, T>(tb, B, w.specA, w.specB, sub, map, st));
}

}  // namespace
}  // namespace shtx

using namespace shtx;

extern "C" {

int shtx_version(void) { return 100; }

int shtx_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  return SHTX_OK;
}

int shtx_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  profile_collect();
  for (int s = 0; s < kNumStages; ++s) {
    g_prof.ms[s] = 0.0;
    g_prof.n[s] = 0;
  }
  return SHTX_OK;
}

int shtx_profile_read(int stage, double *total_ms, long long *launches) {
  if (stage < 0 || stage >= kNumStages || !total_ms || !launches) return SHTX_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  profile_collect();
  *total_ms = g_prof.ms[stage];
  *launches = g_prof.n[stage];
  return SHTX_OK;
}

const char *shtx_stage_name(int stage) {
  if (stage < 0 || stage >= kNumStages) return "unknown";
  return kStageNames[stage];
}

const char *shtx_status_string(int status) {
  switch (status) {
    case SHTX_OK: return "ok";
    case SHTX_ERR_ARG: return "invalid argument";
    case SHTX_ERR_UNSUPPORTED: return "unsupported configuration";
    case SHTX_ERR_WORKSPACE: return "workspace too small";
    case SHTX_ERR_HIP: return "HIP runtime error";
    case SHTX_ERR_TABLES: return "tables not built for this (nside, lmax)";
    case SHTX_ERR_SCRATCH: return "request needs more than the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

size_t shtx_tables_bytes(int nside, int lmax) {
  if (!valid_geom(nside, lmax) || nside > kMaxNside) return 0;
  return table_offsets(nside, lmax).total;
}

int shtx_tables_build(int nside, int lmax, void *tables, size_t tables_bytes, void *stream) {
  if (!valid_geom(nside, lmax) || !tables) return SHTX_ERR_ARG;
  if (nside > kMaxNside) return SHTX_ERR_UNSUPPORTED;
  if (reinterpret_cast<uintptr_t>(tables) % 256 != 0) return SHTX_ERR_ARG;
  if (tables_bytes < shtx_tables_bytes(nside, lmax)) return SHTX_ERR_WORKSPACE;
  const hipError_t e = launch_tables_build(nside, lmax, tables, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return SHTX_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  g_tables[tables] = Registered{nside, lmax, tables_view(tables, nside, lmax)};
  return SHTX_OK;
}

int shtx_tables_work(const void *tables, long long *executed, long long *full, void *stream) {
  if (!executed || !full) return SHTX_ERR_ARG;
  Registered r;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tables.find(tables);
    if (it == g_tables.end()) return SHTX_ERR_TABLES;
    r = it->second;
  }
  const int L = r.lmax, Rp = 2 * r.nside;
  std::vector<int> ls((size_t)(L + 1) * Rp);
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipMemcpy(ls.data(), r.view.seed_l, ls.size() * sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return SHTX_ERR_HIP;
  long long s = 0;
  for (int v : ls) s += (long long)(L + 1 - std::min(v, L + 1));
  *executed = s;
  *full = (long long)nalm_of(L) * Rp;
  return SHTX_OK;
}

int shtx_tables_release(const void *tables) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tables.erase(tables) ? SHTX_OK : SHTX_ERR_TABLES;
}

size_t shtx_workspace_bytes(int nside, int lmax, int batch, int dtype) {
  if (!valid_geom(nside, lmax) || batch < 1) return 0;
  if (dtype != SHTX_F64 && dtype != SHTX_F32 && dtype != SHTX_BF16) return 0;
  if (nside > kMaxNside) return 0;
  const size_t cs = dtype == SHTX_F64 ? 16 : 8;
  size_t nbhat;
  int mmax_bs;
  bluestein_sizes(nside, &nbhat, &mmax_bs);
  const size_t spec = spec_bytes(nside, lmax, mmax_bs, batch, cs);
  // coefficients [idx][batch] plus kCoefPad rows read (and masked) past lmax
  const size_t almt = (nalm_of(lmax) + kCoefPad) * (size_t)batch * cs;
  // BF16 maps: the analysis' spectra in matrix-operand order share that room
  const size_t third =
      dtype == SHTX_BF16 ? std::max(almt, bf16_packed_spectra_bytes(lmax, 2 * nside, batch)) : almt;
  return 2 * align_up(spec, 256) + align_up(third, 256);
}

int shtx_map2alm(int nside, int lmax, int batch, int dtype, const void *map, void *alm, const void *tables,
                 void *work, size_t work_bytes, void *stream) {
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, map, alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case SHTX_F64:
      return run_analysis<double, double>(tb, batch, static_cast<const double *>(map), static_cast<double2 *>(alm),
                                          tb.rp_w, 1.0, 1.0, 1.0, work, st);
    case SHTX_F32:
      return run_analysis<float, float>(tb, batch, static_cast<const float *>(map), static_cast<float2 *>(alm),
                                        tb.rp_w, 1.0, 1.0, 1.0, work, st);
    default:
      return run_analysis<bf16_t, float>(tb, batch, static_cast<const bf16_t *>(map), static_cast<float2 *>(alm),
                                         tb.rp_w, 1.0, 1.0, 1.0, work, st);
  }
}

size_t shtx_noalloc_scratch_bytes(void) { return kScratchBytes; }

int shtx_map2alm_noalloc(int nside, int lmax, int batch, int dtype, const void *map, void *alm, const void *tables,
                         void *stream) {
  if (!valid_geom(nside, lmax) || batch < 1) return SHTX_ERR_ARG;
  if (dtype != SHTX_F64 && dtype != SHTX_F32 && dtype != SHTX_BF16) return SHTX_ERR_ARG;
  if (nside > kMaxNside) return SHTX_ERR_UNSUPPORTED;
  // the analysis uses the two spectrum buffers of the workspace layout and,
  // for BF16 maps, the operand-order spectra after them (the coefficient
  // buffer serves only the synthesis)
  const size_t cs = dtype == SHTX_F64 ? 16 : 8;
  size_t nbhat;
  int mmax_bs;
  bluestein_sizes(nside, &nbhat, &mmax_bs);
  size_t need = 2 * align_up(spec_bytes(nside, lmax, mmax_bs, batch, cs), 256);
  if (dtype == SHTX_BF16) need += align_up(bf16_packed_spectra_bytes(lmax, 2 * nside, batch), 256);
  if (need > kScratchBytes) return SHTX_ERR_SCRATCH;
  int s = SHTX_OK;
  void *work = scratch_ptr(&s);
  if (!work) return s;
  Tables tb;
  // the scratch stands in for a workspace (check_common's size test is met by
  // construction: only the buffers counted in `need` are touched)
  s = check_common(nside, lmax, batch, dtype, map, alm, tables, work, shtx_workspace_bytes(nside, lmax, batch, dtype),
                   &tb, true);
  if (s != SHTX_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case SHTX_F64:
      return run_analysis<double, double>(tb, batch, static_cast<const double *>(map), static_cast<double2 *>(alm),
                                          tb.rp_w, 1.0, 1.0, 1.0, work, st);
    case SHTX_F32:
      return run_analysis<float, float>(tb, batch, static_cast<const float *>(map), static_cast<float2 *>(alm),
                                        tb.rp_w, 1.0, 1.0, 1.0, work, st);
    default:
      return run_analysis<bf16_t, float>(tb, batch, static_cast<const bf16_t *>(map), static_cast<float2 *>(alm),
                                         tb.rp_w, 1.0, 1.0, 1.0, work, st);
  }
}

int shtx_map2alm_nested(int nside, int lmax, int batch, int dtype, const void *map_nest, void *alm,
                        const void *tables, void *work, size_t work_bytes, void *stream) {
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, map_nest, alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case SHTX_F64:
      return run_analysis<double, double>(tb, batch, static_cast<const double *>(map_nest),
                                          static_cast<double2 *>(alm), tb.rp_w, 1.0, 1.0, 1.0, work, st, 0, true);
    case SHTX_F32:
      return run_analysis<float, float>(tb, batch, static_cast<const float *>(map_nest), static_cast<float2 *>(alm),
                                        tb.rp_w, 1.0, 1.0, 1.0, work, st, 0, true);
    default:
      return run_analysis<bf16_t, float>(tb, batch, static_cast<const bf16_t *>(map_nest),
                                         static_cast<float2 *>(alm), tb.rp_w, 1.0, 1.0, 1.0, work, st, 0, true);
  }
}

int shtx_map2alm_weighted(int nside, int lmax, int batch, int dtype, const void *map, void *alm,
                          const double *ring_weights, const void *tables, void *work, size_t work_bytes,
                          void *stream) {
  if (!ring_weights || (reinterpret_cast<uintptr_t>(ring_weights) & 7)) return SHTX_ERR_ARG;
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, map, alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case SHTX_F64:
      return run_analysis<double, double>(tb, batch, static_cast<const double *>(map), static_cast<double2 *>(alm),
                                          ring_weights, 1.0, 1.0, 1.0, work, st);
    case SHTX_F32:
      return run_analysis<float, float>(tb, batch, static_cast<const float *>(map), static_cast<float2 *>(alm),
                                        ring_weights, 1.0, 1.0, 1.0, work, st);
    default:
      return run_analysis<bf16_t, float>(tb, batch, static_cast<const bf16_t *>(map), static_cast<float2 *>(alm),
                                         ring_weights, 1.0, 1.0, 1.0, work, st);
  }
}

int shtx_map2alm_pixel_weighted(int nside, int lmax, int batch, int dtype, const void *map, void *alm,
                                const double *pixel_weights, const void *tables, void *work, size_t work_bytes,
                                void *stream) {
  if (!pixel_weights || (reinterpret_cast<uintptr_t>(pixel_weights) & 15)) return SHTX_ERR_ARG;
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, map, alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (dtype) {
    case SHTX_F64:
      return run_analysis<double, double>(tb, batch, static_cast<const double *>(map), static_cast<double2 *>(alm),
                                          nullptr, 1.0, 1.0, 1.0, work, st, 0, false, pixel_weights);
    case SHTX_F32:
      return run_analysis<float, float>(tb, batch, static_cast<const float *>(map), static_cast<float2 *>(alm),
                                        nullptr, 1.0, 1.0, 1.0, work, st, 0, false, pixel_weights);
    default:
      return run_analysis<bf16_t, float>(tb, batch, static_cast<const bf16_t *>(map), static_cast<float2 *>(alm),
                                         nullptr, 1.0, 1.0, 1.0, work, st, 0, false, pixel_weights);
  }
}

int shtx_alm2map(int nside, int lmax, int batch, int dtype, const void *alm, void *map, const void *tables,
                 void *work, size_t work_bytes, void *stream) {
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, alm, map, tables, work, work_bytes, &tb, false);
  if (s != SHTX_OK) return s;
  if (dtype == SHTX_BF16) return SHTX_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == SHTX_F64)
    return run_synthesis<double, double>(tb, batch, static_cast<const double2 *>(alm), static_cast<double *>(map),
                                         1.0, 1.0, 1.0, work, st);
  return run_synthesis<float, float>(tb, batch, static_cast<const float2 *>(alm), static_cast<float *>(map), 1.0,
                                     1.0, 1.0, work, st);
}

int shtx_map2alm_backward(int nside, int lmax, int batch, int dtype, const void *grad_alm, void *grad_map,
                          const void *tables, void *work, size_t work_bytes, void *stream) {
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, grad_alm, grad_map, tables, work, work_bytes, &tb, false);
  if (s != SHTX_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double w = 4.0 * M_PI / (double)tb.npix;
  switch (dtype) {
    case SHTX_F64:
      return run_synthesis<double, double>(tb, batch, static_cast<const double2 *>(grad_alm),
                                           static_cast<double *>(grad_map), w, 1.0, 0.5, work, st);
    case SHTX_F32:
      return run_synthesis<float, float>(tb, batch, static_cast<const float2 *>(grad_alm),
                                         static_cast<float *>(grad_map), w, 1.0, 0.5, work, st);
    default:
      return run_synthesis<bf16_t, float>(tb, batch, static_cast<const float2 *>(grad_alm),
                                          static_cast<bf16_t *>(grad_map), w, 1.0, 0.5, work, st);
  }
}

int shtx_alm2map_backward(int nside, int lmax, int batch, int dtype, const void *grad_map, void *grad_alm,
                          const void *tables, void *work, size_t work_bytes, void *stream) {
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, grad_map, grad_alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  if (dtype == SHTX_BF16) return SHTX_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == SHTX_F64)
    return run_analysis<double, double>(tb, batch, static_cast<const double *>(grad_map),
                                        static_cast<double2 *>(grad_alm), nullptr, 1.0, 1.0, 2.0, work, st);
  return run_analysis<float, float>(tb, batch, static_cast<const float *>(grad_map), static_cast<float2 *>(grad_alm),
                                    nullptr, 1.0, 1.0, 2.0, work, st);
}

}  // extern "C"

namespace shtx {
namespace {
// Tile offsets of the stored-lambda table of a registered tables buffer
// (reads the checkpoint starts back to the host: a set-up call).
int lam_layout(const void *tables, Registered *r, std::vector<uint32_t> *off, size_t *bytes, hipStream_t st) {
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tables.find(tables);
    if (it == g_tables.end()) return SHTX_ERR_TABLES;
    *r = it->second;
  }
  const Tables &tb = r->view;
  if (tb.nitems == 0) return SHTX_ERR_UNSUPPORTED;
  std::vector<uint8_t> ckt((size_t)tb.nitems * tb.npairs);
  std::vector<int2> items(tb.nitems);
  hipError_t e = hipStreamSynchronize(st);
  if (e == hipSuccess) e = hipMemcpy(ckt.data(), tb.ck_t, ckt.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(items.data(), tb.ck_items, items.size() * sizeof(int2), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return SHTX_ERR_HIP;
  size_t ntiles = 0;
  *off = lam_tile_offsets(tb.nside, tb.lmax, tb.nitems, ckt.data(), items.data(), &ntiles);
  *bytes = lam_header_words(tb.nside, tb.nitems) * 4 + ntiles * kLamTileBytesHost;
  return SHTX_OK;
}
}  // namespace
}  // namespace shtx

extern "C" {

int shtx_lambda_table_bytes(const void *tables, size_t *bytes, void *stream) {
  if (!bytes) return SHTX_ERR_ARG;
  Registered r;
  std::vector<uint32_t> off;
  return lam_layout(tables, &r, &off, bytes, static_cast<hipStream_t>(stream));
}

int shtx_lambda_table_build(const void *tables, void *lam, size_t lam_bytes, void *stream) {
  if (!lam || (reinterpret_cast<uintptr_t>(lam) & 255)) return SHTX_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Registered r;
  std::vector<uint32_t> off;
  size_t need = 0;
  int s = lam_layout(tables, &r, &off, &need, st);
  if (s != SHTX_OK) return s;
  if (lam_bytes < need) return SHTX_ERR_WORKSPACE;
  // the offsets (host memory, synchronous copy), then the tiles by the kernel
  if (hipMemcpy(lam, off.data(), off.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return SHTX_ERR_HIP;
  if (launch_lambda_table_build(r.view, static_cast<uint32_t *>(lam), st) != hipSuccess) return SHTX_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  g_lams[lam] = LamRegistered{tables, need};
  return SHTX_OK;
}

int shtx_lambda_table_release(const void *lam) {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_lams.erase(lam) ? SHTX_OK : SHTX_ERR_TABLES;
}

int shtx_map2alm_stored(int nside, int lmax, int batch, int dtype, const void *map, void *alm, const void *tables,
                        const void *lam, void *work, size_t work_bytes, void *stream) {
  if (!lam) return SHTX_ERR_ARG;
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, map, alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  if (dtype != SHTX_BF16) return SHTX_ERR_UNSUPPORTED;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_lams.find(lam);
    if (it == g_lams.end() || it->second.tables != tables) return SHTX_ERR_TABLES;
  }
  return run_analysis<bf16_t, float>(tb, batch, static_cast<const bf16_t *>(map), static_cast<float2 *>(alm), tb.rp_w,
                                     1.0, 1.0, 1.0, work, static_cast<hipStream_t>(stream), 0, false, nullptr,
                                     static_cast<const uint32_t *>(lam));
}

size_t shtx_iter_workspace_bytes(int nside, int lmax, int batch, int dtype) {
  if (dtype != SHTX_F64 && dtype != SHTX_F32) return 0;
  const size_t base = shtx_workspace_bytes(nside, lmax, batch, dtype);
  if (base == 0) return 0;
  const size_t e = dtype == SHTX_F64 ? 8 : 4;
  return base + align_up((size_t)batch * 12 * (size_t)nside * (size_t)nside * e, 256);
}

}  // extern "C"

namespace shtx {
namespace {
// Refinement of Eq. (4)-(5) with the analysis A of the given quadrature
// weights: a = A f, then niter times a += A (f - S a) (the residual is formed
// in the synthesis' ring FFT store, the update in the analysis' accumulate
// mode).
template <typename T>
int run_iter(const Tables &tb, int batch, const T *f, cplx<T> *a, int niter, const double *wtab,
             const double *pixw, void *work, size_t resid_off, hipStream_t st) {
  T *r = reinterpret_cast<T *>(static_cast<char *>(work) + resid_off);
  int s = run_analysis<T, T>(tb, batch, f, a, wtab, 1.0, 1.0, 1.0, work, st, 0, false, pixw);
  for (int k = 0; k < niter && s == SHTX_OK; ++k) {
    s = run_synthesis<T, T>(tb, batch, a, r, 1.0, 1.0, 1.0, work, st, f);
    if (s == SHTX_OK) s = run_analysis<T, T>(tb, batch, r, a, wtab, 1.0, 1.0, 1.0, work, st, 1, false, pixw);
  }
  return s;
}
}  // namespace
}  // namespace shtx

extern "C" {

int shtx_map2alm_iter(int nside, int lmax, int batch, int dtype, const void *map, void *alm, int niter,
                      const void *tables, void *work, size_t work_bytes, void *stream) {
  return shtx_map2alm_iter_weighted(nside, lmax, batch, dtype, map, alm, niter, nullptr, nullptr, tables, work,
                                    work_bytes, stream);
}

int shtx_map2alm_iter_weighted(int nside, int lmax, int batch, int dtype, const void *map, void *alm, int niter,
                               const double *ring_weights, const double *pixel_weights, const void *tables,
                               void *work, size_t work_bytes, void *stream) {
  if (niter < 0 || niter > kMaxIter) return SHTX_ERR_ARG;
  if (dtype == SHTX_BF16) return SHTX_ERR_UNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(ring_weights) & 7) || (reinterpret_cast<uintptr_t>(pixel_weights) & 15))
    return SHTX_ERR_ARG;
  Tables tb;
  int s = check_common(nside, lmax, batch, dtype, map, alm, tables, work, work_bytes, &tb, true);
  if (s != SHTX_OK) return s;
  if (work_bytes < shtx_iter_workspace_bytes(nside, lmax, batch, dtype)) return SHTX_ERR_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t roff = shtx_workspace_bytes(nside, lmax, batch, dtype);
  // ring weights: the caller's, 1 under pixel weights alone, else the equal 4 pi / Npix
  const double *wtab = ring_weights ? ring_weights : pixel_weights ? nullptr : tb.rp_w;
  if (dtype == SHTX_F64)
    return run_iter<double>(tb, batch, static_cast<const double *>(map), static_cast<double2 *>(alm), niter, wtab,
                            pixel_weights, work, roff, st);
  return run_iter<float>(tb, batch, static_cast<const float *>(map), static_cast<float2 *>(alm), niter, wtab,
                         pixel_weights, work, roff, st);
}

}  // extern "C"
