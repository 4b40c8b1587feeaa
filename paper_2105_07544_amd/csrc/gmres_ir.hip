// Host orchestration and C ABI of the GMRES(m) / GMRES-IR hot path.
//
// One solver template drives both methods:
//   * plain GMRES(m) (Alg. 1 with CGS2, §III-A): inner = outer precision, the
//     implicit residual ends a cycle early, the explicit one confirms;
//   * GMRES-IR (Alg. 2, §III-B): float32 inner cycles of exactly m steps on a
//     float32 copy of A, float64 residual and solution update.
// Per inner iteration the stream receives: [poly steps] + SpMV (with the
// normalisation of v_j fused in), CGS2 dots, update+dots, update+norm with the
// float64 Givens step in its last block.  The host synchronises once per
// restart to read gamma = ||b - A x|| and the cycle status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gmres_ir.h"
#include "host_common.hpp"
#include "kernels.hpp"
#include "bjac.hpp"
#include "half_basis.hpp"

namespace gmr {

std::string& last_error() {
  static thread_local std::string msg;
  return msg;
}

#define GMR_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(GMR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

#define GMR_TRY(expr)               \
  do {                              \
    gmr_status s_ = (expr);         \
    if (s_ != GMR_OK) return s_;    \
  } while (0)

static constexpr inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
static inline size_t dsize(int dtype) { return dtype == GMR_F64 ? 8 : 4; }
static constexpr inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Grid of the SpMV-type kernels (one block per 256 rows).
static constexpr inline int spmv_grid(int n) { return ceil_div(n, kSpmvRows); }
// Grid of the CGS dot kernels: at most kMaxRedBlocks blocks (4 per CU); each
// writes one row of column partials.
static inline int dots_grid(int n) { return std::max(1, std::min(ceil_div(ceil_div(n, kWave), kWavesPerBlock), kMaxRedBlocks)); }
// Grid of the four-rows-per-lane dots pass (256-row groups).
static inline int dots4_grid(int n) { return dots_grid(ceil_div(n, 4)); }
// Grid of the streaming kernels.
static inline int stream_grid(int n) { return std::max(1, std::min(ceil_div(n, kBlock), kMaxRedBlocks)); }

// Blocks of kBlock threads of `fn` that the current device holds at once
// (occupancy per CU times the CU count), cached per device and kernel.
static int resident_blocks(const void* fn) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return kMaxRedBlocks;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, fn);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  int v = kMaxRedBlocks;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && per_cu > 0 &&
      cus > 0)
    v = per_cu * cus;
  cache[key] = v;
  return v;
}

// A grid-stride grid of at most `want` blocks cut to a whole number of
// resident rounds: with 144 VGPRs (three waves per SIMD, 768 blocks on 256
// CUs) a 1024-block grid would leave its last 256 blocks to run alone on a
// mostly idle chip.
static int balanced_grid(int want, const void* fn) {
  const int res = resident_blocks(fn);
  return want <= res ? want : (want / res) * res;
}

// Blocks of the cooperative cycle: one per 256 rows, at most kCoopMaxBlocks;
// 0 when the device cannot hold them all at once (or has no cooperative
// launch), and the multi-kernel cycle is used instead.  Measured at n = 4096
// (float32 inner iteration): 37.1 us with 128 rows per block, 29.1 with 256,
// 31.0 with 512.
constexpr int kCoopRows = 256;
template <class TI, class TO>
static int coop_grid(int n) {
  const int want = std::min(kCoopMaxBlocks, std::max(2, ceil_div(n, kCoopRows)));
  int dev = 0, coop = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop)
    return 0;
  return resident_blocks(reinterpret_cast<const void*>(coop_cycle_kernel<TI, TO>)) >= want ? want : 0;
}

// ---------------------------------------------------------------------------
// Workspace.  A fixed "small" region (reduction partials, the
// Hessenberg problem, status) followed by the n-sized vectors.
// ---------------------------------------------------------------------------
struct Small {
  size_t partial, H, Hraw, cs, sn, g, y, h1d, h2d, h1t, h2t, inv_beta, status, bar, end;
};

static constexpr Small small_layout(int n) {
  Small L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  const size_t npart = std::max<size_t>((size_t)kMaxCols * kPartPitch, (size_t)spmv_grid(n));
  L.partial = take(npart * 8);
  const size_t hsz = (size_t)(kMaxCols + 1) * kMaxCols * 8;
  L.H = take(hsz);
  L.Hraw = take(hsz);
  L.cs = take(kMaxCols * 8);
  L.sn = take(kMaxCols * 8);
  L.g = take((kMaxCols + 1) * 8);
  L.y = take(kMaxCols * 8);
  L.h1d = take(kMaxCols * 8);
  L.h2d = take(kMaxCols * 8);
  L.h1t = take(kMaxCols * 8);
  L.h2t = take(kMaxCols * 8);
  L.inv_beta = take(8 * 8);
  L.status = take(sizeof(Status));
  L.bar = take(sizeof(GridBarrier));
  L.end = o;
  return L;
}

struct Big {
  size_t V, W0, W1, R, U, P0, P1, Tt, Z, X32, Y32, end;
  int64_t ldv;
};

// m: restart; s: inner element size; so: outer element size.
static Big big_layout(size_t base, int n, int m, size_t s, size_t so, bool poly) {
  Big L;
  size_t o = base;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  L.ldv = (int64_t)align_up((size_t)n, 64);
  L.V = take((size_t)(m + 1) * L.ldv * s);
  L.W0 = take((size_t)n * s);
  L.W1 = take((size_t)n * s);
  L.R = take((size_t)n * so);
  L.U = take((size_t)n * s);
  L.P0 = L.P1 = L.Tt = L.Z = L.X32 = L.Y32 = 0;
  if (poly) {
    L.P0 = take((size_t)n * s);
    L.P1 = take((size_t)n * s);
    L.Tt = take((size_t)n * s);
    L.Z = take((size_t)n * s);
    if (s == 8) {
      // a float32 polynomial inside float64 GMRES: float32 copies of its input
      // and output (P0, P1 and Tt then hold its float32 work vectors)
      L.X32 = take((size_t)n * 4);
      L.Y32 = take((size_t)n * 4);
    }
  }
  L.end = o;
  return L;
}

struct Ws {
  char* base;
  Small S;
  double* partial() const { return (double*)(base + S.partial); }
  Status* status() const { return (Status*)(base + S.status); }
  GridBarrier* barrier() const { return (GridBarrier*)(base + S.bar); }
  CycleState cycle(int m) const {
    CycleState c;
    c.H = (double*)(base + S.H);
    c.Hraw = (double*)(base + S.Hraw);
    c.cs = (double*)(base + S.cs);
    c.sn = (double*)(base + S.sn);
    c.g = (double*)(base + S.g);
    c.y = (double*)(base + S.y);
    c.h1d = (double*)(base + S.h1d);
    c.h2d = (double*)(base + S.h2d);
    c.inv_beta = (double*)(base + S.inv_beta);
    c.st = status();
    c.ldh = m + 1;
    return c;
  }
  template <class T> T* h1t() const { return (T*)(base + S.h1t); }
  template <class T> T* h2t() const { return (T*)(base + S.h2t); }
  template <class T> T* at(size_t off) const { return (T*)(base + off); }
};

// ---------------------------------------------------------------------------
// Launch context: the stream plus the optional per-family event timing.
// ---------------------------------------------------------------------------
struct Prof {
  int family = GMR_PROF_NONE;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  double bytes = 0.0;
  int64_t launches = 0;
};

static Prof& prof_state() {
  static thread_local Prof p;
  return p;
}

struct Ctx {
  hipStream_t s;
  Prof* prof = nullptr;  // non-null while a solve is being profiled

  gmr_status begin(int family) {
    if (!prof || prof->family != family) return GMR_OK;
    if (prof->used + 2 > prof->pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        GMR_HIP(hipEventCreate(&e));
        prof->pool.push_back(e);
      }
    }
    GMR_HIP(hipEventRecord(prof->pool[prof->used], s));
    return GMR_OK;
  }
  gmr_status end(int family, double bytes) {
    if (!prof || prof->family != family) return GMR_OK;
    GMR_HIP(hipEventRecord(prof->pool[prof->used + 1], s));
    prof->used += 2;
    prof->bytes += bytes;
    prof->launches += 1;
    return GMR_OK;
  }
};

static gmr_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GMR_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GMR_OK;
}

// ---------------------------------------------------------------------------
// Argument checks
// ---------------------------------------------------------------------------
static gmr_status check_csr(const gmr_csr* A, const char* who) {
  if (!A) return fail(GMR_ERR_INVALID, std::string(who) + ": null matrix");
  if (A->n <= 0) return fail(GMR_ERR_INVALID, std::string(who) + ": n must be > 0");
  if (A->nnz < 0) return fail(GMR_ERR_INVALID, std::string(who) + ": nnz must be >= 0");
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(GMR_ERR_INVALID, std::string(who) + ": null CSR array");
  if (A->dtype != GMR_F32 && A->dtype != GMR_F64)
    return fail(GMR_ERR_INVALID, std::string(who) + ": unknown dtype");
  if (((uintptr_t)A->col_idx | (uintptr_t)A->val) % 16 != 0)
    return fail(GMR_ERR_INVALID, std::string(who) + ": col_idx and val must be 16-byte aligned");
  return GMR_OK;
}

// ---------------------------------------------------------------------------
// Launch helpers (each returns a status; all are asynchronous)
// ---------------------------------------------------------------------------
template <class T>
static double spmv_bytes(const gmr_csr* A) {
  return (double)A->nnz * (4 + sizeof(T)) + (double)(A->n + 1) * 4 + 2.0 * A->n * sizeof(T);
}

template <class T>
static gmr_status launch_spmv(Ctx& c, const gmr_csr* A, const T* x, const double* scale, T* vout,
                              T* y, const int* done) {
  GMR_TRY(c.begin(GMR_PROF_SPMV));
  spmv_kernel<T><<<spmv_grid(A->n), kBlock, 0, c.s>>>(A->n, A->row_ptr, A->col_idx,
                                                      (const T*)A->val, x, scale, vout, y, done);
  GMR_TRY(check_launch("spmv_kernel"));
  return c.end(GMR_PROF_SPMV, spmv_bytes<T>(A) + (vout ? (double)A->n * sizeof(T) : 0.0));
}

template <class T>
static gmr_status launch_dots(Ctx& c, int n, int j, const T* V, int64_t ldv, const T* w,
                              const Ws& ws, double* hd, T* ht, const int* done, int rev) {
  GMR_TRY(c.begin(GMR_PROF_CGS_DOTS));
  double* part = ws.partial();
  // four rows per lane in float32 when the basis is vector-aligned (measured on
  // config 2: 5.23 -> 5.34 TB/s); float64 keeps one row per lane (its 32-byte
  // variant ran at 4.8 TB/s against 5.5)
  const bool rows4 = sizeof(T) == 4 && ldv % 4 == 0 &&
                     ((reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(w)) % (4 * sizeof(T))) == 0;
  if (!rows4) {
    const int G = dots_grid(n);
    if (j <= 8)
      cgs_dots_kernel<T, 8, 1><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev);
    else if (j <= 16)
      cgs_dots_kernel<T, 16, 1><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev);
    else if (j <= 32)
      cgs_dots_kernel<T, 32, 1><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev);
    else if (j <= 64)
      cgs_dots_kernel<T, 64, 1><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev);
    else if (j <= 256)
      cgs_dots_kernel<T, 64, 4><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev);
    else
      cgs_dots_kernel<T, 64, 8><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev);
    GMR_TRY(check_launch("cgs_dots_kernel"));
    GMR_TRY(c.end(GMR_PROF_CGS_DOTS, (double)(j + 1) * n * sizeof(T)));
    finish_cols_kernel<T><<<j, kBlock, 0, c.s>>>(G, part, hd, ht, done);
    return check_launch("finish_cols_kernel");
  }
  // Beyond 32 columns the basis is read in 32-column chunks: a 64-column chunk
  // of four rows per lane keeps 256 VGPRs live and runs one wave per SIMD.
  int G = dots4_grid(n);
#define GMR_D4(K, NQ)                                                                   \
  do {                                                                                  \
    G = balanced_grid(G, reinterpret_cast<const void*>(cgs_dots4_kernel<T, K, NQ>));     \
    cgs_dots4_kernel<T, K, NQ><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, part, done, rev); \
  } while (0)
  if (j <= 8) GMR_D4(8, 1);
  else if (j <= 16) GMR_D4(16, 1);
  else if (j <= 32) GMR_D4(32, 1);
  else if (j <= 64) GMR_D4(32, 2);
  else if (j <= 128) GMR_D4(32, 4);
  else if (j <= 256) GMR_D4(32, 8);
  else GMR_D4(32, 16);
#undef GMR_D4
  GMR_TRY(check_launch("cgs_dots_kernel"));
  GMR_TRY(c.end(GMR_PROF_CGS_DOTS, (double)(j + 1) * n * sizeof(T)));
  finish_cols_kernel<T><<<j, kBlock, 0, c.s>>>(G, part, hd, ht, done);
  return check_launch("finish_cols_kernel");
}

// Largest j for which the update and the second dots fuse (basis row in
// registers).  float32: 128 columns in 151 VGPRs (three waves per SIMD, with
// the coefficients in scalar registers).  float64: beyond 64 columns the
// fused kernel would run one wave per SIMD, and the separate update and dots
// passes are faster although they read V twice.
template <class T> constexpr int fused_max() { return sizeof(T) == 4 ? 128 : 64; }

template <class T>
static gmr_status launch_update_dots(Ctx& c, int n, int j, const T* V, int64_t ldv, const T* hin,
                                     T* w, const Ws& ws, double* hd, T* ht, const int* done, int rev) {
  if (j > fused_max<T>()) {
    // no room to keep the row in registers: update, then a separate dots pass
    GMR_TRY(c.begin(GMR_PROF_CGS_UPDATE_DOTS));
    cgs_update_kernel<T><<<stream_grid(n), kBlock, 0, c.s>>>(n, j, V, ldv, hin, w, done, rev);
    GMR_TRY(check_launch("cgs_update_kernel"));
    GMR_TRY(c.end(GMR_PROF_CGS_UPDATE_DOTS, (double)(j + 2) * n * sizeof(T)));
    return launch_dots<T>(c, n, j, V, ldv, w, ws, hd, ht, done, !rev);
  }
  GMR_TRY(c.begin(GMR_PROF_CGS_UPDATE_DOTS));
  int G = dots_grid(n);
  double* part = ws.partial();
#define GMR_UD(K)                                                                        \
  do {                                                                                   \
    G = balanced_grid(G, reinterpret_cast<const void*>(cgs_update_dots_kernel<T, K>));   \
    cgs_update_dots_kernel<T, K><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, hin, w, part, done, rev); \
  } while (0)
  if (j <= 8) GMR_UD(8);
  else if (j <= 16) GMR_UD(16);
  else if (j <= 32) GMR_UD(32);
  else if (j <= 64) GMR_UD(64);
  else if constexpr (sizeof(T) == 4) GMR_UD(128);
#undef GMR_UD
  GMR_TRY(check_launch("cgs_update_dots_kernel"));
  GMR_TRY(c.end(GMR_PROF_CGS_UPDATE_DOTS, (double)(j + 2) * n * sizeof(T)));
  finish_cols_kernel<T><<<j, kBlock, 0, c.s>>>(G, part, hd, ht, done);
  return check_launch("finish_cols_kernel");
}

template <class T, int MODE>
static gmr_status launch_update_norm(Ctx& c, int n, int j, const T* V, int64_t ldv, const T* hin,
                                     T* w, const Ws& ws, CycleState cs, int last_jc,
                                     double* hout, const int* done, int rev) {
  GMR_TRY(c.begin(GMR_PROF_CGS_UPDATE_NORM));
  const double thresh = sizeof(T) == 4 ? 1e3 * 1.1754943508222875e-38 : 0.0;
  const int G = stream_grid(n);
  cgs_update_norm_kernel<T><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, hin, w, ws.partial(), done, rev);
  GMR_TRY(check_launch("cgs_update_norm_kernel"));
  GMR_TRY(c.end(GMR_PROF_CGS_UPDATE_NORM, (double)(j + 2) * n * sizeof(T)));
  finish_norm_kernel<T, MODE><<<1, kBlock, 0, c.s>>>(G, ws.partial(), cs, j, last_jc, thresh, hout, done);
  return check_launch("finish_norm_kernel");
}

// Direction of the first pass over V at basis size j.  Each pass runs
// opposite to the one before it, so that it starts on the rows the
// memory-side cache still holds.  With the fused update+dots an iteration
// makes three passes (odd), so the first direction flips with j; with the
// separate update and dots it makes four, and the direction stays fixed.
static inline int first_pass_rev(int j, int fused) { return j > fused ? 1 : (j & 1); }

// The three CGS2 passes on w against V[:, 0:j].
template <class T, int MODE>
static gmr_status cgs2_passes(Ctx& c, int n, int j, const T* V, int64_t ldv, T* w, const Ws& ws,
                              CycleState cs, int last_jc, double* hout, const int* done) {
  const int rev = first_pass_rev(j, fused_max<T>());
  const int last = j > fused_max<T>() ? !rev : rev;
  GMR_TRY(launch_dots<T>(c, n, j, V, ldv, w, ws, cs.h1d, ws.h1t<T>(), done, rev));
  GMR_TRY(launch_update_dots<T>(c, n, j, V, ldv, ws.h1t<T>(), w, ws, cs.h2d, ws.h2t<T>(), done, !rev));
  return launch_update_norm<T, MODE>(c, n, j, V, ldv, ws.h2t<T>(), w, ws, cs, last_jc, hout, done, last);
}

// The three CGS2 passes with the basis stored in float16 (scaled by sigma).
static gmr_status hb_cgs2_passes(Ctx& c, int n, int j, const half_t* V, int64_t ldv, float* w, const Ws& ws,
                                 CycleState cs, int last_jc, float inv_sigma, const int* done) {
  double* part = ws.partial();
  const double vb = (double)j * n * sizeof(half_t);
  const int rev = first_pass_rev(j, 64);   // same rule; the fused kernel here takes up to 64 columns
  // pass 1: h1 = V^T w
  GMR_TRY(c.begin(GMR_PROF_CGS_DOTS));
  const int G = dots_grid(ceil_div(n, 2));
#define GMR_HD(K, NQ, R) hb_dots_kernel<K, NQ><<<G, kBlock, 0, c.s>>>(n, j, V, ldv, w, inv_sigma, part, done, R)
  if (j <= 8) GMR_HD(8, 1, rev);
  else if (j <= 16) GMR_HD(16, 1, rev);
  else if (j <= 32) GMR_HD(32, 1, rev);
  else if (j <= 64) GMR_HD(64, 1, rev);
  else if (j <= 256) GMR_HD(64, 4, rev);
  else GMR_HD(64, 8, rev);
  GMR_TRY(check_launch("hb_dots_kernel"));
  GMR_TRY(c.end(GMR_PROF_CGS_DOTS, vb + 4.0 * n));
  finish_cols_kernel<float><<<j, kBlock, 0, c.s>>>(G, part, cs.h1d, ws.h1t<float>(), done);
  GMR_TRY(check_launch("finish_cols_kernel"));
  // pass-1 update and pass-2 dots
  GMR_TRY(c.begin(GMR_PROF_CGS_UPDATE_DOTS));
  int GU = G;   // the grid whose partials the second finish_cols reads
  if (j > 64) {
    hb_update_kernel<false><<<stream_grid(n), kBlock, 0, c.s>>>(n, j, V, ldv, ws.h1t<float>(), inv_sigma, w,
                                                               part, done, !rev);
    GMR_TRY(check_launch("hb_update_kernel"));
    GMR_TRY(c.end(GMR_PROF_CGS_UPDATE_DOTS, vb + 8.0 * n));
    if (j <= 256) GMR_HD(64, 4, rev);
    else GMR_HD(64, 8, rev);
    GMR_TRY(check_launch("hb_dots_kernel"));
  } else {
#define GMR_HUD(K)                                                                                         \
  do {                                                                                                     \
    GU = balanced_grid(G, reinterpret_cast<const void*>(hb_update_dots_kernel<K>));                          \
    hb_update_dots_kernel<K><<<GU, kBlock, 0, c.s>>>(n, j, V, ldv, ws.h1t<float>(), inv_sigma, w, part, done, \
                                                     !rev);                                                  \
  } while (0)
    if (j <= 8) GMR_HUD(8);
    else if (j <= 16) GMR_HUD(16);
    else if (j <= 32) GMR_HUD(32);
    else GMR_HUD(64);
#undef GMR_HUD
    GMR_TRY(check_launch("hb_update_dots_kernel"));
    GMR_TRY(c.end(GMR_PROF_CGS_UPDATE_DOTS, vb + 8.0 * n));
  }
#undef GMR_HD
  finish_cols_kernel<float><<<j, kBlock, 0, c.s>>>(GU, part, cs.h2d, ws.h2t<float>(), done);
  GMR_TRY(check_launch("finish_cols_kernel"));
  // pass-2 update, norm, Givens
  GMR_TRY(c.begin(GMR_PROF_CGS_UPDATE_NORM));
  const int GS = stream_grid(n);
  hb_update_kernel<true><<<GS, kBlock, 0, c.s>>>(n, j, V, ldv, ws.h2t<float>(), inv_sigma, w, part, done,
                                                 j > 64 ? !rev : rev);
  GMR_TRY(check_launch("hb_update_kernel"));
  GMR_TRY(c.end(GMR_PROF_CGS_UPDATE_NORM, vb + 8.0 * n));
  finish_norm_kernel<float, kTailGivens><<<1, kBlock, 0, c.s>>>(GS, part, cs, j, last_jc, 1e3 * 1.1754943508222875e-38,
                                                               nullptr, done);
  return check_launch("finish_norm_kernel");
}

// sigma = 2^round(log2 sqrt(n)), at most 2^15: the scale of the float16 basis.
static float hb_sigma(int n) {
  const int e = std::min(15, std::max(0, (int)std::lround(0.5 * std::log2((double)n))));
  return std::ldexp(1.0f, e);
}

}  // namespace gmr

// ---------------------------------------------------------------------------
// Polynomial object (host-side roots)
// ---------------------------------------------------------------------------
// Handle of a right preconditioner: a GMRES polynomial or block Jacobi.
struct gmr_poly {
  int32_t dtype;
  int32_t kind = 0;            // 0: GMRES polynomial, 1: block Jacobi
  std::vector<double> re, im;  // Leja-ordered roots, rounded to dtype's precision
  std::vector<double> hess;    // Hessenberg matrix of the Arnoldi run, column-major
  int32_t ldh = 0;             // its leading dimension (degree + 2)
  int32_t n = 0;               // block Jacobi: order of A
  int32_t block = 0;           // block Jacobi: rows per diagonal block
  const void* inv = nullptr;   // block Jacobi: inverted blocks (caller's device memory)
};

namespace gmr {

constexpr int kPrecBjac = 1;

static size_t bjac_blocks_offset() { return 256; }  // the singular-block flag comes first

static int bjac_grid(int n, int k) {
  const int nblk = ceil_div(n, k);
  if (k >= kBjacStagedMin) return nblk;  // one block per one-wave workgroup
  return ceil_div(ceil_div(nblk, kWave / k), kBlock / kWave);
}

// Columns per LDS chunk of the staged apply: about 8 KB of the slot, even.
template <class T>
static int bjac_chunk(int k) {
  const int c = (int)(8192 / ((size_t)k * sizeof(T))) & ~1;
  return std::max(2, std::min(c, k + (k & 1)));
}

template <class T>
static size_t bjac_staged_lds(int k) {
  return ((size_t)bjac_chunk<T>(k) * k + kWave) * sizeof(T);
}

template <class T>
static gmr_status poly_apply_impl(Ctx& c, const gmr_poly* P, const gmr_csr* A, const T* x, T* y,
                                  T* P0, T* P1, T* Tt, const int* done) {
  const int n = A->n;
  if (P->kind == kPrecBjac) {
    const int kb = P->block;
    GMR_TRY(c.begin(GMR_PROF_BJAC));
    if (kb >= kBjacStagedMin)
      bjac_apply_staged_kernel<T><<<bjac_grid(n, kb), kWave, bjac_staged_lds<T>(kb), c.s>>>(
          n, kb, bjac_chunk<T>(kb), (const T*)P->inv, x, y, done);
    else
      bjac_apply_kernel<T><<<bjac_grid(n, kb), kBlock, 0, c.s>>>(n, kb, (const T*)P->inv, x, y, done);
    GMR_TRY(check_launch("bjac_apply_kernel"));
    return c.end(GMR_PROF_BJAC, ((double)ceil_div(n, kb) * kb * kb + 2.0 * n) * sizeof(T));
  }
  const int k = (int)P->re.size();
  const int G = spmv_grid(n);
  const int GS = stream_grid(n);
  const int* rp = A->row_ptr;
  const int* ci = A->col_idx;
  const T* val = (const T*)A->val;
  const T* cur = x;
  T* bufs[2] = {P0, P1};
  int nb = 0;
  bool first = true;
  // Algorithmic bytes of a step: the matrix and the gathered input (whose own
  // rows, read again by the epilogue, count once), plus the epilogue's other
  // vectors.  A real step and pair step 1 write y and the next vector (the next
  // P, or Tt) and read y after the first step; pair step 2 reads P and writes
  // the next P (Tt is its gathered input).
  const double vec = (double)n * sizeof(T);
  const double mat_x = spmv_bytes<T>(A) - vec;
  auto step_bytes = [&](bool f) { return mat_x + (f ? 2.0 : 3.0) * vec; };
  int i = 0;
  while (i < k) {
    if (P->im[i] == 0.0) {
      const T cr = T(1.0 / P->re[i]);
      if (i < k - 1) {
        T* nxt = bufs[nb];
        nb ^= 1;
        GMR_TRY(c.begin(GMR_PROF_POLY_STEP));
        if (first)
          poly_real_kernel<T, true><<<G, kBlock, 0, c.s>>>(n, rp, ci, val, cur, cr, y, nxt, done);
        else
          poly_real_kernel<T, false><<<G, kBlock, 0, c.s>>>(n, rp, ci, val, cur, cr, y, nxt, done);
        GMR_TRY(check_launch("poly_real_kernel"));
        GMR_TRY(c.end(GMR_PROF_POLY_STEP, step_bytes(first)));
        cur = nxt;
      } else {
        if (first)
          poly_real_last_kernel<T, true><<<GS, kBlock, 0, c.s>>>(n, cur, cr, y, done);
        else
          poly_real_last_kernel<T, false><<<GS, kBlock, 0, c.s>>>(n, cur, cr, y, done);
        GMR_TRY(check_launch("poly_real_last_kernel"));
      }
      i += 1;
    } else {
      const double a = P->re[i], b = P->im[i];
      const double mod2 = a * a + b * b;
      const T c1 = T(2.0 * a / mod2), c2 = T(1.0 / mod2);
      GMR_TRY(c.begin(GMR_PROF_POLY_STEP));
      if (first)
        poly_pair1_kernel<T, true><<<G, kBlock, 0, c.s>>>(n, rp, ci, val, cur, c1, c2, y, Tt, done);
      else
        poly_pair1_kernel<T, false><<<G, kBlock, 0, c.s>>>(n, rp, ci, val, cur, c1, c2, y, Tt, done);
      GMR_TRY(check_launch("poly_pair1_kernel"));
      GMR_TRY(c.end(GMR_PROF_POLY_STEP, step_bytes(first)));
      if (i < k - 2) {
        T* nxt = bufs[nb];
        nb ^= 1;
        GMR_TRY(c.begin(GMR_PROF_POLY_STEP));
        poly_pair2_kernel<T><<<G, kBlock, 0, c.s>>>(n, rp, ci, val, cur, Tt, c1, c2, nxt, done);
        GMR_TRY(check_launch("poly_pair2_kernel"));
        GMR_TRY(c.end(GMR_PROF_POLY_STEP, mat_x + 2.0 * vec));
        cur = nxt;
      }
      i += 2;
    }
    first = false;
  }
  return GMR_OK;
}

// Small kernel that seeds the Arnoldi state for the polynomial setup.
__global__ void arnoldi_init_kernel(CycleState cs, const double* nrm) {
  const double b0 = *nrm;
  cs.g[0] = b0;
  *cs.inv_beta = 1.0 / b0;
  Status* st = cs.st;
  st->beta0 = b0;
  st->k = 0;
  st->done = 0;
  st->breakdown = 0;
  st->nonfinite = !(b0 > 0.0) || !isfinite(b0);
  st->stop_thresh = -1.0;
  st->gamma = 1.0;
}

// ---------------------------------------------------------------------------
// The solver
// ---------------------------------------------------------------------------
struct SolveArgs {
  const gmr_csr* Ain;    // inner matrix (TI values)
  const gmr_csr* Aout;   // outer matrix (TO values)
  const gmr_poly* P;     // nullable, TI precision
  const void* b;
  void* x;
  const gmr_params* prm;
  void* ws;
  size_t ws_bytes;
  gmr_result* res;
  double* hist;
  hipStream_t stream;
  const gmr_csr* Aprec = nullptr;  // matrix of the polynomial's products (null: Ain)
};

static gmr_status check_params(const gmr_params* p) {
  if (!p) return fail(GMR_ERR_INVALID, "null params");
  if (p->restart < 1) return fail(GMR_ERR_INVALID, "restart must be >= 1");
  if (p->restart > kMaxCols) return fail(GMR_ERR_UNSUPPORTED, "restart > 512 is not supported");
  if (!(p->tol > 0.0)) return fail(GMR_ERR_INVALID, "tol must be > 0");
  if (p->max_iters <= 0) return fail(GMR_ERR_INVALID, "max_iters must be > 0");
  if (p->max_cycles < 0 || p->stagnation_cycles < 0) return fail(GMR_ERR_INVALID, "negative cycle cap");
  return GMR_OK;
}

// One restart cycle captured as a hipGraph and replayed every restart.  The
// kernels' arguments (pointers, column counts) are the same in every cycle;
// a shorter final cycle (max_iters) is captured again.
struct CycleGraph {
  bool use = false;
  hipGraphExec_t exec = nullptr;
  int mc = -1;
  template <class F>
  gmr_status capture(hipStream_t s, F&& body) {
    if (exec) {
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    GMR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const gmr_status st = body();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st != GMR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(GMR_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(GMR_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    return GMR_OK;
  }
  ~CycleGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// out = (To) in, skipped once the cycle has ended (done set).
template <class From, class To>
__global__ __launch_bounds__(kBlock) void cast_vec_kernel(int n, const From* __restrict__ in, To* __restrict__ out,
                                                          const int* __restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) out[i] = To(in[i]);
}

gmr_status library_stream(hipStream_t* out) {
  static thread_local hipStream_t streams[64] = {};
  int dev = 0;
  GMR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(GMR_ERR_UNSUPPORTED, "device index >= 64");
  if (!streams[dev]) GMR_HIP(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  *out = streams[dev];
  return GMR_OK;
}

// Makes the occupancy queries behind balanced_grid for every kernel that uses
// it, so that none of them first happens while a cycle is being captured.
template <class T>
static void warm_grid_cache() {
  const void* fns[] = {
      reinterpret_cast<const void*>(cgs_update_dots_kernel<T, 8>),
      reinterpret_cast<const void*>(cgs_update_dots_kernel<T, 16>),
      reinterpret_cast<const void*>(cgs_update_dots_kernel<T, 32>),
      reinterpret_cast<const void*>(cgs_update_dots_kernel<T, 64>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 8, 1>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 16, 1>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 32, 1>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 32, 2>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 32, 4>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 32, 8>),
      reinterpret_cast<const void*>(cgs_dots4_kernel<T, 32, 16>)};
  for (const void* f : fns) (void)resident_blocks(f);
  if constexpr (sizeof(T) == 4) {
    (void)resident_blocks(reinterpret_cast<const void*>(cgs_update_dots_kernel<T, 128>));
    (void)resident_blocks(reinterpret_cast<const void*>(hb_update_dots_kernel<8>));
    (void)resident_blocks(reinterpret_cast<const void*>(hb_update_dots_kernel<16>));
    (void)resident_blocks(reinterpret_cast<const void*>(hb_update_dots_kernel<32>));
    (void)resident_blocks(reinterpret_cast<const void*>(hb_update_dots_kernel<64>));
  }
}

template <class TI, class TO>
static gmr_status solve_impl(const SolveArgs& a) {
  const auto t_start = std::chrono::steady_clock::now();
  const gmr_params& prm = *a.prm;
  const int n = a.Aout->n;
  const int m = prm.restart;
  const bool implicit_stop = sizeof(TI) == sizeof(TO);  // plain GMRES
  const bool poly = a.P != nullptr;
  // §III-D option (a): a float32 polynomial applied inside float64 GMRES, to
  // float32 copies of its input, the result widened back to float64
  const bool mixed = poly && a.P->dtype == GMR_F32 && sizeof(TI) == 8;
  const gmr_csr* Ap = a.Aprec ? a.Aprec : a.Ain;
  const bool half = (prm.flags & GMR_FLAG_HALF_BASIS) != 0;
  if (half && (sizeof(TI) != 4 || sizeof(TO) != 8))
    return fail(GMR_ERR_UNSUPPORTED, "GMR_FLAG_HALF_BASIS is a GMRES-IR option");
  if (poly && a.P->kind == kPrecBjac && a.P->n != n)
    return fail(GMR_ERR_INVALID, "block Jacobi preconditioner built for another order n");
  Ws ws{(char*)a.ws, small_layout(n)};
  const Big B = big_layout(ws.S.end, n, m, sizeof(TI), sizeof(TO), poly);
  if (!a.ws || a.ws_bytes < B.end)
    return fail(GMR_ERR_WORKSPACE, "workspace too small: need " + std::to_string(B.end) + " bytes");

  Ctx c{a.stream, nullptr};
  CycleGraph graph;
  graph.use = (prm.flags & GMR_FLAG_GRAPH) && prm.prof_kernel == GMR_PROF_NONE;
  warm_grid_cache<TI>();
  if (graph.use) {
    // capture needs a stream other than the legacy default one: the solve runs
    // on the library's own stream once the caller's stream has drained
    GMR_HIP(hipStreamSynchronize(a.stream));
    GMR_TRY(library_stream(&c.s));
  }
  // one block per cycle for a small system without a polynomial (profiling
  // and graph replay keep the multi-kernel cycle)
  const bool persistent = (prm.flags & GMR_FLAG_PERSISTENT) && n <= kCoopMaxN && !poly && !graph.use &&
                          !half && prm.prof_kernel == GMR_PROF_NONE;
  // above one block's size, the cooperative multi-block cycle (when the device
  // holds its grid)
  const int coop_blocks = (persistent && n > kSmallMaxN) ? coop_grid<TI, TO>(n) : 0;
  const double brk_thresh = sizeof(TI) == 4 ? 1e3 * 1.1754943508222875e-38 : 0.0;
  const float sigma = hb_sigma(n);
  Prof& pf = prof_state();
  pf.family = prm.prof_kernel;
  pf.used = 0;
  pf.bytes = 0.0;
  pf.launches = 0;
  if (prm.prof_kernel != GMR_PROF_NONE) c.prof = &pf;

  TI* V = ws.at<TI>(B.V);
  TI* W[2] = {ws.at<TI>(B.W0), ws.at<TI>(B.W1)};
  TO* r = ws.at<TO>(B.R);
  TI* U = ws.at<TI>(B.U);
  const TO* b = (const TO*)a.b;
  TO* x = (TO*)a.x;
  CycleState cs = ws.cycle(m);
  Status* st_dev = ws.status();
  const int* done = &st_dev->done;

  norm2_kernel<TO><<<stream_grid(n), kBlock, 0, c.s>>>(n, b, ws.partial());
  GMR_TRY(check_launch("norm2_kernel"));
  finish_norm2_kernel<<<1, kBlock, 0, c.s>>>(stream_grid(n), ws.partial(), &st_dev->bnorm);
  GMR_TRY(check_launch("finish_norm2_kernel"));
  auto residual = [&]() -> gmr_status {
    GMR_TRY(c.begin(GMR_PROF_RESIDUAL));
    residual_kernel<TO><<<spmv_grid(n), kBlock, 0, c.s>>>(n, a.Aout->row_ptr, a.Aout->col_idx,
                                                         (const TO*)a.Aout->val, x, b, r,
                                                         ws.partial());
    GMR_TRY(check_launch("residual_kernel"));
    // the product (matrix, gathered x, r written) and b read
    GMR_TRY(c.end(GMR_PROF_RESIDUAL, spmv_bytes<TO>(a.Aout) + (double)n * sizeof(TO)));
    finish_residual_kernel<<<1, kBlock, 0, c.s>>>(spmv_grid(n), ws.partial(), st_dev);
    return check_launch("finish_residual_kernel");
  };
  GMR_TRY(residual());
  Status st;
  GMR_HIP(hipMemcpyAsync(&st, st_dev, sizeof(Status), hipMemcpyDeviceToHost, c.s));
  GMR_HIP(hipStreamSynchronize(c.s));

  gmr_result R{};
  R.status = GMR_NOT_CONVERGED;
  const double bnorm = st.bnorm;
  if (!std::isfinite(bnorm) || !std::isfinite(st.gamma)) return fail(GMR_ERR_NONFINITE, "non-finite b or x0");
  const int hist_cap = prm.max_cycles > 0 ? prm.max_cycles + 1 : 4096;
  auto push_hist = [&](double v) {
    if (a.hist && R.history_len < hist_cap) a.hist[R.history_len] = v;
    if (R.history_len < hist_cap) R.history_len++;
  };
  if (bnorm == 0.0) {
    // b = 0: the solution is x = 0
    GMR_HIP(hipMemsetAsync(x, 0, (size_t)n * sizeof(TO), c.s));
    GMR_HIP(hipStreamSynchronize(c.s));
    R.status = GMR_OK;
    R.rel_res = 0.0;
    push_hist(0.0);
    *a.res = R;
    return GMR_OK;
  }
  double gamma = st.gamma;
  push_hist(gamma / bnorm);
  // z = p(A) v in the polynomial's precision
  auto apply_prec = [&](const TI* in, TI* out, const int* dn) -> gmr_status {
    if (!mixed)
      return poly_apply_impl<TI>(c, a.P, Ap, in, out, ws.at<TI>(B.P0), ws.at<TI>(B.P1), ws.at<TI>(B.Tt), dn);
    float* x32 = ws.at<float>(B.X32);
    float* y32 = ws.at<float>(B.Y32);
    cast_vec_kernel<TI, float><<<stream_grid(n), kBlock, 0, c.s>>>(n, in, x32, dn);
    GMR_TRY(check_launch("cast_vec_kernel"));
    GMR_TRY(poly_apply_impl<float>(c, a.P, Ap, x32, y32, ws.at<float>(B.P0), ws.at<float>(B.P1),
                                   ws.at<float>(B.Tt), dn));
    cast_vec_kernel<float, TI><<<stream_grid(n), kBlock, 0, c.s>>>(n, y32, out, dn);
    return check_launch("cast_vec_kernel");
  };
  // Everything one restart cycle enqueues: the cast of r, mc inner iterations,
  // the solution update and the next residual (with its norm).
  auto enqueue_cycle = [&](int mc) -> gmr_status {
    start_cycle_kernel<TO, TI><<<stream_grid(n), kBlock, 0, c.s>>>(n, r, W[0], ws.partial(), st_dev);
    GMR_TRY(check_launch("start_cycle_kernel"));
    finish_start_cycle_kernel<TI><<<1, kBlock, 0, c.s>>>(stream_grid(n), ws.partial(), cs,
                                                         implicit_stop ? prm.tol * bnorm : -1.0);
    GMR_TRY(check_launch("finish_start_cycle_kernel"));
    int cur = 0;
    for (int j = 0; j < mc; ++j) {
      TI* vj = V + (size_t)j * B.ldv;
      TI* wn = W[cur ^ 1];
      if (poly && half) {
        if constexpr (sizeof(TI) == 4 && sizeof(TO) == 8) {
          // v_j in float32 (in U, free until the end of the cycle) for the
          // preconditioner, float16 into the basis
          half_t* Vh = reinterpret_cast<half_t*>(V);
          TI* Z = ws.at<TI>(B.Z);
          hb_scale_kernel<<<stream_grid(n), kBlock, 0, c.s>>>(n, W[cur], cs.inv_beta, sigma,
                                                             Vh + (size_t)j * B.ldv, U, done);
          GMR_TRY(check_launch("hb_scale_kernel"));
          GMR_TRY(apply_prec(U, Z, done));
          GMR_TRY(launch_spmv<TI>(c, a.Ain, Z, nullptr, nullptr, wn, done));
          GMR_TRY(hb_cgs2_passes(c, n, j + 1, Vh, B.ldv, wn, ws, cs, mc - 1, 1.0f / sigma, done));
        }
        cur ^= 1;
        continue;
      } else if (poly) {
        TI* Z = ws.at<TI>(B.Z);
        scale_kernel<TI><<<stream_grid(n), kBlock, 0, c.s>>>(n, W[cur], cs.inv_beta, vj, done);
        GMR_TRY(check_launch("scale_kernel"));
        GMR_TRY(apply_prec(vj, Z, done));
        GMR_TRY(launch_spmv<TI>(c, a.Ain, Z, nullptr, nullptr, wn, done));
      } else if (half) {
        if constexpr (sizeof(TI) == 4 && sizeof(TO) == 8) {
          half_t* Vh = reinterpret_cast<half_t*>(V);
          GMR_TRY(c.begin(GMR_PROF_SPMV));
          spmv_hb_kernel<<<spmv_grid(n), kBlock, 0, c.s>>>(n, a.Ain->row_ptr, a.Ain->col_idx,
                                                          (const float*)a.Ain->val, W[cur], cs.inv_beta, sigma,
                                                          Vh + (size_t)j * B.ldv, wn, done);
          GMR_TRY(check_launch("spmv_hb_kernel"));
          GMR_TRY(c.end(GMR_PROF_SPMV, spmv_bytes<float>(a.Ain) + 2.0 * n));
          GMR_TRY(hb_cgs2_passes(c, n, j + 1, Vh, B.ldv, wn, ws, cs, mc - 1, 1.0f / sigma, done));
        }
        cur ^= 1;
        continue;
      } else {
        GMR_TRY(launch_spmv<TI>(c, a.Ain, W[cur], cs.inv_beta, vj, wn, done));
      }
      GMR_TRY((cgs2_passes<TI, kTailGivens>(c, n, j + 1, V, B.ldv, wn, ws, cs, mc - 1, nullptr, done)));
      cur ^= 1;
    }
    if (poly) {
      TI* Z = ws.at<TI>(B.Z);
      if (half) {
        if constexpr (sizeof(TI) == 4 && sizeof(TO) == 8) {
          hb_solution_update_kernel<<<stream_grid(n), kBlock, 0, c.s>>>(
              n, reinterpret_cast<const half_t*>(V), B.ldv, cs.y, 1.0f / sigma, st_dev, U, nullptr);
          GMR_TRY(check_launch("hb_solution_update_kernel"));
        }
      } else {
        solution_update_kernel<TI, TO><<<stream_grid(n), kBlock, 0, c.s>>>(n, V, B.ldv, cs.y, st_dev, U, nullptr);
        GMR_TRY(check_launch("solution_update_kernel"));
      }
      GMR_TRY(apply_prec(U, Z, nullptr));
      axpy_gamma_kernel<TI, TO><<<stream_grid(n), kBlock, 0, c.s>>>(n, Z, st_dev, x);
      GMR_TRY(check_launch("axpy_gamma_kernel"));
    } else if (half) {
      if constexpr (sizeof(TI) == 4 && sizeof(TO) == 8) {
        hb_solution_update_kernel<<<stream_grid(n), kBlock, 0, c.s>>>(n, reinterpret_cast<const half_t*>(V), B.ldv,
                                                                     cs.y, 1.0f / sigma, st_dev, nullptr, x);
        GMR_TRY(check_launch("hb_solution_update_kernel"));
      }
    } else {
      solution_update_kernel<TI, TO><<<stream_grid(n), kBlock, 0, c.s>>>(n, V, B.ldv, cs.y, st_dev, nullptr, x);
      GMR_TRY(check_launch("solution_update_kernel"));
    }
    if (graph.use) return residual();
    return GMR_OK;
  };
  int64_t it = 0;
  double best = gamma;
  int since_best = 0;
  gmr_status final_status = GMR_NOT_CONVERGED;
  while (true) {
    const double rel = gamma / bnorm;
    if (!std::isfinite(rel)) { final_status = GMR_ERR_NONFINITE; fail(GMR_ERR_NONFINITE, "non-finite residual"); break; }
    if (rel <= prm.tol) { final_status = GMR_OK; break; }
    if (it >= prm.max_iters || (prm.max_cycles > 0 && R.cycles >= prm.max_cycles)) break;
    if (prm.stagnation_cycles > 0 && R.cycles > 0) {
      if (gamma < 0.99 * best) { best = gamma; since_best = 0; }
      else if (++since_best >= prm.stagnation_cycles) { final_status = GMR_STAGNATED; break; }
    }
    // --- one cycle ---
    const int mc = (int)std::min<int64_t>(m, prm.max_iters - it);
    if (graph.use) {
      if (!graph.exec || graph.mc != mc) {
        GMR_TRY(graph.capture(c.s, [&]() { return enqueue_cycle(mc); }));
        graph.mc = mc;
      }
      GMR_HIP(hipGraphLaunch(graph.exec, c.s));
    } else if (coop_blocks > 0) {
      GridBarrier* bar = ws.barrier();
      coop_reset_kernel<<<1, 64, 0, c.s>>>(bar, st_dev);
      GMR_TRY(check_launch("coop_reset_kernel"));
      int nn = n;
      const int* rp = a.Ain->row_ptr;
      const int* ci = a.Ain->col_idx;
      const TI* vi = (const TI*)a.Ain->val;
      const int* rpo = a.Aout->row_ptr;
      const int* cio = a.Aout->col_idx;
      const TO* vo = (const TO*)a.Aout->val;
      TI* Vp = V;
      int64_t ldv = B.ldv;
      TI* w0 = W[0];
      TI* w1 = W[1];
      double* part = ws.partial();
      int mcc = mc;
      double stop_rel = implicit_stop ? prm.tol * bnorm : -1.0;
      double thr = brk_thresh;
      void* args[] = {&nn, &rp, &ci, &vi, &rpo, &cio, &vo, (void*)&b, (void*)&x, &r, &Vp, &ldv, &w0, &w1,
                      &cs, &part, &bar, &mcc, &stop_rel, &thr};
      GMR_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(coop_cycle_kernel<TI, TO>),
                                         dim3(coop_blocks), dim3(kBlock), args, 0, c.s));
    } else if (persistent && n <= kSmallMaxN) {
      small_cycle_kernel<TI, TO><<<1, kBlock, 0, c.s>>>(
          n, a.Ain->row_ptr, a.Ain->col_idx, (const TI*)a.Ain->val, a.Aout->row_ptr, a.Aout->col_idx,
          (const TO*)a.Aout->val, b, x, r, V, B.ldv, W[0], W[1], cs, ws.partial(), ws.h1t<TI>(),
          ws.h2t<TI>(), mc, implicit_stop ? prm.tol * bnorm : -1.0, brk_thresh);
      GMR_TRY(check_launch("small_cycle_kernel"));
    } else {
      GMR_TRY(enqueue_cycle(mc));
      GMR_TRY(residual());
    }
    const double gamma_cycle = gamma;
    GMR_HIP(hipMemcpyAsync(&st, st_dev, sizeof(Status), hipMemcpyDeviceToHost, c.s));
    GMR_HIP(hipStreamSynchronize(c.s));
    it += st.k;
    R.cycles += 1;
    R.implicit_rel_res = st.res * gamma_cycle / bnorm;
    gamma = st.gamma;
    push_hist(gamma / bnorm);
    // (the flag is only maintained by the cooperative cycle, which clears it before each launch)
    if (coop_blocks > 0 && st.barrier_timeout) { final_status = GMR_ERR_HIP; fail(GMR_ERR_HIP, "cooperative cycle: a grid barrier timed out"); break; }
    if (st.nonfinite) { final_status = GMR_ERR_NONFINITE; fail(GMR_ERR_NONFINITE, "non-finite value in the Hessenberg problem"); break; }
    // §V-F: the cycle ended on its implicit residual (or a breakdown) but the
    // explicit one is above tol.  The next restart starts from the explicit
    // residual, which corrects it, unless the caller asked to stop here.
    if (implicit_stop && st.done && gamma / bnorm > prm.tol) {
      R.loss_of_accuracy += 1;
      if (prm.flags & GMR_FLAG_STOP_ON_LOSS) { final_status = GMR_LOSS_OF_ACCURACY; break; }
    }
  }
  GMR_HIP(hipStreamSynchronize(c.s));
  const auto t_end = std::chrono::steady_clock::now();
  R.status = final_status;
  R.iters = it;
  R.rel_res = gamma / bnorm;
  R.seconds = std::chrono::duration<double>(t_end - t_start).count();
  if (c.prof) {
    double ms = 0.0;
    for (size_t i = 0; i + 1 < pf.used; i += 2) {
      float e = 0.f;
      GMR_HIP(hipEventElapsedTime(&e, pf.pool[i], pf.pool[i + 1]));
      ms += e;
    }
    R.prof_ms = ms;
    R.prof_launches = pf.launches;
    R.prof_bytes = pf.bytes;
  }
  *a.res = R;
  return final_status;
}


// ---------------------------------------------------------------------------
// GMRES-FD (§III-C, option 1): float32 GMRES(m) for a fixed number of
// iterations, then float64 GMRES(m) started from the float32 iterate.  Both
// phases are the plain solver above; the driver only adds the two casts.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void narrow_pair_kernel(int n, const double* __restrict__ b,
                                                             const double* __restrict__ x,
                                                             float* __restrict__ b32, float* __restrict__ x32) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    b32[i] = float(b[i]);
    x32[i] = float(x[i]);
  }
}

struct FdLayout {
  size_t solver_end, b32, x32, end;
};

// The two phases share the solver workspace (sized for the larger, float64,
// phase); the float32 copies of b and of the iterate follow it.
static FdLayout fd_layout(int n, int m) {
  const Small S = small_layout(n);
  FdLayout L;
  L.solver_end = std::max(big_layout(S.end, n, m, 8, 8, false).end, big_layout(S.end, n, m, 4, 4, false).end);
  L.b32 = L.solver_end;
  L.x32 = align_up(L.b32 + (size_t)n * 4, 256);
  L.end = align_up(L.x32 + (size_t)n * 4, 256);
  return L;
}

static gmr_status fd_solve(const gmr_csr* A64, const gmr_csr* A32, const double* b, double* x,
                           const gmr_params* prm, int64_t switch_iters, void* ws, size_t ws_bytes,
                           gmr_result* res, gmr_result* res32, double* hist, hipStream_t s) {
  const auto t_start = std::chrono::steady_clock::now();
  const int n = A64->n;
  const FdLayout L = fd_layout(n, prm->restart);
  if (!ws || ws_bytes < L.end)
    return fail(GMR_ERR_WORKSPACE, "gmres_fd_solve: workspace too small: need " + std::to_string(L.end) + " bytes");
  float* b32 = (float*)((char*)ws + L.b32);
  float* x32 = (float*)((char*)ws + L.x32);
  gmr_result R1{};
  R1.status = GMR_OK;
  if (switch_iters > 0) {
    narrow_pair_kernel<<<stream_grid(n), kBlock, 0, s>>>(n, b, x, b32, x32);
    GMR_TRY(check_launch("narrow_pair_kernel"));
    gmr_params p1 = *prm;
    p1.max_iters = switch_iters;
    SolveArgs a1{A32, A32, nullptr, b32, x32, &p1, ws, L.solver_end, &R1, hist, s};
    const gmr_status st1 = solve_impl<float, float>(a1);
    if (st1 < 0) {  // x is left as it was; both records describe phase one
      R1.status = st1;
      if (res32) *res32 = R1;
      *res = R1;
      return st1;
    }
    cast_vec_kernel<float, double><<<stream_grid(n), kBlock, 0, s>>>(n, x32, x, nullptr);
    GMR_TRY(check_launch("cast_vec_kernel"));
  }
  if (res32) *res32 = R1;
  gmr_params p2 = *prm;
  p2.max_iters = prm->max_iters - R1.iters;
  gmr_result R2{};
  SolveArgs a2{A64, A64, nullptr, b, x, &p2, ws, L.solver_end, &R2, hist ? hist + R1.history_len : nullptr, s};
  const gmr_status st2 = solve_impl<double, double>(a2);
  if (st2 < 0 && st2 != GMR_ERR_NONFINITE) return st2;
  gmr_result R = R2;
  R.cycles += R1.cycles;
  R.iters += R1.iters;
  R.history_len += R1.history_len;
  R.loss_of_accuracy += R1.loss_of_accuracy;
  R.prof_ms += R1.prof_ms;
  R.prof_launches += R1.prof_launches;
  R.prof_bytes += R1.prof_bytes;
  R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  *res = R;
  return st2;
}

}  // namespace gmr

using namespace gmr;

// ---------------------------------------------------------------------------
// Library-owned scratch for cgs2_orth_noalloc.  Up to kNoAllocMaxN rows the
// small workspace region (reduction partials, coefficients, status) has one
// fixed size, which is all a standalone CGS2 step uses; every device the
// library runs on holds one copy of the array until the process ends.  Its
// device address comes from hipGetSymbolAddress, once per device: in host
// code the array's name is not a device address.
// ---------------------------------------------------------------------------
constexpr int32_t kNoAllocMaxN = 1 << 27;  // spmv_grid(n) <= kMaxCols * kPartPitch up to here
constexpr size_t kNoAllocScratchBytes = small_layout(1).end;
static_assert(small_layout(kNoAllocMaxN).end == kNoAllocScratchBytes, "small region grows below kNoAllocMaxN");

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

static gmr_status noalloc_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  int dev = 0;
  GMR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GMR_ERR_UNSUPPORTED, "cgs2_orth_noalloc: device ordinal >= 64");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    GMR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GMR_ERR_HIP, "cgs2_orth_noalloc: hipGetSymbolAddress returned a null address");
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return GMR_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* gmr_last_error(void) { return last_error().c_str(); }

size_t gmres_workspace_bytes(int32_t n, const gmr_params* params, int32_t dtype, int32_t with_poly) {
  if (n <= 0 || !params || params->restart < 1 || params->restart > kMaxCols) return 0;
  if (dtype != GMR_F32 && dtype != GMR_F64) return 0;
  const Small S = small_layout(n);
  // the outer precision is float64 except for a float32-only solve; size for float64
  const Big B = big_layout(S.end, n, params->restart, dsize(dtype), 8, with_poly != 0);
  return B.end;
}

gmr_status spmv(const gmr_csr* A, const void* x, void* y, void* stream) {
  GMR_TRY(check_csr(A, "spmv"));
  if (!x || !y) return fail(GMR_ERR_INVALID, "spmv: null vector");
  if (x == y) return fail(GMR_ERR_INVALID, "spmv: x and y must not overlap");
  Ctx c{(hipStream_t)stream, nullptr};
  if (A->dtype == GMR_F64)
    return launch_spmv<double>(c, A, (const double*)x, nullptr, nullptr, (double*)y, nullptr);
  return launch_spmv<float>(c, A, (const float*)x, nullptr, nullptr, (float*)y, nullptr);
}

gmr_status cgs2_orth(int32_t dtype, int32_t n, int32_t k, const void* V, int64_t ldv, void* w,
                     double* h, void* ws, size_t ws_bytes, void* stream) {
  if (dtype != GMR_F32 && dtype != GMR_F64) return fail(GMR_ERR_INVALID, "cgs2_orth: unknown dtype");
  if (n <= 0 || k < 1) return fail(GMR_ERR_INVALID, "cgs2_orth: need n > 0 and k >= 1");
  if (k > kMaxCols) return fail(GMR_ERR_UNSUPPORTED, "cgs2_orth: k > 512 is not supported");
  if (ldv < n) return fail(GMR_ERR_INVALID, "cgs2_orth: ldv < n");
  if (!V || !w || !h) return fail(GMR_ERR_INVALID, "cgs2_orth: null pointer");
  const Small S = small_layout(n);
  if (!ws || ws_bytes < S.end) return fail(GMR_ERR_WORKSPACE, "cgs2_orth: workspace too small");
  Ws W{(char*)ws, S};
  Ctx c{(hipStream_t)stream, nullptr};
  CycleState cs = W.cycle(k);
  if (dtype == GMR_F64) {
    GMR_TRY((cgs2_passes<double, kTailStandalone>(c, n, k, (const double*)V, ldv, (double*)w, W, cs, k - 1, h, nullptr)));
    scale_kernel<double><<<stream_grid(n), kBlock, 0, c.s>>>(n, (const double*)w, cs.inv_beta, (double*)w, nullptr);
  } else {
    GMR_TRY((cgs2_passes<float, kTailStandalone>(c, n, k, (const float*)V, ldv, (float*)w, W, cs, k - 1, h, nullptr)));
    scale_kernel<float><<<stream_grid(n), kBlock, 0, c.s>>>(n, (const float*)w, cs.inv_beta, (float*)w, nullptr);
  }
  return check_launch("scale_kernel");
}

gmr_status cgs2_orth_noalloc(int32_t dtype, int32_t n, int32_t k, const void* V, int64_t ldv, void* w,
                             double* h, void* stream) {
  if (dtype != GMR_F32 && dtype != GMR_F64) return fail(GMR_ERR_INVALID, "cgs2_orth_noalloc: unknown dtype");
  if (n <= 0 || k < 1) return fail(GMR_ERR_INVALID, "cgs2_orth_noalloc: need n > 0 and k >= 1");
  if (n > kNoAllocMaxN)
    return fail(GMR_ERR_UNSUPPORTED, "cgs2_orth_noalloc: n > 134217728 exceeds the static scratch array");
  if (k > kMaxCols) return fail(GMR_ERR_UNSUPPORTED, "cgs2_orth_noalloc: k > 512 is not supported");
  if (ldv < n) return fail(GMR_ERR_INVALID, "cgs2_orth_noalloc: ldv < n");
  if (!V || !w || !h) return fail(GMR_ERR_INVALID, "cgs2_orth_noalloc: null pointer");
  void* ws = nullptr;
  GMR_TRY(noalloc_scratch(&ws));
  return cgs2_orth(dtype, n, k, V, ldv, w, h, ws, kNoAllocScratchBytes, stream);
}

gmr_status csr_values_to_f32(const double* in, float* out, int64_t count, void* stream) {
  if (count < 0 || (count > 0 && (!in || !out))) return fail(GMR_ERR_INVALID, "csr_values_to_f32: bad arguments");
  if (count == 0) return GMR_OK;
  const int G = (int)std::min<int64_t>((count + kBlock - 1) / kBlock, 4096);
  cast_f64_f32_kernel<<<G, kBlock, 0, (hipStream_t)stream>>>(count, in, out);
  return check_launch("cast_f64_f32_kernel");
}

}  // extern "C"

namespace gmr {
template <class T>
static gmr_status poly_setup_t(const gmr_csr* A, int32_t degree, const void* v0, void* wsp,
                               size_t ws_bytes, gmr_poly** out, hipStream_t s) {
  const int n = A->n;
  const int k = degree + 1;
  const Small S = small_layout(n);
  const Big B = big_layout(S.end, n, k, sizeof(T), sizeof(T), false);
  if (!wsp || ws_bytes < B.end) return fail(GMR_ERR_WORKSPACE, "poly_prec_setup: workspace too small");
  Ws ws{(char*)wsp, S};
  Ctx c{s, nullptr};
  T* V = ws.at<T>(B.V);
  T* W[2] = {ws.at<T>(B.W0), ws.at<T>(B.W1)};
  CycleState cs = ws.cycle(k);
  Status* st_dev = ws.status();
  GMR_HIP(hipMemcpyAsync(W[0], v0, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s));
  double* nrm = cs.inv_beta + 1;
  norm2_kernel<T><<<stream_grid(n), kBlock, 0, s>>>(n, W[0], ws.partial());
  GMR_TRY(check_launch("norm2_kernel"));
  finish_norm2_kernel<<<1, kBlock, 0, s>>>(stream_grid(n), ws.partial(), nrm);
  GMR_TRY(check_launch("finish_norm2_kernel"));
  arnoldi_init_kernel<<<1, 1, 0, s>>>(cs, nrm);
  GMR_TRY(check_launch("arnoldi_init_kernel"));
  const int* done = &st_dev->done;
  int cur = 0;
  for (int j = 0; j < k; ++j) {
    GMR_TRY(launch_spmv<T>(c, A, W[cur], cs.inv_beta, V + (size_t)j * B.ldv, W[cur ^ 1], done));
    GMR_TRY((cgs2_passes<T, kTailGivens>(c, n, j + 1, V, B.ldv, W[cur ^ 1], ws, cs, k - 1, nullptr, done)));
    cur ^= 1;
  }
  Status st;
  std::vector<double> Hraw((size_t)(k + 1) * k);
  GMR_HIP(hipMemcpyAsync(&st, st_dev, sizeof(Status), hipMemcpyDeviceToHost, s));
  GMR_HIP(hipMemcpyAsync(Hraw.data(), cs.Hraw, Hraw.size() * 8, hipMemcpyDeviceToHost, s));
  GMR_HIP(hipStreamSynchronize(s));
  if (st.nonfinite && !st.breakdown) return fail(GMR_ERR_NONFINITE, "poly_prec_setup: non-finite Arnoldi");
  const int steps = st.k;
  const int ld = k + 1;
  if (steps < 1) return fail(GMR_ERR_NONFINITE, "poly_prec_setup: start vector is zero");
  std::vector<double> re(steps), im(steps);
  if (steps == k && !st.breakdown) {
    GMR_TRY(gmr_harmonic_ritz(k, Hraw.data(), ld, re.data(), im.data()));
  } else {
    // lucky breakdown: the Ritz values of the s x s Hessenberg matrix are exact
    std::vector<double> M((size_t)steps * steps);
    for (int jcol = 0; jcol < steps; ++jcol)
      for (int i = 0; i < steps; ++i)
        M[(size_t)jcol * steps + i] = (i > jcol + 1) ? 0.0 : Hraw[(size_t)jcol * ld + i];
    GMR_TRY(gmr_hessenberg_eigvals(steps, M.data(), re.data(), im.data()));
  }
  GMR_TRY(gmr_leja_order(steps, re.data(), im.data()));
  gmr_poly* P = new gmr_poly;
  P->dtype = A->dtype;
  P->hess.assign(Hraw.begin(), Hraw.begin() + (size_t)steps * ld);
  P->ldh = ld;
  P->re.resize(steps);
  P->im.resize(steps);
  for (int i = 0; i < steps; ++i) {
    P->re[i] = (double)(T)re[i];
    P->im[i] = (double)(T)im[i];
    if (P->re[i] == 0.0 && P->im[i] == 0.0) {
      delete P;
      return fail(GMR_ERR_NONFINITE, "poly_prec_setup: zero harmonic Ritz value");
    }
  }
  *out = P;
  return GMR_OK;
}

}  // namespace gmr

extern "C" {

gmr_status poly_prec_setup(const gmr_csr* A, int32_t degree, const void* v0, void* ws,
                           size_t ws_bytes, gmr_poly** out, void* stream) {
  GMR_TRY(check_csr(A, "poly_prec_setup"));
  if (!v0 || !out) return fail(GMR_ERR_INVALID, "poly_prec_setup: null pointer");
  if (degree < 0 || degree > 128) return fail(GMR_ERR_UNSUPPORTED, "poly_prec_setup: degree must be in [0, 128]");
  *out = nullptr;
  if (A->dtype == GMR_F64) return poly_setup_t<double>(A, degree, v0, ws, ws_bytes, out, (hipStream_t)stream);
  return poly_setup_t<float>(A, degree, v0, ws, ws_bytes, out, (hipStream_t)stream);
}

size_t bjac_prec_bytes(int32_t n, int32_t block, int32_t dtype) {
  if (n <= 0 || block < 1 || block > kBjacMaxBlock || (dtype != GMR_F32 && dtype != GMR_F64)) return 0;
  return bjac_blocks_offset() + (size_t)ceil_div(n, block) * block * block * dsize(dtype);
}

gmr_status bjac_prec_setup(const gmr_csr* A, int32_t block, void* inv, size_t inv_bytes, gmr_poly** out,
                           void* stream) {
  GMR_TRY(check_csr(A, "bjac_prec_setup"));
  if (!out) return fail(GMR_ERR_INVALID, "bjac_prec_setup: null pointer");
  if (block < 1) return fail(GMR_ERR_INVALID, "bjac_prec_setup: block < 1");
  if (block > kBjacMaxBlock) return fail(GMR_ERR_UNSUPPORTED, "bjac_prec_setup: block > 64 is not supported");
  const size_t need = bjac_prec_bytes(A->n, block, A->dtype);
  if (!inv || inv_bytes < need)
    return fail(GMR_ERR_WORKSPACE, "bjac_prec_setup: inv needs " + std::to_string(need) + " bytes");
  if ((uintptr_t)inv % 256 != 0) return fail(GMR_ERR_INVALID, "bjac_prec_setup: inv must be 256-byte aligned");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  int* flag = (int*)inv;
  char* blocks = (char*)inv + bjac_blocks_offset();
  GMR_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  const int nblk = ceil_div(A->n, block);
  if (A->dtype == GMR_F64)
    bjac_invert_kernel<double><<<nblk, kBlock, 0, s>>>(A->n, block, A->row_ptr, A->col_idx,
                                                      (const double*)A->val, (double*)blocks, flag);
  else
    bjac_invert_kernel<float><<<nblk, kBlock, 0, s>>>(A->n, block, A->row_ptr, A->col_idx,
                                                     (const float*)A->val, (float*)blocks, flag);
  GMR_TRY(check_launch("bjac_invert_kernel"));
  int bad = 0;
  GMR_HIP(hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  GMR_HIP(hipStreamSynchronize(s));
  if (bad) return fail(GMR_ERR_NONFINITE, "bjac_prec_setup: a diagonal block is singular");
  gmr_poly* P = new gmr_poly;
  P->dtype = A->dtype;
  P->kind = kPrecBjac;
  P->n = A->n;
  P->block = block;
  P->inv = blocks;
  *out = P;
  return GMR_OK;
}

int32_t prec_block_size(const gmr_poly* P) { return P && P->kind == kPrecBjac ? P->block : 0; }

gmr_status poly_prec_apply(const gmr_poly* P, const gmr_csr* A, const void* x, void* y, void* wsp,
                           size_t ws_bytes, void* stream) {
  if (!P) return fail(GMR_ERR_INVALID, "poly_prec_apply: null polynomial");
  GMR_TRY(check_csr(A, "poly_prec_apply"));
  if (A->dtype != P->dtype) return fail(GMR_ERR_INVALID, "poly_prec_apply: dtype of A and P differ");
  if (!x || !y || x == y) return fail(GMR_ERR_INVALID, "poly_prec_apply: bad vectors");
  const int n = A->n;
  if (P->kind == kPrecBjac) {
    if (P->n != n) return fail(GMR_ERR_INVALID, "poly_prec_apply: block Jacobi built for another order n");
    Ctx c{(hipStream_t)stream, nullptr};
    if (A->dtype == GMR_F64)
      return poly_apply_impl<double>(c, P, A, (const double*)x, (double*)y, nullptr, nullptr, nullptr, nullptr);
    return poly_apply_impl<float>(c, P, A, (const float*)x, (float*)y, nullptr, nullptr, nullptr, nullptr);
  }
  const Small S = small_layout(n);
  const size_t s = dsize(A->dtype);
  const size_t need = S.end + 3 * align_up((size_t)n * s, 256);
  if (!wsp || ws_bytes < need) return fail(GMR_ERR_WORKSPACE, "poly_prec_apply: workspace too small");
  char* base = (char*)wsp + S.end;
  const size_t stride = align_up((size_t)n * s, 256);
  Ctx c{(hipStream_t)stream, nullptr};
  if (A->dtype == GMR_F64)
    return poly_apply_impl<double>(c, P, A, (const double*)x, (double*)y, (double*)base,
                                   (double*)(base + stride), (double*)(base + 2 * stride), nullptr);
  return poly_apply_impl<float>(c, P, A, (const float*)x, (float*)y, (float*)base,
                                (float*)(base + stride), (float*)(base + 2 * stride), nullptr);
}

void poly_prec_destroy(gmr_poly* P) { delete P; }

gmr_status poly_prec_hessenberg(const gmr_poly* P, double* H) {
  if (!P || !H) return fail(GMR_ERR_INVALID, "poly_prec_hessenberg: null pointer");
  const int s = (int)P->re.size();
  for (int j = 0; j < s; ++j)
    for (int i = 0; i <= s; ++i)
      H[(size_t)j * (s + 1) + i] = (i > j + 1) ? 0.0 : P->hess[(size_t)j * P->ldh + i];
  return GMR_OK;
}

int32_t poly_prec_degree(const gmr_poly* P) { return P ? (int32_t)P->re.size() - 1 : -1; }

gmr_status poly_prec_roots(const gmr_poly* P, double* re, double* im) {
  if (!P || !re || !im) return fail(GMR_ERR_INVALID, "poly_prec_roots: null pointer");
  std::copy(P->re.begin(), P->re.end(), re);
  std::copy(P->im.begin(), P->im.end(), im);
  return GMR_OK;
}

static gmr_status solve_common_checks(const gmr_params* params, const void* b, void* x, gmr_result* result) {
  GMR_TRY(check_params(params));
  if (!b || !x || !result) return fail(GMR_ERR_INVALID, "null b, x or result");
  if (b == x) return fail(GMR_ERR_INVALID, "b and x must not overlap");
  return GMR_OK;
}

gmr_status gmres_solve(const gmr_csr* A, const gmr_poly* P, const void* b, void* x,
                       const gmr_params* params, void* ws, size_t ws_bytes, gmr_result* result,
                       double* hist, void* stream) {
  GMR_TRY(check_csr(A, "gmres_solve"));
  GMR_TRY(solve_common_checks(params, b, x, result));
  if (P && P->dtype != A->dtype) return fail(GMR_ERR_INVALID, "gmres_solve: polynomial dtype differs from A");
  SolveArgs a{A, A, P, b, x, params, ws, ws_bytes, result, hist, (hipStream_t)stream};
  if (A->dtype == GMR_F64) return solve_impl<double, double>(a);
  return solve_impl<float, float>(a);
}

gmr_status gmres_ir_solve(const gmr_csr* A64, const gmr_csr* A32, const gmr_poly* P,
                          const double* b, double* x, const gmr_params* params, void* ws,
                          size_t ws_bytes, gmr_result* result, double* hist, void* stream) {
  GMR_TRY(check_csr(A64, "gmres_ir_solve(A64)"));
  GMR_TRY(check_csr(A32, "gmres_ir_solve(A32)"));
  if (A64->dtype != GMR_F64 || A32->dtype != GMR_F32)
    return fail(GMR_ERR_INVALID, "gmres_ir_solve: A64 must be float64 and A32 float32");
  if (A64->n != A32->n || A64->nnz != A32->nnz)
    return fail(GMR_ERR_INVALID, "gmres_ir_solve: A64 and A32 differ in size");
  if (P && P->dtype != GMR_F32) return fail(GMR_ERR_INVALID, "gmres_ir_solve: the polynomial must be float32");
  GMR_TRY(solve_common_checks(params, b, x, result));
  SolveArgs a{A32, A64, P, b, x, params, ws, ws_bytes, result, hist, (hipStream_t)stream};
  return solve_impl<float, double>(a);
}

gmr_status gmres_f32prec_solve(const gmr_csr* A64, const gmr_csr* A32, const gmr_poly* P32, const double* b,
                               double* x, const gmr_params* params, void* ws, size_t ws_bytes,
                               gmr_result* result, double* hist, void* stream) {
  GMR_TRY(check_csr(A64, "gmres_f32prec_solve(A64)"));
  GMR_TRY(check_csr(A32, "gmres_f32prec_solve(A32)"));
  if (A64->dtype != GMR_F64 || A32->dtype != GMR_F32)
    return fail(GMR_ERR_INVALID, "gmres_f32prec_solve: A64 must be float64 and A32 float32");
  if (A64->n != A32->n || A64->nnz != A32->nnz)
    return fail(GMR_ERR_INVALID, "gmres_f32prec_solve: A64 and A32 differ in size");
  if (!P32 || P32->dtype != GMR_F32)
    return fail(GMR_ERR_INVALID, "gmres_f32prec_solve: needs a float32 polynomial");
  GMR_TRY(solve_common_checks(params, b, x, result));
  SolveArgs a{A64, A64, P32, b, x, params, ws, ws_bytes, result, hist, (hipStream_t)stream, A32};
  return solve_impl<double, double>(a);
}

size_t gmres_fd_workspace_bytes(int32_t n, const gmr_params* params) {
  if (n <= 0 || !params || params->restart < 1 || params->restart > kMaxCols) return 0;
  return fd_layout(n, params->restart).end;
}

gmr_status gmres_fd_solve(const gmr_csr* A64, const gmr_csr* A32, const double* b, double* x,
                          const gmr_params* params, int64_t switch_iters, void* ws, size_t ws_bytes,
                          gmr_result* result, gmr_result* float_result, double* hist, void* stream) {
  GMR_TRY(check_csr(A64, "gmres_fd_solve(A64)"));
  GMR_TRY(check_csr(A32, "gmres_fd_solve(A32)"));
  if (A64->dtype != GMR_F64 || A32->dtype != GMR_F32)
    return fail(GMR_ERR_INVALID, "gmres_fd_solve: A64 must be float64 and A32 float32");
  if (A64->n != A32->n || A64->nnz != A32->nnz)
    return fail(GMR_ERR_INVALID, "gmres_fd_solve: A64 and A32 differ in size");
  GMR_TRY(solve_common_checks(params, b, x, result));
  if (switch_iters < 0) return fail(GMR_ERR_INVALID, "gmres_fd_solve: switch_iters < 0");
  if (switch_iters >= params->max_iters)
    return fail(GMR_ERR_INVALID, "gmres_fd_solve: max_iters must exceed switch_iters");
  return fd_solve(A64, A32, b, x, params, switch_iters, ws, ws_bytes, result, float_result, hist,
                  (hipStream_t)stream);
}

}  // extern "C"
