// HIP kernels of the GMRES(m) / GMRES-IR hot path for gfx950.
//
//  * CSR SpMV (§V-D) as "CSR-stream": a block owns 256 consecutive rows,
//    streams their nonzeros with fully coalesced loads, forms the products
//    val[k] * x[col[k]] into LDS and lets each thread add up its own row in
//    ascending k.  Epilogues fuse the vector work that follows the product:
//    the Arnoldi normalisation, the float64 residual b - A x with its norm,
//    and the GMRES-polynomial recurrences.
//  * CGS2 (§III-A: two classical Gram-Schmidt passes per iteration) as three
//    passes over the basis V: dots, update+dots, update+norm.  A wave owns 64
//    rows (one per lane); the per-column partial dots of those rows are
//    reduced across lanes by a butterfly, and blocks combine their partials
//    in float64 in a fixed order (deterministic).
//  * The least-squares problem of Alg. 1 is solved by Givens rotations in
//    float64 inside the last block of the update+norm pass.
#pragma once

#include <math.h>

#include "device_common.hpp"

namespace gmr {

// Rows of an SpMV-type kernel per thread and per block of kBlock threads:
// thread t owns rows r0 + t + i * kBlock, i < kSpmvRpt.  Two rows per thread
// halve the blocks (and the row-pointer / barrier overhead per row) and keep
// twice the (index, value) loads of a thread in flight.
#ifndef GMR_SPMV_RPT
#define GMR_SPMV_RPT 2
#endif
constexpr int kSpmvRpt = GMR_SPMV_RPT;
constexpr int kSpmvRows = kBlock * kSpmvRpt;
// Nonzeros staged in LDS per pass (16 KB of float32 or 32 KB of float64
// products): a block of 512 rows with up to 8 nonzeros per row takes one pass.
// Measured on the 3D Laplacian 150^3 and the 2500^2 five-point matrix against
// one row per thread and against 8 or 16 KB passes, this is the fastest form
// in float32 (46.8 / 61.2 us) and in float64 (71.8 / 94.9 us).
#ifndef GMR_SPMV_CHUNK
#define GMR_SPMV_CHUNK 4096
#endif
template <class T>
struct SpmvCfg {
  static constexpr int kChunk = GMR_SPMV_CHUNK;
};
// Upper bound on the number of blocks of a reduction kernel (partials per column).
constexpr int kMaxRedBlocks = 1024;
// Basis columns (j) supported by the kernels; H has restart+1 rows.
constexpr int kMaxCols = 512;
// Column partials are stored column-major: partial[c * kPartPitch + block], so
// the finish kernel of column c reads one contiguous run.
constexpr int kPartPitch = kMaxRedBlocks;

// Device-resident state of one GMRES cycle.  Everything the host needs after a
// cycle sits in `Status`, read back with one small copy.
struct Status {
  double gamma;       // ||r|| of the outer residual (float64 or the outer precision)
  double inv_gamma;   // 1 / gamma
  double bnorm;       // ||b||
  double res;         // |g_{k+1}| of the cycle (inner units)
  double beta0;       // norm of the cast, scaled residual (inner start vector)
  double stop_thresh; // stop the cycle when |g_{j+1}| <= stop_thresh (< 0: never)
  int k;              // iterations completed in the cycle
  int done;           // the cycle ended early (implicit convergence or breakdown)
  int breakdown;      // h_{j+1,j} was zero (lucky breakdown)
  int nonfinite;      // NaN/Inf met in the small dense problem
  int barrier_timeout;  // a grid barrier of the cooperative cycle gave up waiting
  int pad;
};

// State of the grid barrier of the cooperative cycle (zeroed before each launch).
struct GridBarrier {
  unsigned int count;  // blocks arrived at the current barrier
  unsigned int gen;    // barriers completed
};

struct CycleState {
  double* H;        // (ldh x m) rotated Hessenberg -> R, column-major
  double* Hraw;     // (ldh x m) Hessenberg as built (for the polynomial setup)
  double* cs;       // m cosines
  double* sn;       // m sines
  double* g;        // ldh entries, gamma e1 rotated
  double* y;        // m entries, least-squares solution (float64)
  double* h1d;      // kMaxCols, first-pass coefficients (float64 sums)
  double* h2d;      // kMaxCols, second-pass coefficients
  double* inv_beta; // 1 / h_{j+1,j} of the latest column (normalisation factor)
  Status* st;
  int ldh;          // m + 1
};

// ===========================================================================
// SpMV core
// ===========================================================================
// Loads the 4 consecutive CSR entries starting at kk (a multiple of 4) with
// 16-byte vector loads when they lie inside the arrays (col_idx and val are
// 16-byte aligned, which the host checks), element by element at the end.
// The matrix is streamed once per product, so the vector loads are marked
// non-temporal: they do not displace the gathered x from the caches.
typedef int ivec4_t __attribute__((ext_vector_type(4)));
typedef float fvec4_t __attribute__((ext_vector_type(4)));
typedef double dvec2_t __attribute__((ext_vector_type(2)));

template <class T>
__device__ __forceinline__ void load_quad(const int* __restrict__ ci, const T* __restrict__ val,
                                          int kk, int nnz, int (&c)[4], T (&a)[4]) {
  if (kk + 4 <= nnz) {
    const ivec4_t c4 = __builtin_nontemporal_load(reinterpret_cast<const ivec4_t*>(ci + kk));
    c[0] = c4.x; c[1] = c4.y; c[2] = c4.z; c[3] = c4.w;
    if constexpr (sizeof(T) == 4) {
      const fvec4_t a4 = __builtin_nontemporal_load(reinterpret_cast<const fvec4_t*>(val + kk));
      a[0] = a4.x; a[1] = a4.y; a[2] = a4.z; a[3] = a4.w;
    } else {
      const dvec2_t a0 = __builtin_nontemporal_load(reinterpret_cast<const dvec2_t*>(val + kk));
      const dvec2_t a1 = __builtin_nontemporal_load(reinterpret_cast<const dvec2_t*>(val + kk + 2));
      a[0] = a0.x; a[1] = a0.y; a[2] = a1.x; a[3] = a1.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = kk + i;
      c[i] = (k < nnz) ? ci[k] : 0;
      a[i] = (k < nnz) ? val[k] : T(0);
    }
  }
}

// Four consecutive products into LDS at a 4-aligned slot (16-byte aligned
// for float, two 16-byte stores for double).
template <class T>
__device__ __forceinline__ void store_quad(T* dst, const T (&p)[4]) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<fvec4_t*>(dst) = fvec4_t{p[0], p[1], p[2], p[3]};
  } else {
    reinterpret_cast<dvec2_t*>(dst)[0] = dvec2_t{p[0], p[1]};
    reinterpret_cast<dvec2_t*>(dst)[1] = dvec2_t{p[2], p[3]};
  }
}

// Computes, for thread t of the block, the dot products of rows
// r0 + t + i * kBlock (i < RPT, by default kSpmvRpt) with x (x scaled by `s` when SCALED) into
// acc[i]; 0 for rows past the last one.  The block's nonzeros are processed in
// passes of SpmvCfg<T>::kChunk entries that start on a multiple of 4.  In a
// pass each thread takes up to Q quads of (col, val) with vector loads (none
// past the block's last nonzero), gathers x for them, and stores the four
// rounded products into LDS with one vector store; after a barrier every
// thread adds up its own rows in ascending k (so the pass length CH does not
// change the result).  Entries of a quad that belong to a neighbouring block
// (before k0 or from k1 on) produce products in LDS slots no row of this
// block reads, so no per-entry masking is needed.  The
// row bounds come straight from global memory: the block's first and last
// (uniform, scalar loads) and each thread's own, with no LDS staging and no
// barrier before the nonzero loads are issued.  A non-null `done` flag is read
// together with those uniform row bounds (one round trip for both instead of
// one before the other); when it is set the whole block returns false and the
// caller skips its epilogue.
template <class T, bool SCALED, int CH = SpmvCfg<T>::kChunk, int RPT = kSpmvRpt>
__device__ __forceinline__ bool spmv_rows(int n, int r0, const int* __restrict__ rp,
                                          const int* __restrict__ ci, const T* __restrict__ val,
                                          const T* __restrict__ x, T s, T* s_prod, T (&acc)[RPT],
                                          const int* __restrict__ done = nullptr) {
  constexpr int Q = CH / (4 * kBlock);  // quads per thread per pass
  const int t = threadIdx.x;
  const int nr = min(kBlock * RPT, n - r0);
  // without a flag the load reads row_ptr[0] (0 by the CSR convention), so
  // the four uniform loads have no branch between them
  const int* flag = done ? done : rp;
  const int k0 = rp[r0];
  const int k1 = rp[r0 + nr];
  const int nnz = rp[n];
  if (*flag != 0 && done) return false;
  int rs[RPT], re[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int rl = t + i * kBlock;
    rs[i] = (rl < nr) ? rp[r0 + rl] : 0;
    re[i] = (rl < nr) ? rp[r0 + rl + 1] : 0;
    acc[i] = T(0);
  }
  for (int base = k0 & ~3; base < k1; base += CH) {
    // all loads of the pass are issued before the first one is waited for:
    // the quads, then the gathers (a quad past k1 gathers x[0], in bounds)
    int col[Q][4];
    T a[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kk = base + 4 * (t + q * kBlock);
      if (kk < k1) {
        load_quad<T>(ci, val, kk, nnz, col[q], a[q]);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          col[q][i] = 0;
          a[q][i] = T(0);
        }
      }
    }
    T v[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[q][i] = x[col[q][i]];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kk = base + 4 * (t + q * kBlock);
      T p[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        T xv = v[q][i];
        if constexpr (SCALED) xv = xv * s;
        p[i] = a[q][i] * xv;
      }
      if (kk < k1) store_quad<T>(s_prod + (kk - base), p);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int lo = max(rs[i], base);
      const int hi = min(re[i], base + CH);
      for (int k = lo; k < hi; ++k) acc[i] += s_prod[k - base];
    }
    __syncthreads();
  }
  return true;
}

// y = A x.  When `scale` is non-null the input is x * (*scale) and, when `vout`
// is non-null, that scaled input is also written to vout for the block's rows
// (this is how v_{j+1} = w / h_{j+1,j} is stored without a separate pass).
template <class T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void spmv_kernel(int n, const int* __restrict__ rp,
                                                      const int* __restrict__ ci,
                                                      const T* __restrict__ val,
                                                      const T* __restrict__ x,
                                                      const double* __restrict__ scale,
                                                      T* __restrict__ vout, T* __restrict__ y,
                                                      const int* __restrict__ done) {
  __shared__ __align__(16) T s_prod[SpmvCfg<T>::kChunk];
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * kSpmvRows;
  T acc[kSpmvRpt];
  if (scale) {
    const T s = T(*scale);
    if (!spmv_rows<T, true>(n, r0, rp, ci, val, x, s, s_prod, acc, done)) return;
    if (vout) {
#pragma unroll
      for (int i = 0; i < kSpmvRpt; ++i) {
        const int r = r0 + threadIdx.x + i * kBlock;
        if (r < n) vout[r] = x[r] * s;
      }
    }
  } else {
    if (!spmv_rows<T, false>(n, r0, rp, ci, val, x, T(1), s_prod, acc, done)) return;
  }
#pragma unroll
  for (int i = 0; i < kSpmvRpt; ++i) {
    const int r = r0 + threadIdx.x + i * kBlock;
    if (r < n) y[r] = acc[i];
  }
}

// r = b - A x with the block's partial ||r||^2 (float64) in partial[blockIdx.x];
// finish_residual_kernel turns the partials into gamma.
template <class T>
__global__ __launch_bounds__(kBlock) void residual_kernel(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci,
                                                          const T* __restrict__ val,
                                                          const T* __restrict__ x,
                                                          const T* __restrict__ b,
                                                          T* __restrict__ r, double* partial) {
  __shared__ __align__(16) T s_prod[SpmvCfg<T>::kChunk];
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * kSpmvRows;
  T acc[kSpmvRpt];
  spmv_rows<T, false>(n, r0, rp, ci, val, x, T(1), s_prod, acc);
  double sq = 0.0;
#pragma unroll
  for (int i = 0; i < kSpmvRpt; ++i) {
    const int row = r0 + threadIdx.x + i * kBlock;
    if (row < n) {
      T rv = b[row] - acc[i];
      r[row] = rv;
      sq += double(rv) * double(rv);
    }
  }
  sq = block_sum(sq);
  if (threadIdx.x == 0) partial[blockIdx.x] = sq;
}

// Sum of nparts float64 partials in a fixed order (one block).
__device__ __forceinline__ double sum_partials(int nparts, const double* __restrict__ partial) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += partial[i];
  return block_sum(s);
}

__global__ __launch_bounds__(kBlock) void finish_residual_kernel(int nparts, const double* partial,
                                                                 Status* st) {
  const double s = sum_partials(nparts, partial);
  if (threadIdx.x == 0) {
    const double g = sqrt(s);
    st->gamma = g;
    st->inv_gamma = 1.0 / g;
  }
}

// ||v||^2 partials of a vector (float64 accumulation).
template <class T>
__global__ __launch_bounds__(kBlock) void norm2_kernel(int n, const T* __restrict__ v,
                                                       double* partial) {
  double sq = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double a = double(v[i]);
    sq += a * a;
  }
  sq = block_sum(sq);
  if (threadIdx.x == 0) partial[blockIdx.x] = sq;
}

// *out = sqrt(sum of partials)
__global__ __launch_bounds__(kBlock) void finish_norm2_kernel(int nparts, const double* partial,
                                                              double* out) {
  const double s = sum_partials(nparts, partial);
  if (threadIdx.x == 0) *out = sqrt(s);
}

// Start of a cycle: w = cast(r * (1/gamma)) into the inner precision with the
// block's partial ||w||^2 accumulated in the inner precision.
template <class TO, class TI>
__device__ __forceinline__ void start_cycle_body(int n, const TO* __restrict__ r,
                                                 TI* __restrict__ w, double* partial,
                                                 const Status* __restrict__ st) {
  const TO ig = TO(st->inv_gamma);
  TI sq = TI(0);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const TI v = TI(r[i] * ig);
    w[i] = v;
    sq += v * v;
  }
  sq = block_sum(sq);
  if (threadIdx.x == 0) partial[blockIdx.x] = double(sq);
}

template <class TO, class TI>
__global__ __launch_bounds__(kBlock) void start_cycle_kernel(int n, const TO* __restrict__ r,
                                                             TI* __restrict__ w, double* partial,
                                                             const Status* __restrict__ st) {
  start_cycle_body<TO, TI>(n, r, w, partial, st);
}

// beta0 = ||w|| (rounded to the inner precision), g = beta0 e1, cycle flags reset.
// `stop_rel` >= 0 arms the implicit residual test |g_{j+1}| * gamma <= stop_rel.
template <class TI>
__device__ __forceinline__ void finish_start_cycle_body(int nparts, const double* partial,
                                                        CycleState cs, double stop_rel) {
  const double s = sum_partials(nparts, partial);
  if (threadIdx.x == 0) {
    const double b0 = sqrt(double(TI(s)));
    Status* st = cs.st;
    st->beta0 = b0;
    cs.g[0] = b0;
    *cs.inv_beta = 1.0 / b0;
    st->k = 0;
    st->done = 0;
    st->breakdown = 0;
    st->nonfinite = !(b0 > 0.0) || !isfinite(b0);
    st->res = b0;
    st->stop_thresh = (stop_rel >= 0.0) ? stop_rel * st->inv_gamma : -1.0;
  }
}

template <class TI>
__global__ __launch_bounds__(kBlock) void finish_start_cycle_kernel(int nparts, const double* partial,
                                                                    CycleState cs, double stop_rel) {
  finish_start_cycle_body<TI>(nparts, partial, cs, stop_rel);
}

// ===========================================================================
// CGS2 passes.  All three share the row mapping: wave `gw` of the grid walks
// row groups grp = gw, gw + G, ... of 64 rows; lane l owns row 64*grp + l.
// ===========================================================================

// Writes the block's per-column partial sums (held per lane after the
// butterfly, column = col_of(lane, i), duplicated lanes skipped) into
// partial[col * kPartPitch + blockIdx.x] as float64, combining the waves of
// the block in a fixed order.
template <int K, class T, int NACC>
__device__ __forceinline__ void publish_col_partials(const T (&acc)[NACC][Butterfly<K>::KOut],
                                                     int j, double* partial) {
  constexpr int KO = Butterfly<K>::KOut;
  __shared__ double s_cols[kWavesPerBlock][kMaxCols];
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  if (Butterfly<K>::owner(lane)) {
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
#pragma unroll
      for (int i = 0; i < KO; ++i) {
        const int col = q * K + Butterfly<K>::col_of(lane, i);
        if (col < j) s_cols[wave][col] = double(acc[q][i]);
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < j; c += kBlock) {
    double s = s_cols[0][c];
#pragma unroll
    for (int w = 1; w < kWavesPerBlock; ++w) s += s_cols[w][c];
    partial[(size_t)c * kPartPitch + blockIdx.x] = s;
  }
}

// out[c] = sum over the nparts blocks of partial[b][c] (one block per column,
// fixed order), plus the copy rounded to the working precision.
template <class T>
__global__ __launch_bounds__(kBlock) void finish_cols_kernel(int nparts, const double* __restrict__ partial,
                                                             double* out, T* outT,
                                                             const int* __restrict__ done) {
  if (done && *done) return;
  const int c = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBlock) s += partial[(size_t)c * kPartPitch + b];
  s = block_sum(s);
  if (threadIdx.x == 0) {
    out[c] = s;
    outT[c] = T(s);
  }
}

// Pass order.  The memory-side cache keeps the rows of V that a pass touched
// last.  Every pass over V takes a direction flag `rev` (row groups in
// descending order), and the host alternates it so that each pass starts on
// the rows the pass before it ended on: a basis larger than the cache then
// still finds about a cache's worth of it there, where passes that all ran
// upward would each evict what the next one needs first.  The order of the
// rows changes only which rows a block sums, not what is computed.

// Pass 1: h = V_j^T w  (j <= NQ * K columns, in NQ chunks of K columns).
template <class T, int K, int NQ>
__device__ __forceinline__ void cgs_dots_body(int n, int j, const T* __restrict__ V,
                                              int64_t ldv, const T* __restrict__ w,
                                              double* partial,
                                              const int* __restrict__ done, bool rev = false) {
  constexpr int KO = Butterfly<K>::KOut;
  if (done && *done) return;
  const int lane = threadIdx.x % kWave;
  const int gw = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const int G = gridDim.x * kWavesPerBlock;
  const int ngrp = (n + kWave - 1) / kWave;
  T acc[NQ][KO];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < KO; ++i) acc[q][i] = T(0);
  for (int it = gw; it < ngrp; it += G) {
    const int grp = rev ? ngrp - 1 - it : it;
    const int r = grp * kWave + lane;
    const bool ok = r < n;
    const T wv = ok ? w[r] : T(0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q * K < j) {
        T a[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int col = q * K + c;
          a[c] = (col < j && ok) ? V[(size_t)col * ldv + r] : T(0);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) a[c] *= wv;
        Butterfly<K>::run(a, lane);
#pragma unroll
        for (int i = 0; i < KO; ++i) acc[q][i] += a[i];
      }
    }
  }
  publish_col_partials<K, T, NQ>(acc, j, partial);
}

// Pass 1 with four rows per lane: lane l of row group grp owns rows
// 256 grp + 4 l .. + 3 and reads them with one 16-byte (float) or 32-byte
// (double) vector load per column (V columns and w are 256-byte aligned); the
// four products of a column are added in the lane before the butterfly.
template <class T, int K, int NQ>
__device__ __forceinline__ void cgs_dots4_body(int n, int j, const T* __restrict__ V, int64_t ldv,
                                               const T* __restrict__ w, double* partial,
                                               const int* __restrict__ done, bool rev = false) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  constexpr int KO = Butterfly<K>::KOut;
  if (done && *done) return;
  const int lane = threadIdx.x % kWave;
  const int gw = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const int G = gridDim.x * kWavesPerBlock;
  const int ngrp = (n + 4 * kWave - 1) / (4 * kWave);
  T acc[NQ][KO];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < KO; ++i) acc[q][i] = T(0);
  for (int it = gw; it < ngrp; it += G) {
    const int grp = rev ? ngrp - 1 - it : it;
    const int r = grp * 4 * kWave + 4 * lane;
    const bool full = r + 3 < n;
    v4 wv;
    if (full) {
      wv = *reinterpret_cast<const v4*>(w + r);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) wv[e] = r + e < n ? w[r + e] : T(0);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q * K < j) {
        T a[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int col = q * K + c;
          v4 v = v4{T(0), T(0), T(0), T(0)};
          if (col < j) {
            const T* Vc = V + (size_t)col * ldv + r;
            if (full) {
              v = *reinterpret_cast<const v4*>(Vc);
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e) v[e] = r + e < n ? Vc[e] : T(0);
            }
          }
          a[c] = ((v.x * wv.x + v.y * wv.y) + v.z * wv.z) + v.w * wv.w;
        }
        Butterfly<K>::run(a, lane);
#pragma unroll
        for (int i = 0; i < KO; ++i) acc[q][i] += a[i];
      }
    }
  }
  publish_col_partials<K, T, NQ>(acc, j, partial);
}

template <class T, int K, int NQ>
__global__ __launch_bounds__(kBlock) void cgs_dots4_kernel(int n, int j, const T* __restrict__ V,
                                                           int64_t ldv, const T* __restrict__ w,
                                                           double* partial,
                                                           const int* __restrict__ done, int rev) {
  cgs_dots4_body<T, K, NQ>(n, j, V, ldv, w, partial, done, rev != 0);
}

template <class T, int K, int NQ>
__global__ __launch_bounds__(kBlock) void cgs_dots_kernel(int n, int j, const T* __restrict__ V,
                                                          int64_t ldv, const T* __restrict__ w,
                                                          double* partial,
                                                          const int* __restrict__ done, int rev) {
  cgs_dots_body<T, K, NQ>(n, j, V, ldv, w, partial, done, rev != 0);
}

// Pass-1 update fused with pass-2 dots: w -= V_j h_in ; h_out = V_j^T w.
// The j basis entries of a row stay in registers between the two uses, so V
// is read once.  Needs j <= K.
// STANDALONE (the kernel below, not the single-block cycle) selects two
// register-saving forms where they pay:
//  * float64, and float32 beyond 64 columns, read the coefficients with
//    wave-uniform loads, which keeps them in scalar registers across the
//    row-group loop; staged in LDS they are hoisted into K vector registers
//    (float64, K = 64: 256 VGPRs -> 149; float32, K = 128: 151).  For
//    float32 up to 64 columns the LDS form measured faster (5.64 against
//    5.50 TB/s at K = 64 on a 3.4M-row basis);
//  * float64 reduces the dots of more than 32 columns in 32-column chunks
//    (149 VGPRs at K = 64 against 187).
template <class T, int K, bool STANDALONE = false>
__device__ __forceinline__ void cgs_update_dots_body(
    int n, int j, const T* __restrict__ V, int64_t ldv, const T* __restrict__ h_in,
    T* __restrict__ w, double* partial, const int* __restrict__ done, bool rev = false) {
  constexpr bool kScalarH = STANDALONE && (sizeof(T) == 8 || K > 64);
  constexpr int KC = (STANDALONE && K > 32 && sizeof(T) == 8) ? 32 : K;
  constexpr int NQ = K / KC;
  constexpr int KO = Butterfly<KC>::KOut;
  __shared__ T s_h[kScalarH ? 1 : K];
  if (done && *done) return;
  T hc[kScalarH ? K : 1];
  if constexpr (kScalarH) {
#pragma unroll
    for (int c = 0; c < K; ++c) hc[c] = (c < j) ? h_in[c] : T(0);
  } else {
    for (int c = threadIdx.x; c < K; c += kBlock) s_h[c] = (c < j) ? h_in[c] : T(0);
    __syncthreads();
  }
  const int lane = threadIdx.x % kWave;
  const int gw = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const int G = gridDim.x * kWavesPerBlock;
  const int ngrp = (n + kWave - 1) / kWave;
  T acc[NQ][KO];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < KO; ++i) acc[q][i] = T(0);
  // rev: row groups in descending order (see the pass-order note above)
  for (int it = gw; it < ngrp; it += G) {
    const int grp = rev ? ngrp - 1 - it : it;
    const int r = grp * kWave + lane;
    const bool ok = r < n;
    T v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = (c < j && ok) ? V[(size_t)c * ldv + r] : T(0);
    T wv = ok ? w[r] : T(0);
#pragma unroll
    for (int c = 0; c < K; ++c) wv -= v[c] * (kScalarH ? hc[c] : s_h[c]);
    if (ok) w[r] = wv;
    // the dots in chunks of KC columns: a chunk's butterfly needs half as
    // many received values live as one over all K columns
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      T a[KC];
#pragma unroll
      for (int c = 0; c < KC; ++c) a[c] = v[q * KC + c] * wv;
      Butterfly<KC>::run(a, lane);
#pragma unroll
      for (int i = 0; i < KO; ++i) acc[q][i] += a[i];
    }
  }
  publish_col_partials<KC, T, NQ>(acc, j, partial);
}

template <class T, int K>
__global__ __launch_bounds__(kBlock) void cgs_update_dots_kernel(
    int n, int j, const T* __restrict__ V, int64_t ldv, const T* __restrict__ h_in,
    T* __restrict__ w, double* partial, const int* __restrict__ done, int rev) {
  cgs_update_dots_body<T, K, true>(n, j, V, ldv, h_in, w, partial, done, rev != 0);
}

// w[r..r+3] -= sum_c V[c][r..r+3] h[c] over the j columns in ascending c: the
// four rows of a 16-byte (float) or 32-byte (double) vector load per column.
// Element by element this is the same arithmetic as the one-row form.
template <class T>
__device__ __forceinline__ void update_rows4(int j, const T* __restrict__ V, int64_t ldv,
                                             const T* __restrict__ s_h, T* __restrict__ w, int r,
                                             T (&out)[4]) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  v4 wv = *reinterpret_cast<const v4*>(w + r);
  int c = 0;
  for (; c + 8 <= j; c += 8) {
    v4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const v4*>(V + (size_t)(c + u) * ldv + r);
#pragma unroll
    for (int u = 0; u < 8; ++u) wv -= v[u] * s_h[c + u];
  }
  for (; c < j; ++c) wv -= *reinterpret_cast<const v4*>(V + (size_t)c * ldv + r) * s_h[c];
  *reinterpret_cast<v4*>(w + r) = wv;
  out[0] = wv.x;
  out[1] = wv.y;
  out[2] = wv.z;
  out[3] = wv.w;
}

// Whether the four-row vector form applies: V's columns and w aligned to the
// 4-element vector (the solver's own buffers always are; a caller's may not).
template <class T>
__device__ __forceinline__ bool rows4_ok(const T* V, int64_t ldv, const T* w) {
  return ((reinterpret_cast<uintptr_t>(V) | reinterpret_cast<uintptr_t>(w)) & (4 * sizeof(T) - 1)) == 0 &&
         (ldv & 3) == 0;
}

// The same for one row (the rows past the last multiple of 4).
template <class T>
__device__ __forceinline__ T update_row(int j, const T* __restrict__ V, int64_t ldv,
                                        const T* __restrict__ s_h, T* __restrict__ w, int r) {
  T wv = w[r];
  for (int c = 0; c < j; ++c) wv -= V[(size_t)c * ldv + r] * s_h[c];
  w[r] = wv;
  return wv;
}

// Plain update w -= V_j h_in (used when j is too large to fuse).  A thread
// takes four consecutive rows at a time (V columns are 256-byte aligned, so
// every 4-row group is one aligned vector load per column).
template <class T>
__device__ __forceinline__ void cgs_update_body(int n, int j, const T* __restrict__ V,
                                                int64_t ldv, const T* __restrict__ h_in,
                                                T* __restrict__ w,
                                                const int* __restrict__ done, bool rev = false) {
  __shared__ T s_h[kMaxCols];
  if (done && *done) return;
  for (int c = threadIdx.x; c < j; c += kBlock) s_h[c] = h_in[c];
  __syncthreads();
  const int nq = rows4_ok(V, ldv, w) ? n / 4 : 0;
  T o[4];
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < nq; q += gridDim.x * kBlock)
    update_rows4<T>(j, V, ldv, s_h, w, 4 * (rev ? nq - 1 - q : q), o);
  for (int r = 4 * nq + blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock)
    update_row<T>(j, V, ldv, s_h, w, r);
}

template <class T>
__global__ __launch_bounds__(kBlock) void cgs_update_kernel(int n, int j, const T* __restrict__ V,
                                                            int64_t ldv, const T* __restrict__ h_in,
                                                            T* __restrict__ w,
                                                            const int* __restrict__ done, int rev) {
  cgs_update_body<T>(n, j, V, ldv, h_in, w, done, rev != 0);
}

// ---------------------------------------------------------------------------
// Tail of the update+norm pass, run by the last block after beta is known.
// ---------------------------------------------------------------------------
enum TailMode { kTailGivens = 0, kTailStandalone = 1 };

// Givens step on column jc (0-based) and, when the cycle ends, the triangular
// solve R y = g.  The block first stages the new column (h1 + h2, beta) and
// the earlier rotations in LDS with one round of parallel loads; thread 0 then
// does the sequential rotation work on LDS, and the block writes the raw and
// rotated columns back.  The back-substitution is column-oriented.
__device__ __forceinline__ void givens_tail(CycleState cs, int jc, int last_jc, double beta,
                                            double breakdown_thresh) {
  __shared__ int s_finish;
  __shared__ double s_col[kMaxCols + 1];
  __shared__ double s_c[kMaxCols];
  __shared__ double s_s[kMaxCols];
  __shared__ double s_g[kMaxCols + 1];
  __shared__ double s_y;
  const int ldh = cs.ldh;
  const int t = threadIdx.x;
  for (int i = t; i <= jc; i += kBlock) {
    s_col[i] = cs.h1d[i] + cs.h2d[i];
    if (i < jc) {
      s_c[i] = cs.cs[i];
      s_s[i] = cs.sn[i];
    }
  }
  if (t == 0) {
    s_col[jc + 1] = beta;
    s_g[jc] = cs.g[jc];
  }
  __syncthreads();
  double* hraw = cs.Hraw + (size_t)jc * ldh;
  for (int i = t; i < ldh; i += kBlock) hraw[i] = (i <= jc + 1) ? s_col[i] : 0.0;
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < jc; ++i) {
      const double hi = s_col[i], hi1 = s_col[i + 1];
      const double c = s_c[i], s = s_s[i];
      s_col[i] = c * hi + s * hi1;
      s_col[i + 1] = -s * hi + c * hi1;
    }
    const double a = s_col[jc], b = s_col[jc + 1];
    const double rho = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (rho != 0.0) {
      c = a / rho;
      s = b / rho;
    }
    cs.cs[jc] = c;
    cs.sn[jc] = s;
    s_col[jc] = c * a + s * b;
    s_col[jc + 1] = 0.0;
    const double gj = s_g[jc];
    cs.g[jc + 1] = -s * gj;
    cs.g[jc] = c * gj;
    s_g[jc] = c * gj;
    const double res = fabs(s * gj);
    Status* st = cs.st;
    st->res = res;
    const bool brk = !(beta > breakdown_thresh);
    const bool nonfin = !isfinite(res) || !isfinite(beta) || !isfinite(s_col[jc]);
    const bool conv = st->stop_thresh >= 0.0 && res <= st->stop_thresh;
    if (brk) st->breakdown = 1;
    if (nonfin) st->nonfinite = 1;
    const bool finish = brk || nonfin || conv || jc == last_jc;
    if (finish) {
      st->k = jc + 1;
      if (brk || conv || nonfin) st->done = 1;
    }
    *cs.inv_beta = 1.0 / beta;
    s_finish = finish ? 1 : 0;
  }
  __syncthreads();
  double* hcol = cs.H + (size_t)jc * ldh;
  for (int i = t; i < ldh; i += kBlock) hcol[i] = (i <= jc + 1) ? s_col[i] : 0.0;
  if (!s_finish) return;
  const int k = jc + 1;
  for (int i = t; i < jc; i += kBlock) s_g[i] = cs.g[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    if (t == 0) {
      const double rii = (i == jc) ? s_col[jc] : cs.H[(size_t)i * ldh + i];
      const double yi = s_g[i] / rii;
      cs.y[i] = yi;
      s_y = yi;
    }
    __syncthreads();
    const double yi = s_y;
    for (int r = t; r < i; r += kBlock) {
      const double rri = (i == jc) ? s_col[r] : cs.H[(size_t)i * ldh + r];
      s_g[r] -= rri * yi;
    }
    __syncthreads();
  }
}

// Pass-2 update and norm: w -= V_j h_in with the block's partial ||w||^2
// accumulated in the working precision; four rows per thread at a time.
// With rev the row quads are taken in descending order (so that the pass
// starts on the rows the previous pass over V ended on).
template <class T>
__device__ __forceinline__ void cgs_update_norm_body(
    int n, int j, const T* __restrict__ V, int64_t ldv, const T* __restrict__ h_in,
    T* __restrict__ w, double* partial, const int* __restrict__ done, bool rev = false) {
  __shared__ T s_h[kMaxCols];
  if (done && *done) return;
  for (int c = threadIdx.x; c < j; c += kBlock) s_h[c] = h_in[c];
  __syncthreads();
  T sq = T(0);
  const int nq = rows4_ok(V, ldv, w) ? n / 4 : 0;
  T o[4];
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < nq; q += gridDim.x * kBlock) {
    update_rows4<T>(j, V, ldv, s_h, w, 4 * (rev ? nq - 1 - q : q), o);
#pragma unroll
    for (int i = 0; i < 4; ++i) sq += o[i] * o[i];
  }
  for (int r = 4 * nq + blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    const T wv = update_row<T>(j, V, ldv, s_h, w, r);
    sq += wv * wv;
  }
  sq = block_sum(sq);
  if (threadIdx.x == 0) partial[blockIdx.x] = double(sq);
}

template <class T>
__global__ __launch_bounds__(kBlock) void cgs_update_norm_kernel(
    int n, int j, const T* __restrict__ V, int64_t ldv, const T* __restrict__ h_in,
    T* __restrict__ w, double* partial, const int* __restrict__ done, int rev) {
  cgs_update_norm_body<T>(n, j, V, ldv, h_in, w, partial, done, rev != 0);
}

// beta = ||w|| from the partials, then the tail: the Givens step (solver) or
// h = h1 + h2, beta (standalone CGS2).
template <class T, int MODE>
__device__ __forceinline__ void finish_norm_body(int nparts, const double* partial,
                                                 CycleState cs, int j, int last_jc,
                                                 double breakdown_thresh, double* hout,
                                                 const int* __restrict__ done) {
  if (done && *done) return;
  const double s = sum_partials(nparts, partial);
  // beta in the working precision, as the float32 inner solver would have it
  const double beta = double(T(sqrt(double(T(s)))));
  if constexpr (MODE == kTailGivens) {
    givens_tail(cs, j - 1, last_jc, beta, breakdown_thresh);
  } else {
    if (threadIdx.x == 0) *cs.inv_beta = (beta > 0.0) ? 1.0 / beta : 1.0;
    for (int c = threadIdx.x; c < j; c += kBlock) hout[c] = cs.h1d[c] + cs.h2d[c];
    if (threadIdx.x == 0) hout[j] = beta;
  }
}

template <class T, int MODE>
__global__ __launch_bounds__(kBlock) void finish_norm_kernel(int nparts, const double* partial,
                                                             CycleState cs, int j, int last_jc,
                                                             double breakdown_thresh, double* hout,
                                                             const int* __restrict__ done) {
  finish_norm_body<T, MODE>(nparts, partial, cs, j, last_jc, breakdown_thresh, hout, done);
}

// ===========================================================================
// Element-wise kernels
// ===========================================================================
template <class T>
__global__ __launch_bounds__(kBlock) void scale_kernel(int n, const T* __restrict__ x,
                                                       const double* __restrict__ scale,
                                                       T* __restrict__ y,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  const T s = T(*scale);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) y[i] = x[i] * s;
}

// u = V[:, 0:k] y in the working precision (k read from the status), then,
// when x is given, x += gamma * (TO) u; otherwise u is stored.
template <class TI, class TO>
__device__ __forceinline__ void solution_update_body(
    int n, const TI* __restrict__ V, int64_t ldv, const double* __restrict__ y,
    const Status* __restrict__ st, TI* __restrict__ u, TO* __restrict__ x) {
  __shared__ TI s_y[kMaxCols];
  const int k = st->k;
  for (int c = threadIdx.x; c < k; c += kBlock) s_y[c] = TI(y[c]);
  __syncthreads();
  const TO gam = TO(st->gamma);
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    TI s = TI(0);
    for (int c = 0; c < k; ++c) s += V[(size_t)c * ldv + r] * s_y[c];
    if (x) x[r] += gam * TO(s);
    else u[r] = s;
  }
}

template <class TI, class TO>
__global__ __launch_bounds__(kBlock) void solution_update_kernel(
    int n, const TI* __restrict__ V, int64_t ldv, const double* __restrict__ y,
    const Status* __restrict__ st, TI* __restrict__ u, TO* __restrict__ x) {
  solution_update_body<TI, TO>(n, V, ldv, y, st, u, x);
}

// x += gamma * (TO) u
template <class TI, class TO>
__global__ __launch_bounds__(kBlock) void axpy_gamma_kernel(int n, const TI* __restrict__ u,
                                                            const Status* __restrict__ st,
                                                            TO* __restrict__ x) {
  const TO gam = TO(st->gamma);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    x[i] += gam * TO(u[i]);
}

__global__ __launch_bounds__(kBlock) void cast_f64_f32_kernel(int64_t n, const double* __restrict__ in,
                                                              float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    out[i] = float(in[i]);
}

// ===========================================================================
// GMRES polynomial p(A) = (1 - pi(A)) A^{-1}, pi(z) = prod (1 - z/theta_i),
// applied from its Leja-ordered roots (§III-D).  With P the running product
// pi_{i-1}(A) x and Y the running p_{i-1}(A) x:
//   real root, c = 1/theta:          Y += c P ;  P <- P - c A P
//   pair a +- ib, c1 = 2a/|theta|^2, c2 = 1/|theta|^2:
//        T = A P ;  Y += c1 P - c2 T ;  P <- P - (c1 T - c2 A T)
// Each kernel below is one SpMV with the matching update as its epilogue.
// ===========================================================================

// Real root: Y (+)= c P ; P_next = P - c (A P)  (first: Y is not read).
template <class T, bool FIRST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void poly_real_kernel(int n, const int* __restrict__ rp,
                                                           const int* __restrict__ ci,
                                                           const T* __restrict__ val,
                                                           const T* __restrict__ P, T c,
                                                           T* __restrict__ Y, T* __restrict__ Pn,
                                                           const int* __restrict__ done) {
  __shared__ __align__(16) T s_prod[SpmvCfg<T>::kChunk];
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * kSpmvRows;
  T ap[kSpmvRpt];
  if (!spmv_rows<T, false>(n, r0, rp, ci, val, P, T(1), s_prod, ap, done)) return;
#pragma unroll
  for (int i = 0; i < kSpmvRpt; ++i) {
    const int r = r0 + threadIdx.x + i * kBlock;
    if (r < n) {
      const T p = P[r];
      Y[r] = FIRST ? c * p : Y[r] + c * p;
      Pn[r] = p - c * ap[i];
    }
  }
}

// Last real root (no product with A): Y (+)= c P.
template <class T, bool FIRST>
__global__ __launch_bounds__(kBlock) void poly_real_last_kernel(int n, const T* __restrict__ P,
                                                                T c, T* __restrict__ Y,
                                                                const int* __restrict__ done) {
  if (done && *done) return;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    Y[i] = FIRST ? c * P[i] : Y[i] + c * P[i];
}

// Pair, first half: Tt = A P ; Y (+)= c1 P - c2 Tt.
template <class T, bool FIRST>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void poly_pair1_kernel(int n, const int* __restrict__ rp,
                                                            const int* __restrict__ ci,
                                                            const T* __restrict__ val,
                                                            const T* __restrict__ P, T c1, T c2,
                                                            T* __restrict__ Y, T* __restrict__ Tt,
                                                            const int* __restrict__ done) {
  __shared__ __align__(16) T s_prod[SpmvCfg<T>::kChunk];
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * kSpmvRows;
  T t[kSpmvRpt];
  if (!spmv_rows<T, false>(n, r0, rp, ci, val, P, T(1), s_prod, t, done)) return;
#pragma unroll
  for (int i = 0; i < kSpmvRpt; ++i) {
    const int r = r0 + threadIdx.x + i * kBlock;
    if (r < n) {
      const T p = P[r];
      Tt[r] = t[i];
      const T inc = c1 * p - c2 * t[i];
      Y[r] = FIRST ? inc : Y[r] + inc;
    }
  }
}

// Pair, second half: P_next = P - (c1 Tt - c2 A Tt).
template <class T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void poly_pair2_kernel(int n, const int* __restrict__ rp,
                                                            const int* __restrict__ ci,
                                                            const T* __restrict__ val,
                                                            const T* __restrict__ P,
                                                            const T* __restrict__ Tt, T c1, T c2,
                                                            T* __restrict__ Pn,
                                                            const int* __restrict__ done) {
  __shared__ __align__(16) T s_prod[SpmvCfg<T>::kChunk];
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * kSpmvRows;
  T at[kSpmvRpt];
  if (!spmv_rows<T, false>(n, r0, rp, ci, val, Tt, T(1), s_prod, at, done)) return;
#pragma unroll
  for (int i = 0; i < kSpmvRpt; ++i) {
    const int r = r0 + threadIdx.x + i * kBlock;
    if (r < n) Pn[r] = P[r] - (c1 * Tt[r] - c2 * at[i]);
  }
}

// ===========================================================================
// Persistent single-block cycle for small systems
// ===========================================================================
// Largest n run as one block per cycle.  Measured on the 2D Laplacian,
// GMRES(50): the single block is 2-4x faster than the multi-kernel cycle at
// n = 144, 1.3x at n = 576, even at n = 1024, and 3x slower at n = 4096, where
// four waves cannot hide the latency of the block's serial SpMV chunks.
constexpr int kSmallMaxN = 1024;

// Column sums of the single block's CGS partials: out = partial[c][0].
template <class T>
__device__ __forceinline__ void take_cols(int j, const double* __restrict__ partial, double* out,
                                          T* outT) {
  for (int c = threadIdx.x; c < j; c += kBlock) {
    const double s = partial[(size_t)c * kPartPitch];
    out[c] = s;
    outT[c] = T(s);
  }
}

// The three CGS2 passes on w against the j columns of V, the update+dots pass
// fused up to 64 columns, as the multi-kernel path does.
template <class T>
__device__ __forceinline__ void small_cgs2(int n, int j, const T* V, int64_t ldv, T* w, double* partial,
                                           CycleState cs, T* h1t, T* h2t, int last_jc, double thresh) {
  if (j <= 8) cgs_dots_body<T, 8, 1>(n, j, V, ldv, w, partial, nullptr);
  else if (j <= 16) cgs_dots_body<T, 16, 1>(n, j, V, ldv, w, partial, nullptr);
  else if (j <= 32) cgs_dots_body<T, 32, 1>(n, j, V, ldv, w, partial, nullptr);
  else if (j <= 64) cgs_dots_body<T, 64, 1>(n, j, V, ldv, w, partial, nullptr);
  else if (j <= 256) cgs_dots_body<T, 64, 4>(n, j, V, ldv, w, partial, nullptr);
  else cgs_dots_body<T, 64, 8>(n, j, V, ldv, w, partial, nullptr);
  __syncthreads();
  take_cols<T>(j, partial, cs.h1d, h1t);
  __syncthreads();
  if (j <= 8) cgs_update_dots_body<T, 8>(n, j, V, ldv, h1t, w, partial, nullptr);
  else if (j <= 16) cgs_update_dots_body<T, 16>(n, j, V, ldv, h1t, w, partial, nullptr);
  else if (j <= 32) cgs_update_dots_body<T, 32>(n, j, V, ldv, h1t, w, partial, nullptr);
  else if (j <= 64) cgs_update_dots_body<T, 64>(n, j, V, ldv, h1t, w, partial, nullptr);
  else {
    cgs_update_body<T>(n, j, V, ldv, h1t, w, nullptr);
    __syncthreads();
    if (j <= 256) cgs_dots_body<T, 64, 4>(n, j, V, ldv, w, partial, nullptr);
    else cgs_dots_body<T, 64, 8>(n, j, V, ldv, w, partial, nullptr);
  }
  __syncthreads();
  take_cols<T>(j, partial, cs.h2d, h2t);
  __syncthreads();
  cgs_update_norm_body<T>(n, j, V, ldv, h2t, w, partial, nullptr);
  __syncthreads();
  finish_norm_body<T, kTailGivens>(1, partial, cs, j, last_jc, thresh, nullptr, nullptr);
  __syncthreads();
}

// One whole restart cycle in one block of 256 threads: the cast of r, up to
// mc inner iterations (SpMV with the fused normalisation, CGS2, the float64
// Givens step), the solution update and the next residual with its norm.  The
// device steps are those of the multi-kernel cycle, with block barriers where
// that path has kernel boundaries; for a small system this replaces some 8
// launches per iteration by one launch per cycle.  Launched as <<<1, kBlock>>>.
template <class TI, class TO>
__global__ __launch_bounds__(kBlock) void small_cycle_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const TI* __restrict__ vin,
    const int* __restrict__ rpo, const int* __restrict__ cio, const TO* __restrict__ vout,
    const TO* __restrict__ b, TO* __restrict__ x, TO* __restrict__ r, TI* V,
    int64_t ldv, TI* w0, TI* w1, CycleState cs, double* partial, TI* h1t, TI* h2t, int mc, double stop_rel,
    double thresh) {
  // passes of 2048 entries keep the single block's LDS within 160 KB
  constexpr int kSmallChunk = 2048;
  __shared__ __align__(16) TI s_pi[kSmallChunk];
  __shared__ __align__(16) TO s_po[kSmallChunk];
  Status* st = cs.st;
  start_cycle_body<TO, TI>(n, r, w0, partial, st);
  __syncthreads();
  finish_start_cycle_body<TI>(1, partial, cs, stop_rel);
  __syncthreads();
  TI* wc = w0;  // the current w (the unnormalised v_j)
  TI* wn = w1;  // A v_j
  __shared__ int s_done;
  for (int j = 0; j < mc; ++j) {
    // implicit convergence or breakdown: one thread reads the flag and the
    // block takes the same branch
    if (threadIdx.x == 0) s_done = st->done;
    __syncthreads();
    if (s_done) break;
    TI* vj = V + (size_t)j * ldv;
    const TI s = TI(*cs.inv_beta);
    for (int r0 = 0; r0 < n; r0 += kSpmvRows) {
      TI acc[kSpmvRpt];
      spmv_rows<TI, true, kSmallChunk>(n, r0, rp, ci, vin, wc, s, s_pi, acc);
#pragma unroll
      for (int i = 0; i < kSpmvRpt; ++i) {
        const int row = r0 + threadIdx.x + i * kBlock;
        if (row < n) {
          vj[row] = wc[row] * s;
          wn[row] = acc[i];
        }
      }
    }
    __syncthreads();  // wn and vj complete before the CGS2 passes read them
    small_cgs2<TI>(n, j + 1, V, ldv, wn, partial, cs, h1t, h2t, mc - 1, thresh);
    TI* t = wc;
    wc = wn;
    wn = t;
  }
  solution_update_body<TI, TO>(n, V, ldv, cs.y, st, nullptr, x);
  __syncthreads();
  double sq = 0.0;
  for (int r0 = 0; r0 < n; r0 += kSpmvRows) {
    TO acc[kSpmvRpt];
    spmv_rows<TO, false, kSmallChunk>(n, r0, rpo, cio, vout, x, TO(1), s_po, acc);
#pragma unroll
    for (int i = 0; i < kSpmvRpt; ++i) {
      const int row = r0 + threadIdx.x + i * kBlock;
      if (row < n) {
        const TO rv = b[row] - acc[i];
        r[row] = rv;
        sq += double(rv) * double(rv);
      }
    }
  }
  sq = block_sum(sq);
  if (threadIdx.x == 0) {
    const double g = sqrt(sq);
    st->gamma = g;
    st->inv_gamma = 1.0 / g;
  }
}

// ===========================================================================
// Cooperative multi-block cycle for mid-size systems
// ===========================================================================
// Above kSmallMaxN one block cannot hide the latency of a whole cycle, while
// the multi-kernel cycle pays about eight launches per iteration.  Here a
// cooperative launch of G co-resident blocks runs the whole restart cycle, with
// grid barriers where the multi-kernel cycle has kernel boundaries that carry
// data between blocks: three per inner iteration of GMRES-IR, four for plain
// GMRES (one more beyond 64 basis columns, where the first update and the
// second dots run apart).
// Above about 6000 rows the grid barriers cost more than the launches they
// replace (n = 9216: 34.7 ms per GMRES-IR solve against 29.3 for the
// multi-kernel cycle).
constexpr int kCoopMaxN = 6144;
constexpr int kCoopMaxBlocks = 64;
// Column partials of consecutive CGS passes alternate between two halves of
// each column's pitch, so a block may write the next pass's partials while a
// slower one still reads the previous pass's.
constexpr int kCoopAlt = kPartPitch / 2;
static_assert(kCoopMaxBlocks <= kCoopAlt, "partials of one pass must fit half a column pitch");

// Grid-wide barrier on device-scope vector atomics.  After the block barrier,
// thread 0 of each block counts itself in with a release add, which makes the
// block's writes visible at device scope.  The last to arrive takes an acquire
// fence, resets the count and publishes the next generation with a release
// store; the others poll the generation with relaxed loads and take a single
// acquire fence once it has moved (an acquire on every poll would invalidate
// the caches on every probe).  All blocks of a cooperative launch are
// resident, so every wait ends; a wait that has not ended after about a second
// gives up, flags barrier_timeout and lets the kernel run to its end, so a
// broken barrier cannot hang the device.
// Thread 0: count the block in; the last to arrive publishes generation g+1.
// Returns whether this block was the last.
__device__ __forceinline__ bool grid_arrive(GridBarrier* bar, unsigned int g) {
  const unsigned int arrived =
      __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  if (arrived != gridDim.x - 1) return false;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&bar->gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

// Thread 0: wait until generation g has passed (bounded).
__device__ __forceinline__ void grid_wait(GridBarrier* bar, unsigned int g, Status* st) {
  int spins = 0;
  while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > (1 << 24)) {
      __hip_atomic_store(&st->barrier_timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void grid_sync(GridBarrier* bar, unsigned int& gen, Status* st) {
  __syncthreads();
  if (threadIdx.x == 0 && !grid_arrive(bar, gen)) grid_wait(bar, gen, st);
  gen += 1;
  __syncthreads();
}

// grid_sync in which block 0 runs work0 (with all its threads) after it has
// arrived and before it waits, so that work no other block needs before a
// later barrier overlaps the wait instead of delaying block 0's arrival.
// work0's writes are published by the next barrier.
template <class F>
__device__ __forceinline__ void grid_sync_then(GridBarrier* bar, unsigned int& gen, Status* st, F&& work0) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) s_last = grid_arrive(bar, gen) ? 1 : 0;
  __syncthreads();
  if (blockIdx.x == 0) work0();
  if (threadIdx.x == 0 && !s_last) grid_wait(bar, gen, st);
  gen += 1;
  __syncthreads();
}

// Column sums of the G block partials of a CGS pass, added in block order:
// every block keeps them (in the inner precision) in LDS, block 0 also stores
// the float64 sums for the Givens step.
template <class T>
__device__ __forceinline__ void coop_take_cols(int j, int G, const double* __restrict__ part, double* out_d,
                                               T* s_out) {
  for (int c = threadIdx.x; c < j; c += kBlock) {
    double s = 0.0;
    for (int b = 0; b < G; ++b) s += part[(size_t)c * kPartPitch + b];
    s_out[c] = T(s);
    if (blockIdx.x == 0) out_d[c] = s;
  }
}

// beta of the latest column from the norm partials, as the Givens step
// computes it (same partial sum, same roundings), so every block has it.
template <class T>
__device__ __forceinline__ double coop_beta(int G, const double* __restrict__ part) {
  __shared__ double s_b;
  const double s = sum_partials(G, part);
  if (threadIdx.x == 0) s_b = double(T(sqrt(double(T(s)))));
  __syncthreads();
  return s_b;
}

// One whole restart cycle on G = gridDim.x co-resident blocks (cooperative
// launch): the cast of r, up to mc inner iterations, the solution update and
// the next residual with its norm.  Per iteration: the SpMV | CGS2 dots |
// barrier | update + dots | barrier | update + norm | barrier; every block
// then takes beta from the norm partials and goes on with the next SpMV;
// block 0 runs the float64 Givens step first (plain GMRES) or inside the next
// iteration's first barrier (GMRES-IR).  The SpMV walks 256-row groups, one
// row per thread, so a block's SpMV rows are exactly the rows its waves take
// in the dots and the fused update + dots, and no barrier separates them.
// Only when the Givens step may end the cycle early (the implicit residual
// test of plain GMRES) does a barrier follow the SpMV, after which every block
// reads block 0's flags; without it (GMRES-IR) the only early end is a
// breakdown, which every block sees in beta.  Sums of block partials are
// added in block order (deterministic).
template <class TI, class TO>
__global__ __launch_bounds__(kBlock) void coop_cycle_kernel(
    int n, const int* __restrict__ rp, const int* __restrict__ ci, const TI* __restrict__ vin,
    const int* __restrict__ rpo, const int* __restrict__ cio, const TO* __restrict__ vout,
    const TO* __restrict__ b, TO* __restrict__ x, TO* __restrict__ r, TI* V,
    int64_t ldv, TI* w0, TI* w1, CycleState cs, double* partial, GridBarrier* bar, int mc, double stop_rel,
    double thresh) {
  // passes of 1024 entries keep the block's LDS (with the CGS bodies') within 160 KB
  constexpr int kChunk = 1024;
  __shared__ __align__(16) TI s_pi[kChunk];
  __shared__ __align__(16) TO s_po[kChunk];
  __shared__ TI s_h[kMaxCols];
  __shared__ int s_done;
  Status* st = cs.st;
  const int G = gridDim.x;
  double* partA = partial;
  double* partB = partial + kCoopAlt;
  unsigned int gen = 0;
  start_cycle_body<TO, TI>(n, r, w0, partA, st);
  grid_sync(bar, gen, st);
  double inv_beta;
  {
    __shared__ double s_ib0;
    const double s = sum_partials(G, partA);
    if (threadIdx.x == 0) s_ib0 = 1.0 / sqrt(double(TI(s)));
    __syncthreads();
    inv_beta = s_ib0;
  }
  if (blockIdx.x == 0) finish_start_cycle_body<TI>(G, partA, cs, stop_rel);
  const bool implicit_stop = stop_rel >= 0.0;
  TI* wc = w0;  // the current w (the unnormalised v_j)
  TI* wn = w1;  // A v_j
  // Without the implicit residual test no block reads the Givens step before
  // the cycle ends: block 0 then runs column j's step while it waits at the
  // next iteration's first barrier (same steps, same order, same results).
  int pend_jc = -1;
  double pend_beta = 0.0;
  for (int j = 0; j < mc; ++j) {
    TI* vj = V + (size_t)j * ldv;
    const TI s = TI(inv_beta);
    for (int r0 = blockIdx.x * kBlock; r0 < n; r0 += G * kBlock) {
      TI acc[1];
      spmv_rows<TI, true, kChunk, 1>(n, r0, rp, ci, vin, wc, s, s_pi, acc);
      const int row = r0 + threadIdx.x;
      if (row < n) {
        vj[row] = wc[row] * s;
        wn[row] = acc[0];
      }
    }
    if (implicit_stop) {
      grid_sync(bar, gen, st);
      // block 0's Givens step of the previous column is complete: the cycle may be over
      if (threadIdx.x == 0) s_done = st->done || st->barrier_timeout;
      __syncthreads();
      if (s_done) break;
    } else {
      __syncthreads();  // the block's own rows of w and v_j, read next by its own waves
    }
    const int jj = j + 1;  // basis columns
    if (jj <= 8) cgs_dots_body<TI, 8, 1>(n, jj, V, ldv, wn, partA, nullptr);
    else if (jj <= 16) cgs_dots_body<TI, 16, 1>(n, jj, V, ldv, wn, partA, nullptr);
    else if (jj <= 32) cgs_dots_body<TI, 32, 1>(n, jj, V, ldv, wn, partA, nullptr);
    else if (jj <= 64) cgs_dots_body<TI, 64, 1>(n, jj, V, ldv, wn, partA, nullptr);
    else if (jj <= 256) cgs_dots_body<TI, 64, 4>(n, jj, V, ldv, wn, partA, nullptr);
    else cgs_dots_body<TI, 64, 8>(n, jj, V, ldv, wn, partA, nullptr);
    if (pend_jc >= 0) {
      grid_sync_then(bar, gen, st, [&] { givens_tail(cs, pend_jc, mc - 1, pend_beta, thresh); });
      pend_jc = -1;
    } else {
      grid_sync(bar, gen, st);
    }
    coop_take_cols<TI>(jj, G, partA, cs.h1d, s_h);
    __syncthreads();
    if (jj <= 8) cgs_update_dots_body<TI, 8>(n, jj, V, ldv, s_h, wn, partB, nullptr);
    else if (jj <= 16) cgs_update_dots_body<TI, 16>(n, jj, V, ldv, s_h, wn, partB, nullptr);
    else if (jj <= 32) cgs_update_dots_body<TI, 32>(n, jj, V, ldv, s_h, wn, partB, nullptr);
    else if (jj <= 64) cgs_update_dots_body<TI, 64>(n, jj, V, ldv, s_h, wn, partB, nullptr);
    else {
      // the update walks rows four per thread, the dots a row per lane: the
      // rows change hands between blocks, so a grid barrier separates them
      cgs_update_body<TI>(n, jj, V, ldv, s_h, wn, nullptr);
      grid_sync(bar, gen, st);
      if (jj <= 256) cgs_dots_body<TI, 64, 4>(n, jj, V, ldv, wn, partB, nullptr);
      else cgs_dots_body<TI, 64, 8>(n, jj, V, ldv, wn, partB, nullptr);
    }
    grid_sync(bar, gen, st);
    coop_take_cols<TI>(jj, G, partB, cs.h2d, s_h);
    __syncthreads();
    cgs_update_norm_body<TI>(n, jj, V, ldv, s_h, wn, partA, nullptr);
    grid_sync(bar, gen, st);
    const double beta = coop_beta<TI>(G, partA);
    inv_beta = 1.0 / beta;
    if (implicit_stop) {
      if (blockIdx.x == 0) finish_norm_body<TI, kTailGivens>(G, partA, cs, jj, mc - 1, thresh, nullptr, nullptr);
    } else {
      pend_jc = jj - 1;
      pend_beta = beta;
    }
    // a breakdown ends the cycle here in every block (the Givens step flags it too)
    if (!implicit_stop && !(beta > thresh && isfinite(beta))) break;
    TI* t = wc;
    wc = wn;
    wn = t;
  }
  // y and k of block 0's last Givens step
  if (pend_jc >= 0 && blockIdx.x == 0) givens_tail(cs, pend_jc, mc - 1, pend_beta, thresh);
  grid_sync(bar, gen, st);
  solution_update_body<TI, TO>(n, V, ldv, cs.y, st, nullptr, x);
  grid_sync(bar, gen, st);
  double sq = 0.0;
  for (int r0 = blockIdx.x * kSpmvRows; r0 < n; r0 += G * kSpmvRows) {
    TO acc[kSpmvRpt];
    spmv_rows<TO, false, kChunk>(n, r0, rpo, cio, vout, x, TO(1), s_po, acc);
#pragma unroll
    for (int i = 0; i < kSpmvRpt; ++i) {
      const int row = r0 + threadIdx.x + i * kBlock;
      if (row < n) {
        const TO rv = b[row] - acc[i];
        r[row] = rv;
        sq += double(rv) * double(rv);
      }
    }
  }
  sq = block_sum(sq);
  if (threadIdx.x == 0) partA[blockIdx.x] = sq;
  grid_sync(bar, gen, st);
  if (blockIdx.x == 0) {
    const double g = sqrt(sum_partials(G, partA));
    if (threadIdx.x == 0) {
      st->gamma = g;
      st->inv_gamma = 1.0 / g;
    }
  }
}

__global__ void coop_reset_kernel(GridBarrier* bar, Status* st) {
  if (threadIdx.x == 0) {
    bar->count = 0;
    bar->gen = 0;
    st->barrier_timeout = 0;
  }
}

}  // namespace gmr
