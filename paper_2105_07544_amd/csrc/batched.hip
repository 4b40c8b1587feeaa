// Batched block GMRES(m)-IR: many independent sparse systems, each with P = 16
// right-hand sides, solved together.
//
// The paper's solver handles one right-hand side (§IV).  Here every system's
// P right-hand sides share one block Krylov space: the new block W = A V_j is
// orthogonalised against the earlier blocks by two block classical
// Gram-Schmidt passes (the block form of the CGS2 of §III-A) and within itself
// by Cholesky QR done twice.  The block Gram-Schmidt products V^T W and V C
// are dense contractions of shape (16 j x rows) x (rows x 16) and
// (rows x 16 j) x (16 j x 16); they run on the matrix cores
// (v_mfma_f32_16x16x4f32 with FP32 accumulation for the float32 inner solve,
// v_mfma_f64_16x16x4f64 for the float64 one).  The outer loop is GMRES-IR
// (Alg. 2) per system: float64 block residual B - A X, every column scaled by
// its own residual norm, float64 update of X.  With a float64 inner solve the
// same loop is plain restarted block GMRES(m) in float64, the baseline the
// mixed-precision solve is compared with.  The block least-squares problem is
// solved per system in float64 with block Householder reflectors.
//
// Work is described by a tile table: every system's rows are cut into tiles
// of at most `tile_rows` rows; a kernel launch covers all tiles of all
// systems and skips the systems that are converged or have broken down in the
// current cycle.  Multivectors are row-major with 16 columns (64 bytes per
// row), which is exactly the operand layout the 16x16x4 MFMA wants.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/gmres_ir.h"
#include "device_common.hpp"
#include "host_common.hpp"

namespace gmr {
namespace bat {

constexpr int P = 16;          // right-hand sides per system = block size
constexpr int PP = P * P;      // entries of a 16 x 16 block
constexpr int kMaxBlocks = 65; // restart m <= 64 block steps
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// The 16x16x4 matrix-core step for the inner precision T.  Operand A: lane l
// holds A[l%16][l/16]; operand B: lane l holds B[l/16][l%16]; element q of the
// result in lane l is D[row(l/16, q)][l%16] (the two instructions order the
// result rows differently).
template <class T> struct Mx;
template <> struct Mx<float> {
  typedef floatx4 v4;
  static __device__ __forceinline__ v4 mfma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int q) { return 4 * g + q; }
};
template <> struct Mx<double> {
  typedef doublex4 v4;
  static __device__ __forceinline__ v4 mfma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int q) { return 4 * q + g; }
};

struct BTile { int sys, r0, nr, pad; };
struct BSys { int row_off, n, tile_start, tile_count; };
struct BState {
  int active;      // some column still above the tolerance (0 once the system failed)
  int cycle_done;  // the current cycle ended (after a block breakdown)
  int kblk;        // block columns completed in the current cycle
  int failed;      // the start block could not be formed: the system is frozen
  int brk;         // the current block column broke down: it is the cycle's last
  int pad;
};
// The state array has nsys + 1 entries: entry nsys is an idle system that is
// never active.  Tiles past the current table's end belong to it, so a launch
// of a fixed grid runs whatever the table holds and the rest exit at once.

// A system whose block step is in progress.
__device__ __forceinline__ bool running(const BState& s) { return s.active && !s.cycle_done && !s.brk; }

// ---------------------------------------------------------------------------
// Tile table of the active systems, built on the device at the start of every
// restart cycle, so that a captured cycle replays with the table its cycle
// needs (the same table an eager cycle builds, hence the same bits).  Tiles
// have tile_rows rows, halved (to multiples of 16, down to min_rows) while the
// active systems give fewer than `fill` tiles; system s owns tiles
// [tile_start, tile_start + tile_count) in system order.  Entries from the
// table's end up to `grid` (the fixed launch grid) are idle tiles of system
// nsys.  A table longer than `grid` (excluded by the bound the host puts on
// `grid`) sets failed on the idle system instead.  One block of kBlock threads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void btiles_kernel(int nsys, BSys* __restrict__ sys, BState* st,
                                                        int tile_rows, int min_rows, int fill, int grid,
                                                        BTile* __restrict__ tiles) {
  __shared__ int s_part[kBlock];
  __shared__ int s_total;
  const int t = threadIdx.x;
  const int per = (nsys + kBlock - 1) / kBlock;  // a contiguous share of systems per thread
  const int s0 = min(nsys, t * per);
  const int s1 = min(nsys, s0 + per);
  int tr = tile_rows;
  int total = 0;
  for (;;) {
    int c = 0;
    for (int s = s0; s < s1; ++s)
      if (st[s].active) c += (sys[s].n + tr - 1) / tr;
    s_part[t] = c;
    __syncthreads();
    if (t == 0) {
      int sum = 0;
      for (int i = 0; i < kBlock; ++i) sum += s_part[i];
      s_total = sum;
    }
    __syncthreads();
    total = s_total;
    __syncthreads();
    if (tr > min_rows && total < fill) tr = max(min_rows, tr / 2 / 16 * 16);
    else break;
  }
  if (total > grid) {
    if (t == 0) st[nsys].failed = 1;
    return;
  }
  int c = 0;
  for (int s = s0; s < s1; ++s)
    if (st[s].active) c += (sys[s].n + tr - 1) / tr;
  s_part[t] = c;
  __syncthreads();
  if (t == 0) {  // exclusive scan of the per-thread counts
    int acc = 0;
    for (int i = 0; i < kBlock; ++i) {
      const int v = s_part[i];
      s_part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int at = s_part[t];
  for (int s = s0; s < s1; ++s) {
    const int n = sys[s].n;
    const int cnt = st[s].active ? (n + tr - 1) / tr : 0;
    sys[s].tile_start = at;
    sys[s].tile_count = cnt;
    for (int i = 0; i < cnt; ++i) tiles[at + i] = BTile{s, sys[s].row_off + i * tr, min(tr, n - i * tr), 0};
    at += cnt;
  }
  for (int i = total + t; i < grid; i += kBlock) tiles[i] = BTile{nsys, 0, 0, 0};
}

// ---------------------------------------------------------------------------
// SpMM in the inner precision: Y = A X for the tiles of running systems.  16 lanes per
// row (one per right-hand side), 16 rows per block pass, nonzeros in ascending k.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(kBlock) void bspmm_kernel(const BTile* __restrict__ tiles,
                                                       const BState* __restrict__ st,
                                                       const int* __restrict__ rp,
                                                       const int* __restrict__ ci,
                                                       const T* __restrict__ val,
                                                       const T* __restrict__ X,
                                                       T* __restrict__ Y) {
  const BTile tl = tiles[blockIdx.x];
  if (!running(st[tl.sys])) return;
  const int c = threadIdx.x % P;
  const int rs = threadIdx.x / P;
  const int rend = tl.r0 + tl.nr;
  // RU rows per thread at a time.  The 16 lanes of a row load KU of its
  // (index, value) pairs with one load each and pass them to each other with
  // lane shuffles, so each nonzero costs one memory instruction (the gather of
  // its X row) instead of three; every row is still summed in ascending k.
  constexpr int RU = 4, KU = 8, RS = kBlock / P;
  const int gbase = threadIdx.x % kWave - c;  // first lane of this row's 16-lane group
  for (int r = tl.r0 + rs; r < rend; r += RU * RS) {
    int k0[RU], len[RU];
    int kmax = 0;
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int rr = r + u * RS;
      k0[u] = rr < rend ? rp[rr] : 0;
      len[u] = rr < rend ? rp[rr + 1] - k0[u] : 0;
      kmax = max(kmax, len[u]);
    }
    T acc[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) acc[u] = T(0);
    for (int o = 0; o < kmax; o += KU) {
      int myc[RU];
      T myv[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const bool in = c < KU && o + c < len[u];
        myc[u] = in ? ci[k0[u] + o + c] : 0;
        myv[u] = in ? val[k0[u] + o + c] : T(0);
      }
      T xv[RU][KU], av[RU][KU];
#pragma unroll
      for (int t = 0; t < KU; ++t)
#pragma unroll
        for (int u = 0; u < RU; ++u) {
          const int col = __shfl(myc[u], gbase + t, kWave);
          av[u][t] = __shfl(myv[u], gbase + t, kWave);
          xv[u][t] = (o + t < len[u]) ? X[(size_t)col * P + c] : T(0);
        }
#pragma unroll
      for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int t = 0; t < KU; ++t)
          if (o + t < len[u]) acc[u] += av[u][t] * xv[u][t];
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int rr = r + u * RS;
      if (rr < rend) Y[(size_t)rr * P + c] = acc[u];
    }
  }
}

// Float64 block residual R = B - A X (X may be null: R = B) with per-tile,
// per-column partial sums of squares in rpart[tile * 16 + c].
__global__ __launch_bounds__(kBlock) void bresidual_kernel(const BTile* __restrict__ tiles,
                                                           const BState* __restrict__ st,
                                                           const int* __restrict__ rp,
                                                           const int* __restrict__ ci,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ X,
                                                           const double* __restrict__ B,
                                                           double* __restrict__ R,
                                                           double* __restrict__ rpart) {
  __shared__ double s_sq[kBlock];
  const BTile tl = tiles[blockIdx.x];
  if (st && !st[tl.sys].active) return;
  const int c = threadIdx.x % P;
  const int rs = threadIdx.x / P;
  const int rend = tl.r0 + tl.nr;
  double sq = 0.0;
  for (int r = tl.r0 + rs; r < rend; r += kBlock / P) {
    double acc = 0.0;
    if (X) {
      const int k1 = rp[r + 1];
      for (int k = rp[r]; k < k1; ++k) acc += val[k] * X[(size_t)ci[k] * P + c];
    }
    const double rv = B[(size_t)r * P + c] - acc;
    R[(size_t)r * P + c] = rv;
    sq += rv * rv;
  }
  s_sq[threadIdx.x] = sq;
  __syncthreads();
  if (threadIdx.x < P) {
    double s = 0.0;
    for (int g = 0; g < kBlock / P; ++g) s += s_sq[g * P + threadIdx.x];
    rpart[(size_t)blockIdx.x * P + threadIdx.x] = s;
  }
}

// Per system: the column norms from the tile partials (fixed order).
// mode 0: bnorm = ||B||; mode 1: gam = ||R||, active = some column above tol.
__global__ void bfinish_res_kernel(int nsys, const BSys* __restrict__ sys, BState* st,
                                   const double* __restrict__ rpart, double* gam, double* bnorm,
                                   double tol, int mode) {
  const int s = blockIdx.x;
  if (s >= nsys) return;
  if (mode == 1 && !st[s].active) return;
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  if (threadIdx.x < P) {
    const int c = threadIdx.x;
    double sum = 0.0;
    for (int t = 0; t < sys[s].tile_count; ++t) sum += rpart[(size_t)(sys[s].tile_start + t) * P + c];
    const double nrm = sqrt(sum);
    if (mode == 0) {
      bnorm[s * P + c] = nrm;
    } else {
      gam[s * P + c] = nrm;
      const double bn = bnorm[s * P + c];
      if (bn > 0.0 && !(nrm <= tol * bn)) atomicOr(&s_any, 1);
    }
  }
  __syncthreads();
  if (mode == 1 && threadIdx.x == 0) st[s].active = s_any;
}

// Start of a cycle: W = T(R / gamma_c) per column (0 for a column with gamma 0).
template <class T>
__global__ __launch_bounds__(kBlock) void bstart_kernel(const BTile* __restrict__ tiles,
                                                        const BState* __restrict__ st,
                                                        const double* __restrict__ R,
                                                        const double* __restrict__ gam,
                                                        T* __restrict__ W) {
  const BTile tl = tiles[blockIdx.x];
  if (!running(st[tl.sys])) return;
  const int c = threadIdx.x % P;
  const double g = gam[tl.sys * P + c];
  const double ig = g > 0.0 ? 1.0 / g : 0.0;
  for (int r = tl.r0 + (int)threadIdx.x / P; r < tl.r0 + tl.nr; r += kBlock / P)
    W[(size_t)r * P + c] = T(R[(size_t)r * P + c] * ig);
}

// ---------------------------------------------------------------------------
// Block dots on the matrix cores: for the tile's rows, C_b = V_b^T W for the
// nblk blocks V_b (b = 0..nblk-1), 16 x 16 each, into
// partial[tile][b][i * 16 + c].  Operand A of one MFMA is V_b^T restricted to
// 4 rows (lane l holds V_b[r + l/16][l % 16]), operand B is W on the same 4
// rows (lane l holds W[r + l/16][l % 16]): both are one contiguous 256-byte
// load.  The row sum is the MFMA's K accumulation; GB blocks are accumulated
// per pass over the rows.
// ---------------------------------------------------------------------------
template <class T, int GB>
__global__ __launch_bounds__(kBlock) void bdots_kernel(const BTile* __restrict__ tiles,
                                                       const BState* __restrict__ st,
                                                       const T* __restrict__ V,
                                                       size_t vstride, int nblk,
                                                       const T* __restrict__ W,
                                                       T* __restrict__ partial,
                                                       size_t pstride) {
  typedef typename Mx<T>::v4 v4;
  __shared__ T s_acc[kWavesPerBlock][GB][PP];
  const BTile tl = tiles[blockIdx.x];
  if (!running(st[tl.sys])) return;
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int rsub = lane / P;
  const int col = lane % P;
  const int rend = tl.r0 + tl.nr;
  for (int g0 = 0; g0 < nblk; g0 += GB) {
    v4 acc[GB];
#pragma unroll
    for (int b = 0; b < GB; ++b) acc[b] = v4{T(0), T(0), T(0), T(0)};
    // two 4-row slices per iteration (rows r .. r+3 and r+4 .. r+7), so that
    // 2 (GB + 1) loads are in flight per lane
    for (int r = tl.r0 + 8 * wave; r < rend; r += 8 * kWavesPerBlock) {
      const int row0 = r + rsub;
      const int row1 = r + 4 + rsub;
      const bool ok0 = row0 < rend;
      const bool ok1 = row1 < rend;
      const T bw0 = ok0 ? W[(size_t)row0 * P + col] : T(0);
      const T bw1 = ok1 ? W[(size_t)row1 * P + col] : T(0);
      T a0[GB], a1[GB];
#pragma unroll
      for (int b = 0; b < GB; ++b) {
        const T* Vb = V + (size_t)(g0 + b) * vstride;
        a0[b] = (ok0 && g0 + b < nblk) ? Vb[(size_t)row0 * P + col] : T(0);
        a1[b] = (ok1 && g0 + b < nblk) ? Vb[(size_t)row1 * P + col] : T(0);
      }
#pragma unroll
      for (int b = 0; b < GB; ++b)
        if (g0 + b < nblk) {
          acc[b] = Mx<T>::mfma(a0[b], bw0, acc[b]);
          acc[b] = Mx<T>::mfma(a1[b], bw1, acc[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < GB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) s_acc[wave][b][Mx<T>::row(rsub, q) * P + col] = acc[b][q];
    __syncthreads();
    for (int b = 0; b < GB && g0 + b < nblk; ++b) {
      const int e = threadIdx.x;
      T sum = s_acc[0][b][e];
#pragma unroll
      for (int w = 1; w < kWavesPerBlock; ++w) sum += s_acc[w][b][e];
      partial[(size_t)blockIdx.x * pstride + (size_t)(g0 + b) * PP + e] = sum;
    }
    __syncthreads();
  }
}

// The same products with the blocks split over the waves instead of the rows:
// wave w accumulates blocks w*WB .. w*WB+WB-1 (then the next 4*WB) over all
// rows of the tile, SL 4-row slices per iteration, and writes its 16 x 16
// results straight from the accumulators to the tile's partials, so there is
// no cross-wave reduction and no LDS.  The four waves walk the same rows, so
// the W rows they share are L1 hits after the first.
template <class T, int WB, int SL>
__global__ __launch_bounds__(kBlock) void bdots_w_kernel(const BTile* __restrict__ tiles,
                                                         const BState* __restrict__ st,
                                                         const T* __restrict__ V, size_t vstride,
                                                         int nblk, const T* __restrict__ W,
                                                         T* __restrict__ partial, size_t pstride) {
  typedef typename Mx<T>::v4 v4;
  const BTile tl = tiles[blockIdx.x];
  if (!running(st[tl.sys])) return;
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int rsub = lane / P;
  const int col = lane % P;
  const int rend = tl.r0 + tl.nr;
  for (int g0 = wave * WB; g0 < nblk; g0 += kWavesPerBlock * WB) {
    v4 acc[WB];
#pragma unroll
    for (int b = 0; b < WB; ++b) acc[b] = v4{T(0), T(0), T(0), T(0)};
    for (int r = tl.r0; r < rend; r += 4 * SL) {
      T bw[SL], a[SL][WB];
#pragma unroll
      for (int sl = 0; sl < SL; ++sl) {
        const int row = r + 4 * sl + rsub;
        const bool ok = row < rend;
        bw[sl] = ok ? W[(size_t)row * P + col] : T(0);
#pragma unroll
        for (int b = 0; b < WB; ++b)
          a[sl][b] = (ok && g0 + b < nblk) ? V[(size_t)(g0 + b) * vstride + (size_t)row * P + col] : T(0);
      }
#pragma unroll
      for (int b = 0; b < WB; ++b)
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) acc[b] = Mx<T>::mfma(a[sl][b], bw[sl], acc[b]);
    }
#pragma unroll
    for (int b = 0; b < WB; ++b)
      if (g0 + b < nblk) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
          partial[(size_t)blockIdx.x * pstride + (size_t)(g0 + b) * PP + Mx<T>::row(rsub, q) * P + col] =
              acc[b][q];
      }
  }
}

// The LDS-reduced products with wide loads: each wave stages its 16-row slab
// of every block (16 rows x 16 columns: one 16-byte (float) or 32-byte
// (double) vector per lane, lane l holding row l/4, columns 4(l%4)..+3)
// through LDS and reads it back in the operand layout.  The wave reads each
// slab with one vector load per block instead of four scalar ones.  The
// staging area is reused for the cross-wave reduction at the end of a group.
template <class T, int GB>
__global__ __launch_bounds__(kBlock) void bdots_v_kernel(const BTile* __restrict__ tiles,
                                                         const BState* __restrict__ st,
                                                         const T* __restrict__ V, size_t vstride,
                                                         int nblk, const T* __restrict__ W,
                                                         T* __restrict__ partial, size_t pstride) {
  typedef typename Mx<T>::v4 v4;
  __shared__ __align__(16) T s_st[kWavesPerBlock][GB][PP];
  const BTile tl = tiles[blockIdx.x];
  if (!running(st[tl.sys])) return;
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int rsub = lane / P;
  const int col = lane % P;
  const int lr = lane / 4;       // staged row of this lane
  const int lc = (lane % 4) * 4; // first staged column
  const int rend = tl.r0 + tl.nr;
  const v4 z = v4{T(0), T(0), T(0), T(0)};
  for (int g0 = 0; g0 < nblk; g0 += GB) {
    typename Mx<T>::v4 acc[GB];
#pragma unroll
    for (int b = 0; b < GB; ++b) acc[b] = z;
    for (int slab = tl.r0 + 16 * wave; slab < rend; slab += 16 * kWavesPerBlock) {
      const int row = slab + lr;
      const bool ok = row < rend;
      v4 vv[GB];
#pragma unroll
      for (int b = 0; b < GB; ++b)
        vv[b] = (ok && g0 + b < nblk)
                    ? __builtin_nontemporal_load(reinterpret_cast<const v4*>(V + (size_t)(g0 + b) * vstride + (size_t)row * P + lc))
                    : z;
      T bw[4];
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        const int wr = slab + 4 * sl + rsub;
        bw[sl] = wr < rend ? W[(size_t)wr * P + col] : T(0);
      }
#pragma unroll
      for (int b = 0; b < GB; ++b) *reinterpret_cast<v4*>(&s_st[wave][b][lr * P + lc]) = vv[b];
#pragma unroll
      for (int b = 0; b < GB; ++b)
        if (g0 + b < nblk) {
#pragma unroll
          for (int sl = 0; sl < 4; ++sl)
            acc[b] = Mx<T>::mfma(s_st[wave][b][(4 * sl + rsub) * P + col], bw[sl], acc[b]);
        }
    }
    __syncthreads();  // every wave is done staging: the area holds the partial results now
#pragma unroll
    for (int b = 0; b < GB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) s_st[wave][b][Mx<T>::row(rsub, q) * P + col] = acc[b][q];
    __syncthreads();
    for (int b = 0; b < GB && g0 + b < nblk; ++b) {
      const int e = threadIdx.x;
      T sum = s_st[0][b][e];
#pragma unroll
      for (int w = 1; w < kWavesPerBlock; ++w) sum += s_st[w][b][e];
      partial[(size_t)blockIdx.x * pstride + (size_t)(g0 + b) * PP + e] = sum;
    }
    __syncthreads();
  }
}

// Per system and block b: the tile partials added in tile order (float64),
// stored as Cd[s][b][.] and rounded into Cf[s][b][.] (matrix-core operand).
template <class T>
__global__ __launch_bounds__(kBlock) void bfinish_c_kernel(const BSys* __restrict__ sys,
                                                           const BState* __restrict__ st,
                                                           const T* __restrict__ partial,
                                                           size_t pstride, double* Cd, T* Cf,
                                                           size_t cstride) {
  const int s = blockIdx.x;
  const int b = blockIdx.y;
  if (!running(st[s])) return;
  const int e = threadIdx.x;
  double sum = 0.0;
  for (int t = 0; t < sys[s].tile_count; ++t)
    sum += partial[(size_t)(sys[s].tile_start + t) * pstride + (size_t)b * PP + e];
  Cd[(size_t)s * cstride + (size_t)b * PP + e] = sum;
  if (Cf) Cf[(size_t)s * cstride + (size_t)b * PP + e] = T(sum);
}

// ---------------------------------------------------------------------------
// Block update on the matrix cores: for 16-row groups of the tile,
// D = sum_b V_b(rows) C_b with C_b[i][c] from Cf[s][b], then
//   kSub: out -= D;  kSet: out = D (out may alias V when nblk = 1);
//   kXupd: X64[row][c] += gamma_c * D for the columns still above tol.
// The inner index i of V_b C_b is split as i = 4 g + kk (g = lane / 16, kk the
// MFMA step): lane l loads V_b[r0 + l%16][4g .. 4g+3] as one 16-byte vector
// (the wave reads 16 whole rows, 1 KB contiguous) and feeds element kk to step
// kk, whose B operand is C_b[4g + kk][l%16].  The coefficients sit in LDS as
// s_C[b][g][c][kk], so the four B values of a lane are one 16-byte LDS read.
// (float64: 32-byte loads and reads, same order.)  Result: lane l holds rows
// r0 + Mx::row(l/16, q), column l%16.
// ---------------------------------------------------------------------------
enum { kSub = 0, kSet = 1, kXupd = 2 };

// Basis loads of the block update.  The basis is streamed once per pass and
// is far larger than the caches, so float32 loads are non-temporal (keeps W
// and the coefficients cached: config-4 float32 solve 22.5 s -> 21.0 s);
// float64 measured no better with them.
template <class T, class V4>
__device__ __forceinline__ V4 ld_basis(const V4* p) {
  if constexpr (sizeof(T) == 4) return __builtin_nontemporal_load(p);
  else return *p;
}

template <class T, int MODE>
__global__ __launch_bounds__(kBlock) void bgemm_kernel(const BTile* __restrict__ tiles,
                                                       const BState* __restrict__ st,
                                                       const T* V, size_t vstride, int nblk_arg,
                                                       const T* __restrict__ Cf, size_t cstride,
                                                       T* out, double* __restrict__ X64,
                                                       const double* __restrict__ gam,
                                                       const double* __restrict__ bnorm, double tol) {
  typedef typename Mx<T>::v4 v4;
  extern __shared__ __align__(16) char s_dyn[];
  T* s_C = reinterpret_cast<T*>(s_dyn);  // nblk x 16 x 16 coefficients (dynamic)
  const BTile tl = tiles[blockIdx.x];
  const BState ss = st[tl.sys];
  int nblk = nblk_arg;
  if constexpr (MODE == kXupd) {
    if (!ss.active || ss.kblk <= 0) return;
    nblk = ss.kblk;
  } else {
    if (!running(ss)) return;
  }
  const T* C = Cf + (size_t)tl.sys * cstride;
  for (int e = threadIdx.x; e < nblk * PP; e += kBlock) {
    const int b = e / PP, i = (e / P) % P, c = e % P;  // C_b[i][c], i = 4 g + kk
    s_C[((b * 4 + i / 4) * P + c) * 4 + i % 4] = C[e];
  }
  __syncthreads();
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int rend = tl.r0 + tl.nr;
  bool upd_col = true;
  double gc = 0.0;
  if constexpr (MODE == kXupd) {
    const int c = lane % P;
    gc = gam[tl.sys * P + c];
    upd_col = !(gc <= tol * bnorm[tl.sys * P + c]);
  }
  // RG 16-row groups per iteration (rows r0 .. r0+15, r0+64 .. r0+79, ... of the
  // wave's stride) would share the coefficient reads; two measured slower than
  // one (float32 config 4: 21.1 s -> 21.5 s, from the lower occupancy).  The old
  // output values are loaded before the first MFMA.
  const int g = lane / 16;
  const T* Cl = s_C + (g * P + lane % 16) * 4;
  const v4 z = v4{T(0), T(0), T(0), T(0)};
  constexpr int RG = 1;
  for (int r0 = tl.r0 + 16 * wave; r0 < rend; r0 += 16 * kWavesPerBlock * RG) {
    const T* Vr[RG];
    bool aok[RG];
    T old[RG][4];
#pragma unroll
    for (int h = 0; h < RG; ++h) {
      const int rg = r0 + 16 * kWavesPerBlock * h;
      const int arow = rg + lane % 16;
      aok[h] = arow < rend;
      Vr[h] = V + (size_t)arow * P + 4 * g;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rg + Mx<T>::row(g, q);
        old[h][q] = T(0);
        if constexpr (MODE == kSub) {
          if (row < rend) old[h][q] = out[(size_t)row * P + lane % 16];
        }
      }
    }
    // two accumulators per group (even and odd b) so that consecutive MFMAs are independent
    v4 acc[RG][2];
#pragma unroll
    for (int h = 0; h < RG; ++h) acc[h][0] = acc[h][1] = z;
    int b = 0;
    for (; b + 7 < nblk; b += 8) {
      v4 a[RG][8], cb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        cb[u] = *(const v4*)(Cl + (b + u) * PP);
#pragma unroll
        for (int h = 0; h < RG; ++h) a[h][u] = aok[h] ? ld_basis<T>((const v4*)(Vr[h] + (size_t)(b + u) * vstride)) : z;
      }
#pragma unroll
      for (int u = 0; u < 8; u += 2)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int h = 0; h < RG; ++h) {
            acc[h][0] = Mx<T>::mfma(a[h][u][kk], cb[u][kk], acc[h][0]);
            acc[h][1] = Mx<T>::mfma(a[h][u + 1][kk], cb[u + 1][kk], acc[h][1]);
          }
    }
    for (; b < nblk; ++b) {
      const v4 c0 = *(const v4*)(Cl + b * PP);
#pragma unroll
      for (int h = 0; h < RG; ++h) {
        const v4 a0 = aok[h] ? ld_basis<T>((const v4*)(Vr[h] + (size_t)b * vstride)) : z;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) acc[h][0] = Mx<T>::mfma(a0[kk], c0[kk], acc[h][0]);
      }
    }
#pragma unroll
    for (int h = 0; h < RG; ++h) {
      const v4 d = acc[h][0] + acc[h][1];
      const int rg = r0 + 16 * kWavesPerBlock * h;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = rg + Mx<T>::row(g, q);
        if (row < rend) {
          const size_t idx = (size_t)row * P + lane % 16;
          if constexpr (MODE == kSub) out[idx] = old[h][q] - d[q];
          else if constexpr (MODE == kSet) out[idx] = d[q];
          else if (upd_col) X64[idx] += gc * double(d[q]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Small per-system dense steps (float64)
// ---------------------------------------------------------------------------
// Cholesky factorisation G = R^T R (R upper) of a 16 x 16 Gram matrix held in
// LDS, one thread per entry (thread e owns row e / 16, column e % 16).
// Right-looking: after step k the trailing entries hold
// G_iq - sum_{k' <= k} R_k'i R_k'q, subtracted in the order of k, the same order
// as the column-by-column form.  A pivot <= tau G_cc (G_cc the original
// diagonal entry), or a non-finite one, skips column c: row c of R stays
// zero.  Returns the mask of skipped columns (the same in every thread).
// All 256 threads of the block must call it.
__device__ int chol16_lds(double* sG, const double* gdiag, double* sR, double tau) {
  const int i = threadIdx.x / P;
  const int q = threadIdx.x % P;
  sR[threadIdx.x] = 0.0;
  __syncthreads();
  int mask = 0;
  for (int c = 0; c < P; ++c) {
    const double d = sG[c * P + c];
    if (!(d > tau * gdiag[c]) || !isfinite(d)) {  // uniform over the block
      mask |= 1 << c;
      continue;
    }
    const double rcc = sqrt(d);
    if (i == c && q >= c) sR[c * P + q] = (q == c) ? rcc : sG[c * P + q] / rcc;
    __syncthreads();
    if (i > c && q >= i) sG[i * P + q] -= sR[c * P + i] * sR[c * P + q];
    __syncthreads();
  }
  return mask;
}

// Loads the Gram matrix of system s into LDS (and its diagonal).
__device__ void load_gram(const double* __restrict__ G, double* sG, double* gdiag) {
  const double v = G[threadIdx.x];
  sG[threadIdx.x] = v;
  if (threadIdx.x / P == threadIdx.x % P) gdiag[threadIdx.x / P] = v;
  __syncthreads();
}

// Columns of W that (nearly) depend on earlier ones, from G = W^T W (the
// Cholesky factorisation that skips a column whose pivot is <= tau G_cc).
// One block of 256 threads per system.
__global__ __launch_bounds__(kBlock) void bdep_kernel(const BState* __restrict__ st,
                                                      const double* __restrict__ Gd, size_t gstride,
                                                      int* depmask, double tau) {
  const int s = blockIdx.x;
  if (!running(st[s])) return;
  __shared__ double sG[PP], sR[PP], gdiag[P];
  load_gram(Gd + (size_t)s * gstride, sG, gdiag);
  const int mask = chol16_lds(sG, gdiag, sR, tau);
  if (threadIdx.x == 0) depmask[s] = mask;
}

// T = W with the flagged columns taken from the random block Z.
template <class T>
__global__ __launch_bounds__(kBlock) void breplace_kernel(const BTile* __restrict__ tiles,
                                                          const BState* __restrict__ st,
                                                          const int* __restrict__ depmask,
                                                          const T* __restrict__ W,
                                                          const float* __restrict__ Z,
                                                          T* __restrict__ out) {
  const BTile tl = tiles[blockIdx.x];
  if (!running(st[tl.sys])) return;
  const int c = threadIdx.x % P;
  const bool dep = (depmask[tl.sys] >> c) & 1;
  for (int r = tl.r0 + (int)threadIdx.x / P; r < tl.r0 + tl.nr; r += kBlock / P) {
    const size_t i = (size_t)r * P + c;
    out[i] = dep ? T(Z[i]) : W[i];
  }
}

// Cholesky G = R^T R (R upper) and Rinv = R^{-1} (inner precision, matrix-core operand).
// When Rprev is given, Rout = R Rprev (the two Cholesky QR passes combined).
// A pivot <= tau G_cc (or non-finite) is handled by `mode`:
//   kCholStart: the start block failed (the system stops);
//   kCholPass1: breakdown of the block step; Rbrk receives the Cholesky factor
//               that skips the dependent columns, and the block column is the
//               cycle's last;
//   kCholPass2: breakdown in the second pass; Rbrk receives Rprev.
enum { kCholStart = 0, kCholPass1 = 1, kCholPass2 = 2 };

template <class T>
__global__ __launch_bounds__(kBlock) void bchol_kernel(BState* st, const double* __restrict__ Gd,
                                                       size_t gstride, const double* __restrict__ Rprev,
                                                       double* __restrict__ Rout, T* __restrict__ Rinv_f,
                                                       size_t rstride, double tau, int mode,
                                                       double* __restrict__ Rbrk) {
  const int s = blockIdx.x;
  if (!running(st[s])) return;
  __shared__ double sG[PP], sR[PP], sRi[PP], gdiag[P];
  load_gram(Gd + (size_t)s * gstride, sG, gdiag);
  const int mask = chol16_lds(sG, gdiag, sR, tau);
  const int e = threadIdx.x;
  const int i = e / P;
  const int c = e % P;
  if (mask) {
    if (mode == kCholStart) {
      if (e == 0) {  // the system is frozen at its current iterate; the others go on
        st[s].cycle_done = 1;
        st[s].failed = 1;
        st[s].active = 0;
      }
    } else {
      double* Rb = Rbrk + (size_t)s * PP;
      Rb[e] = (mode == kCholPass1) ? (isfinite(sR[e]) ? sR[e] : 0.0) : Rprev[(size_t)s * PP + e];
      if (e == 0) st[s].brk = 1;
    }
    return;
  }
  // upper-triangular inverse, one row per step from the bottom:
  // Ri[r][c] = -(sum_{k=r+1..c} R[r][k] Ri[k][c]) / R[r][r], Ri[r][r] = 1 / R[r][r]
  sRi[e] = 0.0;
  __syncthreads();
  for (int r = P - 1; r >= 0; --r) {
    if (i == r && c >= r) {
      if (c == r) {
        sRi[e] = 1.0 / sR[r * P + r];
      } else {
        double v = 0.0;
        for (int k = r + 1; k <= c; ++k) v += sR[r * P + k] * sRi[k * P + c];
        sRi[e] = -v / sR[r * P + r];
      }
    }
    __syncthreads();
  }
  Rinv_f[(size_t)s * rstride + e] = T(sRi[e]);
  if (Rout) {
    double v = sR[e];
    if (Rprev) {  // the two Cholesky QR passes combined: Rout = R Rprev
      const double* Rp = Rprev + (size_t)s * PP;
      v = 0.0;
      for (int k = i; k <= c; ++k) v += sR[i * P + k] * Rp[k * P + c];
    }
    Rout[(size_t)s * PP + e] = v;
  }
}

// Reset of the per-cycle state and of the right-hand side of the block least
// squares problem: Grhs = [R0; 0] with R0 = V0^T W in Cd.
__global__ void bcycle_reset_kernel(int nsys, BState* st) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  st[s].cycle_done = 0;
  st[s].kblk = 0;
  st[s].brk = 0;
}

__global__ __launch_bounds__(kBlock) void binit_rhs_kernel(const BState* __restrict__ st,
                                                           const double* __restrict__ R0d,
                                                           size_t cstride, double* Grhs,
                                                           size_t gstride) {
  const int s = blockIdx.x;
  if (!running(st[s])) return;
  double* G = Grhs + (size_t)s * gstride;
  for (size_t e = threadIdx.x; e < gstride; e += kBlock) G[e] = (e < PP) ? R0d[(size_t)s * cstride + e] : 0.0;
}

// One block column of the block Hessenberg matrix, [C1 + C2; R], reduced by the
// earlier block Householder reflectors, then a new set of 16 reflectors on its
// 32 x 16 panel; the same reflectors are applied to Grhs.  The wave's 64 lanes
// form 16 quads, quad c owning column c: lane q of the quad keeps rows
// 8q .. 8q+7 of a 32-row window of the column in registers, and a reflector's
// dot product is the quad's sum of four 8-row partial sums.  The reflectors of
// block column bi act on rows 16 bi .. 16 bi + 31 only, so after block column
// bi the top 16 rows of the window are final and the window slides down by 16
// rows; after the last earlier block column it is the new panel.  Reflector t
// of block column i acts on rows 16 i + t .. 16 i + 31 and is stored as v
// (v_t = 1, entries above t unused) with its tau.
__device__ __forceinline__ double quad_sum(double v) {
  v += xor_lane<1>(v);
  v += xor_lane<2>(v);
  return v;
}

__global__ __launch_bounds__(kWave) void bls_kernel(int j, BState* st, const double* __restrict__ C1d,
                                                    const double* __restrict__ C2d, size_t cstride,
                                                    const double* __restrict__ Rn, double* Hq,
                                                    size_t hstride, int ldh, double* refl,
                                                    double* tauv, size_t rfstride, double* Grhs,
                                                    size_t gstride) {
  const int s = blockIdx.x;
  if (!st[s].active || st[s].cycle_done) return;  // a block column that broke down is kept
  __shared__ double s_V[2][32 * P];  // reflectors of one earlier block column, double-buffered
  __shared__ double s_tau[2][P];
  __shared__ double s_v[32];
  __shared__ double s_t;
  const int lane = threadIdx.x;
  const int col = lane / 4;
  const int q = lane % 4;
  double* H = Hq + (size_t)s * hstride;
  double* RF = refl + (size_t)s * rfstride * 32;   // [blockcol][32 rows][16 refl]
  double* TU = tauv + (size_t)s * rfstride;       // [blockcol][16]
  double* G = Grhs + (size_t)s * gstride;          // [row][16]
  double* hcol = H + (size_t)(16 * j + col) * ldh;
  const double* C1 = C1d + (size_t)s * cstride;
  const double* C2 = C2d + (size_t)s * cstride;
  const double* Rs = Rn + (size_t)s * PP;
  // entry of the new column in row 16 b + i
  auto entry = [&](int b, int i) -> double {
    if (b <= j) return C1[b * PP + i * P + col] + C2[b * PP + i * P + col];
    if (b == j + 1) return Rs[i * P + col];
    return 0.0;
  };
  double w[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = entry(q / 2, 8 * (q % 2) + i);
  // earlier reflectors; block column bi + 1's reflectors and the window rows
  // that enter next are loaded while block column bi is applied
  constexpr int kPer = 32 * P / kWave;  // reflector entries per lane
  if (j > 0) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) s_V[0][lane + kWave * u] = RF[lane + kWave * u];
    if (lane < P) s_tau[0][lane] = TU[lane];
    __syncthreads();
  }
  for (int bi = 0; bi < j; ++bi) {
    const int cur = bi & 1;
    double nV[kPer], nT = 0.0, nw[8];
    if (bi + 1 < j) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) nV[u] = RF[(size_t)(bi + 1) * 32 * P + lane + kWave * u];
      if (lane < P) nT = TU[(bi + 1) * P + lane];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) nw[i] = q < 2 ? 0.0 : entry(bi + 2, 8 * (q % 2) + i);
#pragma unroll
    for (int t = 0; t < P; ++t) {
      const double tau = s_tau[cur][t];
      if (tau == 0.0) continue;
      double v[8];
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = 8 * q + i;
        v[i] = r > t ? s_V[cur][r * P + t] : (r == t ? 1.0 : 0.0);
        d += v[i] * w[i];
      }
      d = quad_sum(d) * tau;
#pragma unroll
      for (int i = 0; i < 8; ++i) w[i] -= d * v[i];
    }
    if (q < 2) {
#pragma unroll
      for (int i = 0; i < 8; ++i) hcol[16 * bi + 8 * q + i] = w[i];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double up = __shfl(w[i], lane + 2, kWave);
      w[i] = q < 2 ? up : nw[i];
    }
    if (bi + 1 < j) {
#pragma unroll
      for (int u = 0; u < kPer; ++u) s_V[cur ^ 1][lane + kWave * u] = nV[u];
      if (lane < P) s_tau[cur ^ 1][lane] = nT;
    }
    __syncthreads();  // the other buffer is complete; this one is free for block column bi + 2
  }
  // new reflectors on the panel rows 16 j .. 16 j + 31
  double g[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) g[i] = G[(size_t)(16 * j + 8 * q + i) * P + col];
  double* Vn = RF + (size_t)j * 32 * P;
#pragma unroll
  for (int t = 0; t < P; ++t) {
    // every quad forms the reflector of its own column; quad t's is the one used
    double xn2 = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (8 * q + i > t) xn2 += w[i] * w[i];
    xn2 = quad_sum(xn2);
    const double alpha = quad_sum(q == t / 8 ? w[t % 8] : 0.0);
    if (col == t) {
      double tau = 0.0;
      double beta = alpha;
      double sc = 0.0;
      if (xn2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tau = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = 8 * q + i;
        if (r > t) {
          const double v = w[i] * sc;
          s_v[r] = v;
          Vn[r * P + t] = v;
          w[i] = 0.0;
        }
      }
      if (q == t / 8) w[t % 8] = beta;
      if (q == 0) {
        s_t = tau;
        TU[j * P + t] = tau;
      }
    }
    __syncthreads();
    const double tau = s_t;
    if (tau != 0.0) {
      double v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int r = 8 * q + i;
        v[i] = r > t ? s_v[r] : (r == t ? 1.0 : 0.0);
      }
      if (col > t) {
        double d = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) d += v[i] * w[i];
        d = quad_sum(d) * tau;
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] -= d * v[i];
      }
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < 8; ++i) d += v[i] * g[i];
      d = quad_sum(d) * tau;
#pragma unroll
      for (int i = 0; i < 8; ++i) g[i] -= d * v[i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    hcol[16 * j + 8 * q + i] = w[i];
    G[(size_t)(16 * j + 8 * q + i) * P + col] = g[i];
  }
  for (int i = 16 * (j + 2) + q; i < ldh; i += 4) hcol[i] = 0.0;
  if (lane == 0) {
    st[s].kblk = j + 1;
    if (st[s].brk) {
      st[s].cycle_done = 1;
      st[s].brk = 0;
    }
  }
}

// Y = R^{-1} G over the K = 16 kblk leading rows, rounded into
// Yf[s][b][i * 16 + c] (row 16 b + i).  Block back-substitution from the
// bottom: the 16 x 16 diagonal block of R and the 16 right-hand-side rows are
// solved in LDS (column-oriented), then the rows above are updated with that
// block's 16 solution rows.  Every G row receives its subtractions in the
// order of decreasing solution row, as in the row-by-row column-oriented form.
template <class T>
__global__ __launch_bounds__(kBlock) void bbacksolve_kernel(const BState* __restrict__ st,
                                                            const double* __restrict__ Hq,
                                                            size_t hstride, int ldh, double* Grhs,
                                                            size_t gstride, T* Yf,
                                                            size_t ystride) {
  const int s = blockIdx.x;
  const BState ss = st[s];
  if (!ss.active || ss.kblk <= 0) return;
  __shared__ double sR[PP];  // sR[k][i] = R[16 b + k][16 b + i]
  __shared__ double sG[PP];  // the block's 16 rows of G, then of Y
  const double* H = Hq + (size_t)s * hstride;  // column-major, H[col * ldh + row]
  double* G = Grhs + (size_t)s * gstride;
  T* Y = Yf + (size_t)s * ystride;
  const int e = threadIdx.x;
  const int ei = e / P;  // row within the block
  const int c = e % P;   // right-hand side
  for (int b = ss.kblk - 1; b >= 0; --b) {
    const int r0 = 16 * b;
    sR[ei * P + c] = H[(size_t)(r0 + c) * ldh + r0 + ei];
    sG[e] = G[(size_t)(r0 + ei) * P + c];
    __syncthreads();
    for (int i = P - 1; i >= 0; --i) {
      if (ei == i) sG[e] = sG[e] / sR[i * P + i];
      __syncthreads();
      if (ei < i) sG[e] -= sR[ei * P + i] * sG[i * P + c];
      __syncthreads();
    }
    G[(size_t)(r0 + ei) * P + c] = sG[e];
    Y[(size_t)(r0 + ei) * P + c] = T(sG[e]);
    // rows above the block: G[r] -= sum over the block's rows i (decreasing) of R[r][i] y_i
    for (int r = ei; r < r0; r += kBlock / P) {
      double g = G[(size_t)r * P + c];
      for (int i = P - 1; i >= 0; --i) g -= H[(size_t)(r0 + i) * ldh + r] * sG[i * P + c];
      G[(size_t)r * P + c] = g;
    }
    __syncthreads();
  }
}

}  // namespace bat
}  // namespace gmr

// ===========================================================================
// Host side
// ===========================================================================
using namespace gmr;
using namespace gmr::bat;

struct gmr_batch {
  int nsys = 0;
  int m = 0;
  int tile_rows = 1024;
  int gb = 8;
  int64_t rows = 0;
  std::vector<int> sys_rows;
  std::vector<BSys> sys;
  std::vector<BTile> tiles;
  int max_tiles = 0;  // tile count at the smallest tile size (workspace sizing)
  bool graph = false; // replay each restart cycle as a captured hipGraph
  std::vector<int32_t> sys_status;  // per system, gmr_status of the last solve
};

namespace {

#define BH(call)                                                                          \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return gmr::fail(GMR_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)
#define BT(expr)                    \
  do {                              \
    gmr_status s_ = (expr);         \
    if (s_ != GMR_OK) return s_;    \
  } while (0)

constexpr int kMinTileRows = 256;
// Tiles wanted per launch (4 blocks on each of the 256 CUs): while the active
// systems give fewer, their tiles are halved, down to kMinTileRows.
constexpr int kFillTiles = 1024;
// group_blocks codes of the wave-split dots kernel (blocks per wave x row slices)
constexpr int kDotsW2x8 = 2, kDotsW4x4 = 3, kDotsW4x8 = 5;
// group_blocks codes of the staged wide-load dots kernel (8 or 16 blocks per pass)
constexpr int kDotsV8 = 6, kDotsV16 = 7;
inline bool valid_gb(int g) {
  return g == 4 || g == 8 || g == 16 || g == kDotsW2x8 || g == kDotsW4x4 || g == kDotsW4x8 || g == kDotsV8 ||
         g == kDotsV16;
}
inline size_t al(size_t v) { return (v + 255) / 256 * 256; }

// Tile table over the systems with use[s] set (the others get no tiles), with
// tiles of tile_rows rows; b->tile_rows (the tuned size) is not changed.
void fill_tiles(gmr_batch* b, int tile_rows, const std::vector<char>& use) {
  b->tiles.clear();
  b->sys.resize(b->nsys);
  int64_t off = 0;
  for (int s = 0; s < b->nsys; ++s) {
    BSys& y = b->sys[s];
    y.row_off = (int)off;
    y.n = b->sys_rows[s];
    y.tile_start = (int)b->tiles.size();
    if (use[s])
      for (int r = 0; r < y.n; r += tile_rows) b->tiles.push_back({s, (int)off + r, std::min(tile_rows, y.n - r), 0});
    y.tile_count = (int)b->tiles.size() - y.tile_start;
    off += y.n;
  }
}

void build_tiles(gmr_batch* b, int tile_rows) {
  b->tile_rows = tile_rows;
  fill_tiles(b, tile_rows, std::vector<char>(b->nsys, 1));
}

int count_tiles(const gmr_batch* b, int tile_rows) {
  int t = 0;
  for (int s = 0; s < b->nsys; ++s) t += (b->sys_rows[s] + tile_rows - 1) / tile_rows;
  return t;
}

struct BLayout {
  size_t tiles, sys, st, gam, bnorm, dep, V, W, T, R64, partial, rpart, C1d, C2d, Cd, Cf, R1, Rn,
      Hq, refl, tau, Grhs, Yf, end;
  size_t vstride, pstride, cstride, hstride, gstride, rfstride, ystride;
  int ldh;
};

// Workspace layout; `elt` is the size of the inner precision (4 or 8 bytes).
BLayout layout(const gmr_batch* b, size_t elt) {
  BLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = al(o + bytes); return at; };
  const int m = b->m;
  const size_t rows = (size_t)b->rows;
  L.vstride = rows * P;
  L.pstride = (size_t)(m + 1) * PP;
  L.cstride = (size_t)(m + 1) * PP;
  L.ldh = 16 * (m + 1);
  L.hstride = (size_t)L.ldh * 16 * m;
  L.gstride = (size_t)L.ldh * P;
  L.rfstride = (size_t)m * P;
  L.ystride = (size_t)m * PP;
  const size_t ns = b->nsys;
  L.tiles = take((size_t)b->max_tiles * sizeof(BTile));
  L.sys = take(ns * sizeof(BSys));
  L.st = take((ns + 1) * sizeof(BState));
  L.gam = take(ns * P * 8);
  L.bnorm = take(ns * P * 8);
  L.dep = take(ns * 4);
  L.V = take((size_t)(m + 1) * L.vstride * elt);
  L.W = take(L.vstride * elt);
  L.T = take(L.vstride * elt);
  L.R64 = take(L.vstride * 8);
  L.partial = take((size_t)b->max_tiles * L.pstride * elt);
  L.rpart = take((size_t)b->max_tiles * P * 8);
  L.C1d = take(ns * L.cstride * 8);
  L.C2d = take(ns * L.cstride * 8);
  L.Cd = take(ns * L.cstride * 8);
  L.Cf = take(ns * L.cstride * elt);
  L.R1 = take(ns * PP * 8);
  L.Rn = take(ns * PP * 8);
  L.Hq = take(ns * L.hstride * 8);
  L.refl = take(ns * L.rfstride * 32 * 8);
  L.tau = take(ns * L.rfstride * 8);
  L.Grhs = take(ns * L.gstride * 8);
  L.Yf = take(ns * L.ystride * elt);
  L.end = o;
  return L;
}

struct BRun {
  const gmr_batch* b;
  BLayout L;
  char* base;
  hipStream_t s;
  int grid = 0;  // fixed launch grid over a device-built table (0: the host table)
  template <class T> T* at(size_t off) const { return (T*)(base + off); }
  int ntiles() const { return grid > 0 ? grid : (int)b->tiles.size(); }
};

gmr_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return gmr::fail(GMR_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GMR_OK;
}

// C[s][b] = V_b^T W for b < nblk, summed per system into Cd (and Cf).
// Float64 uses at most 8 blocks per group (its LDS partials are twice as big).
template <class T>
gmr_status dots(const BRun& R, const T* V, int nblk, const T* W, double* Cd, T* Cf) {
  const BTile* tl = R.at<BTile>(R.L.tiles);
  const BState* st = R.at<BState>(R.L.st);
  T* part = R.at<T>(R.L.partial);
  const int gb = (sizeof(T) == 8 && R.b->gb == 16) ? 8 : R.b->gb;
  const int g = R.ntiles();
  const size_t vs = R.L.vstride, ps = R.L.pstride;
  switch (gb) {
    case 4: bdots_kernel<T, 4><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps); break;
    case 16: bdots_kernel<T, 16><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps); break;
    case kDotsW2x8: bdots_w_kernel<T, 2, 8><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps); break;
    case kDotsW4x4: bdots_w_kernel<T, 4, 4><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps); break;
    case kDotsW4x8: bdots_w_kernel<T, 4, 8><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps); break;
    case kDotsV8:
    case kDotsV16:
      // float64 keeps the scalar-load variant: its 32-byte staged form was slower
      // (float64 config-4 solve 40.4 s -> 42.4 s)
      if constexpr (sizeof(T) == 8)
        bdots_kernel<T, 8><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps);
      else if (gb == kDotsV8)
        bdots_v_kernel<T, 8><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps);
      else
        bdots_v_kernel<T, 16><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps);
      break;
    default: bdots_kernel<T, 8><<<g, kBlock, 0, R.s>>>(tl, st, V, vs, nblk, W, part, ps); break;
  }
  BT(launch_check("bdots_kernel"));
  bfinish_c_kernel<T><<<dim3(R.b->nsys, nblk), kBlock, 0, R.s>>>(R.at<BSys>(R.L.sys), st, part, R.L.pstride, Cd,
                                                                   Cf, R.L.cstride);
  return launch_check("bfinish_c_kernel");
}

// Dynamic LDS of the block update: the nblk coefficient blocks (up to 130 KB
// in float64 at the largest restart, within the 160 KB a workgroup may use).
template <class T, int MODE>
gmr_status gemm_launch(const BRun& R, const T* V, int nblk, const T* Cf, size_t cstride, T* out, double* X64,
                       double tol) {
  const size_t lds = (size_t)nblk * PP * sizeof(T);
  bgemm_kernel<T, MODE><<<R.ntiles(), kBlock, lds, R.s>>>(R.at<BTile>(R.L.tiles), R.at<BState>(R.L.st), V,
                                                          R.L.vstride, nblk, Cf, cstride, out, X64,
                                                          R.at<double>(R.L.gam), R.at<double>(R.L.bnorm), tol);
  return launch_check("bgemm_kernel");
}

// Raises the dynamic LDS limit of the block-update kernels to the largest
// coefficient set (called before any launch, outside graph capture).
template <class T>
gmr_status raise_lds_limits() {
  const int bytes = (int)(kMaxBlocks * PP * sizeof(T));
  BH(hipFuncSetAttribute(reinterpret_cast<const void*>(&bgemm_kernel<T, kSub>),
                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  BH(hipFuncSetAttribute(reinterpret_cast<const void*>(&bgemm_kernel<T, kSet>),
                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  BH(hipFuncSetAttribute(reinterpret_cast<const void*>(&bgemm_kernel<T, kXupd>),
                         hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  return GMR_OK;
}

template <class T, int MODE>
gmr_status gemm(const BRun& R, const T* V, int nblk, const T* Cf, T* out) {
  return gemm_launch<T, MODE>(R, V, nblk, Cf, R.L.cstride, out, nullptr, 0.0);
}

template <class T>
gmr_status chol(const BRun& R, const double* Gd, const double* Rprev, double* Rout, double tau, int mode) {
  const int ns = R.b->nsys;
  bchol_kernel<T><<<ns, kBlock, 0, R.s>>>(R.at<BState>(R.L.st), Gd, R.L.cstride, Rprev, Rout, R.at<T>(R.L.Cf),
                                          R.L.cstride, tau, mode, R.at<double>(R.L.Rn));
  return launch_check("bchol_kernel");
}

// Cholesky QR twice of T in place: on success T is orthonormal; the
// orthonormal block is written to `dst`, and, for a block step, Rn = R2 R1.
// A start block uses only a positivity threshold (its dependent columns were
// replaced before); a block step breaks down below tau.
template <class T>
gmr_status cholqr2(const BRun& R, T* Tm, T* dst, double tau, bool start) {
  double* Cd = R.at<double>(R.L.Cd);
  T* Cf = R.at<T>(R.L.Cf);
  const int m1 = start ? kCholStart : kCholPass1;
  const int m2 = start ? kCholStart : kCholPass2;
  BT(dots<T>(R, Tm, 1, Tm, Cd, nullptr));
  BT(chol<T>(R, Cd, nullptr, start ? nullptr : R.at<double>(R.L.R1), tau, m1));
  BT((gemm<T, kSet>(R, Tm, 1, Cf, Tm)));
  BT(dots<T>(R, Tm, 1, Tm, Cd, nullptr));
  BT(chol<T>(R, Cd, start ? nullptr : R.at<double>(R.L.R1), start ? nullptr : R.at<double>(R.L.Rn), tau, m2));
  return gemm<T, kSet>(R, Tm, 1, Cf, dst);
}

// Captures what `body` enqueues on stream s into an executable graph.
template <class F>
gmr_status capture_graph(hipStream_t s, hipGraphExec_t* out, F&& body) {
  BH(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const gmr_status st = body();
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &g);
  if (st != GMR_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return gmr::fail(GMR_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return gmr::fail(GMR_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
  return GMR_OK;
}

gmr_status check_batch_csr(const gmr_csr* A, int dtype, int64_t rows) {
  if (!A || A->dtype != dtype || A->n != rows || !A->row_ptr || !A->col_idx || !A->val)
    return gmr::fail(GMR_ERR_INVALID, "batched: matrix does not match the batch (dtype or rows)");
  return GMR_OK;
}

}  // namespace

extern "C" {

gmr_status batch_create(int32_t nsys, const int32_t* sys_rows, int32_t nrhs, int32_t restart,
                        gmr_batch** out) {
  if (!out || !sys_rows || nsys <= 0) return gmr::fail(GMR_ERR_INVALID, "batch_create: bad arguments");
  if (nrhs != P) return gmr::fail(GMR_ERR_UNSUPPORTED, "batch_create: the block size is 16 right-hand sides");
  if (restart < 1 || restart > kMaxBlocks - 1)
    return gmr::fail(GMR_ERR_UNSUPPORTED, "batch_create: restart must be in [1, 64]");
  gmr_batch* b = new gmr_batch;
  b->nsys = nsys;
  b->m = restart;
  b->sys_rows.assign(sys_rows, sys_rows + nsys);
  int64_t rows = 0;
  for (int s = 0; s < nsys; ++s) {
    if (sys_rows[s] <= 0) {
      delete b;
      return gmr::fail(GMR_ERR_INVALID, "batch_create: every system needs rows > 0");
    }
    rows += sys_rows[s];
  }
  if (rows >= (int64_t)1 << 31) {
    delete b;
    return gmr::fail(GMR_ERR_UNSUPPORTED, "batch_create: total rows must fit int32");
  }
  b->rows = rows;
  b->max_tiles = count_tiles(b, kMinTileRows);
  build_tiles(b, 1024);
  *out = b;
  return GMR_OK;
}

void batch_destroy(gmr_batch* b) { delete b; }

size_t batch_workspace_bytes(const gmr_batch* b, int32_t inner_dtype) {
  if (!b || (inner_dtype != GMR_F32 && inner_dtype != GMR_F64)) return 0;
  return layout(b, inner_dtype == GMR_F64 ? 8 : 4).end;
}

gmr_status batch_set_tiling(gmr_batch* b, int32_t tile_rows, int32_t group_blocks) {
  if (!b) return gmr::fail(GMR_ERR_INVALID, "batch_set_tiling: null batch");
  if (tile_rows < kMinTileRows || tile_rows % 16 != 0)
    return gmr::fail(GMR_ERR_INVALID, "batch_set_tiling: tile_rows must be a multiple of 16, >= 256");
  if (!valid_gb(group_blocks))
    return gmr::fail(GMR_ERR_INVALID, "batch_set_tiling: group_blocks must be 4, 8, 16 (LDS-reduced dots), "
                                      "2, 3, 5 (wave-split dots) or 6, 7 (staged wide-load dots)");
  build_tiles(b, tile_rows);
  b->gb = group_blocks;
  return GMR_OK;
}

gmr_status batch_set_graph(gmr_batch* b, int32_t on) {
  if (!b) return gmr::fail(GMR_ERR_INVALID, "batch_set_graph: null batch");
  b->graph = on != 0;
  return GMR_OK;
}

gmr_status batch_system_status(const gmr_batch* b, int32_t* out) {
  if (!b || !out) return gmr::fail(GMR_ERR_INVALID, "batch_system_status: null pointer");
  if ((int)b->sys_status.size() != b->nsys) return gmr::fail(GMR_ERR_INVALID, "batch_system_status: no solve yet");
  std::copy(b->sys_status.begin(), b->sys_status.end(), out);
  return GMR_OK;
}

gmr_status batch_get_tiling(const gmr_batch* b, int32_t* tile_rows, int32_t* group_blocks) {
  if (!b || !tile_rows || !group_blocks) return gmr::fail(GMR_ERR_INVALID, "batch_get_tiling: null pointer");
  *tile_rows = b->tile_rows;
  *group_blocks = b->gb;
  return GMR_OK;
}

}  // extern "C"

namespace {

gmr_status upload_tables(const BRun& R) {
  BH(hipMemcpyAsync(R.at<BTile>(R.L.tiles), R.b->tiles.data(), R.b->tiles.size() * sizeof(BTile),
                    hipMemcpyHostToDevice, R.s));
  BH(hipMemcpyAsync(R.at<BSys>(R.L.sys), R.b->sys.data(), R.b->sys.size() * sizeof(BSys),
                    hipMemcpyHostToDevice, R.s));
  return GMR_OK;
}

// The batched solve with inner precision T (float: GMRES-IR; double: plain
// float64 block GMRES(m)).  Ain is A in precision T.
template <class T>
gmr_status solve_impl(const char* name, gmr_batch* b, const gmr_csr* A64, const gmr_csr* Ain, const double* B,
                      double* X, const float* Z, double tol, int32_t max_cycles, void* ws, size_t ws_bytes,
                      gmr_batch_result* res, int32_t* sys_cycles, double* sys_rel_res, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  const std::string nm(name);
  if (!b || !B || !X || !Z || !res) return gmr::fail(GMR_ERR_INVALID, nm + ": null argument");
  if (!(tol > 0.0) || max_cycles < 1) return gmr::fail(GMR_ERR_INVALID, nm + ": bad tol or max_cycles");
  BT(check_batch_csr(A64, GMR_F64, b->rows));
  BT(check_batch_csr(Ain, sizeof(T) == 8 ? GMR_F64 : GMR_F32, b->rows));
  BRun R{b, layout(b, sizeof(T)), (char*)ws, (hipStream_t)stream};
  if (!ws || ws_bytes < R.L.end) return gmr::fail(GMR_ERR_WORKSPACE, nm + ": workspace too small");
  BT(raise_lds_limits<T>());
  if (b->graph) {
    // capture needs a stream other than the legacy one: the solve runs on the
    // library's own stream once the caller's stream has drained
    BH(hipStreamSynchronize(R.s));
    BT(library_stream(&R.s));
  }
  const int ns = b->nsys;
  const int m = b->m;
  // the host table supplies the systems' row ranges; the device rebuilds the
  // tile list of the active systems at the start of every cycle
  fill_tiles(b, b->tile_rows, std::vector<char>(ns, 1));
  BT(upload_tables(R));
  // Fixed grid of every tile launch.  No device-built table is longer: tiles
  // are halved only while there are fewer than kFillTiles of them, and one
  // halving at most triples a system's tile count.
  R.grid = std::min(b->max_tiles, std::max(count_tiles(b, b->tile_rows), 3 * kFillTiles));
  const int nt = R.ntiles();
  BTile* tl = R.at<BTile>(R.L.tiles);
  BSys* sy = R.at<BSys>(R.L.sys);
  BState* st = R.at<BState>(R.L.st);
  double* gam = R.at<double>(R.L.gam);
  double* bnorm = R.at<double>(R.L.bnorm);
  T* V = R.at<T>(R.L.V);
  T* W = R.at<T>(R.L.W);
  T* Tm = R.at<T>(R.L.T);
  double* R64 = R.at<double>(R.L.R64);
  double* rpart = R.at<double>(R.L.rpart);
  double* Cd = R.at<double>(R.L.Cd);
  double* C1d = R.at<double>(R.L.C1d);
  double* C2d = R.at<double>(R.L.C2d);
  T* Cf = R.at<T>(R.L.Cf);
  std::vector<BState> hst(ns + 1);
  for (auto& h : hst) h = BState{1, 0, 0, 0, 0, 0};
  hst[ns] = BState{0, 0, 0, 0, 0, 0};  // the idle system of the unused tiles
  BH(hipMemcpyAsync(st, hst.data(), (ns + 1) * sizeof(BState), hipMemcpyHostToDevice, R.s));
  auto tile_table = [&]() -> gmr_status {
    btiles_kernel<<<1, kBlock, 0, R.s>>>(ns, sy, st, b->tile_rows, kMinTileRows, kFillTiles, R.grid, tl);
    return launch_check("btiles_kernel");
  };
  BT(tile_table());
  // ||B|| per column, then the residual of the initial X
  bresidual_kernel<<<nt, kBlock, 0, R.s>>>(tl, nullptr, A64->row_ptr, A64->col_idx, (const double*)A64->val,
                                           nullptr, B, R64, rpart);
  BT(launch_check("bresidual_kernel"));
  bfinish_res_kernel<<<ns, 64, 0, R.s>>>(ns, sy, st, rpart, gam, bnorm, tol, 0);
  BT(launch_check("bfinish_res_kernel"));
  auto residual = [&]() -> gmr_status {
    bresidual_kernel<<<nt, kBlock, 0, R.s>>>(tl, st, A64->row_ptr, A64->col_idx, (const double*)A64->val, X, B,
                                             R64, rpart);
    BT(launch_check("bresidual_kernel"));
    bfinish_res_kernel<<<ns, 64, 0, R.s>>>(ns, sy, st, rpart, gam, bnorm, tol, 1);
    return launch_check("bfinish_res_kernel");
  };
  BT(residual());
  // Everything one restart cycle enqueues, from the start block to the next
  // residual; the same launches with the same arguments every cycle, so it
  // can be captured once and replayed.
  auto enqueue_cycle = [&]() -> gmr_status {
    BT(tile_table());  // the systems still active after the last residual
    // --- start block: W = R/gamma, dependent columns from Z, Cholesky QR twice
    bcycle_reset_kernel<<<(ns + 63) / 64, 64, 0, R.s>>>(ns, st);
    bstart_kernel<T><<<nt, kBlock, 0, R.s>>>(tl, st, R64, gam, W);
    BT(launch_check("bstart_kernel"));
    BT(dots<T>(R, W, 1, W, Cd, nullptr));
    // a start column is replaced when its part outside the span of the earlier
    // kept columns has relative squared norm <= tau: with a float32 inner solve
    // 1e-3, which keeps the start block's condition number within the range
    // (about u^-1/2) where Cholesky QR twice in float32 is reliable
    bdep_kernel<<<ns, kBlock, 0, R.s>>>(st, Cd, R.L.cstride, R.at<int>(R.L.dep), sizeof(T) == 4 ? 1e-3 : 1e-5);
    BT(launch_check("bdep_kernel"));
    breplace_kernel<T><<<nt, kBlock, 0, R.s>>>(tl, st, R.at<int>(R.L.dep), W, Z, Tm);
    BT(launch_check("breplace_kernel"));
    BT(cholqr2<T>(R, Tm, V, 1e-12, true));
    BT(dots<T>(R, V, 1, W, Cd, nullptr));  // R0 = V0^T W
    binit_rhs_kernel<<<ns, kBlock, 0, R.s>>>(st, Cd, R.L.cstride, R.at<double>(R.L.Grhs), R.L.gstride);
    BT(launch_check("binit_rhs_kernel"));
    // --- m block steps
    for (int j = 0; j < m; ++j) {
      const int nb = j + 1;
      bspmm_kernel<T><<<nt, kBlock, 0, R.s>>>(tl, st, Ain->row_ptr, Ain->col_idx, (const T*)Ain->val,
                                              V + (size_t)j * R.L.vstride, W);
      BT(launch_check("bspmm_kernel"));
      BT(dots<T>(R, V, nb, W, C1d, Cf));
      BT((gemm<T, kSub>(R, V, nb, Cf, W)));
      BT(dots<T>(R, V, nb, W, C2d, Cf));
      BT((gemm<T, kSub>(R, V, nb, Cf, W)));
      BT(cholqr2<T>(R, W, V + (size_t)(j + 1) * R.L.vstride, 1e-5, false));
      bls_kernel<<<ns, kWave, 0, R.s>>>(j, st, C1d, C2d, R.L.cstride, R.at<double>(R.L.Rn),
                                        R.at<double>(R.L.Hq), R.L.hstride, R.L.ldh, R.at<double>(R.L.refl),
                                        R.at<double>(R.L.tau), R.L.rfstride, R.at<double>(R.L.Grhs), R.L.gstride);
      BT(launch_check("bls_kernel"));
    }
    // --- solution update and the next residual
    T* Yf = R.at<T>(R.L.Yf);
    bbacksolve_kernel<T><<<ns, kBlock, 0, R.s>>>(st, R.at<double>(R.L.Hq), R.L.hstride, R.L.ldh,
                                                 R.at<double>(R.L.Grhs), R.L.gstride, Yf, R.L.ystride);
    BT(launch_check("bbacksolve_kernel"));
    // the update reads C from Yf, laid out like the Gram-Schmidt coefficients
    BT((gemm_launch<T, kXupd>(R, V, m, Yf, R.L.ystride, nullptr, X, tol)));
    return residual();
  };
  struct GraphExec {
    hipGraphExec_t g = nullptr;
    ~GraphExec() {
      if (g) (void)hipGraphExecDestroy(g);
    }
  } graph;
  std::vector<int> cycles(ns, 0);
  int total_cycles = 0;
  int64_t block_iters = 0;
  gmr_status status = GMR_NOT_CONVERGED;
  int failed = 0;
  for (int cyc = 0;; ++cyc) {
    BH(hipMemcpyAsync(hst.data(), st, (ns + 1) * sizeof(BState), hipMemcpyDeviceToHost, R.s));
    BH(hipStreamSynchronize(R.s));
    if (hst[ns].failed) {
      status = gmr::fail(GMR_ERR_HIP, nm + ": internal error, the tile table outgrew its launch grid");
      break;
    }
    int active = 0;
    failed = 0;
    for (int s = 0; s < ns; ++s) {
      if (hst[s].failed) ++failed;  // frozen (its start block could not be formed); the others go on
      else if (hst[s].active) ++active;
    }
    if (cyc > 0)
      for (int s = 0; s < ns; ++s)
        if (hst[s].kblk > 0) block_iters += hst[s].kblk;
    if (active == 0) {
      status = failed ? GMR_SYSTEMS_FAILED : GMR_OK;
      break;
    }
    if (cyc >= max_cycles) break;
    for (int s = 0; s < ns; ++s)
      if (hst[s].active) ++cycles[s];
    ++total_cycles;
    // every launch of the cycle covers the device-built table of the systems
    // still active, with smaller tiles when those are too few to fill the GPU
    if (b->graph) {
      if (!graph.g) BT(capture_graph(R.s, &graph.g, enqueue_cycle));
      BH(hipGraphLaunch(graph.g, R.s));
    } else {
      BT(enqueue_cycle());
    }
  }
  BH(hipStreamSynchronize(R.s));
  if (status < 0) return status;
  BH(hipMemcpy(hst.data(), st, (ns + 1) * sizeof(BState), hipMemcpyDeviceToHost));
  std::vector<double> hg(ns * P), hb(ns * P);
  BH(hipMemcpy(hg.data(), gam, ns * P * 8, hipMemcpyDeviceToHost));
  BH(hipMemcpy(hb.data(), bnorm, ns * P * 8, hipMemcpyDeviceToHost));
  double worst = 0.0;
  b->sys_status.assign(ns, GMR_OK);
  for (int s = 0; s < ns; ++s) {
    b->sys_status[s] = hst[s].failed ? GMR_ERR_NONFINITE : (hst[s].active ? GMR_NOT_CONVERGED : GMR_OK);
    for (int c = 0; c < P; ++c) {
      const int i = s * P + c;
      const double r = hb[i] > 0.0 ? hg[i] / hb[i] : 0.0;
      if (!hst[s].failed) worst = std::max(worst, r);
      if (sys_rel_res) sys_rel_res[i] = r;
    }
  }
  if (status == GMR_SYSTEMS_FAILED)
    gmr::fail(GMR_SYSTEMS_FAILED, nm + ": " + std::to_string(failed) +
                                      " system(s) stopped: a start block could not be orthonormalised");
  if (sys_cycles)
    for (int s = 0; s < ns; ++s) sys_cycles[s] = cycles[s];
  const auto t1 = std::chrono::steady_clock::now();
  res->status = status;
  res->cycles = total_cycles;
  res->block_iters = block_iters;
  res->max_rel_res = worst;
  res->seconds = std::chrono::duration<double>(t1 - t0).count();
  return status;
}

}  // namespace

extern "C" {

gmr_status batch_gmres_ir_solve(gmr_batch* b, const gmr_csr* A64, const gmr_csr* A32, const double* B,
                                double* X, const float* Z, double tol, int32_t max_cycles, void* ws,
                                size_t ws_bytes, gmr_batch_result* res, int32_t* sys_cycles,
                                double* sys_rel_res, void* stream) {
  return solve_impl<float>("batch_gmres_ir_solve", b, A64, A32, B, X, Z, tol, max_cycles, ws, ws_bytes, res,
                           sys_cycles, sys_rel_res, stream);
}

gmr_status batch_gmres_solve(gmr_batch* b, const gmr_csr* A64, const double* B, double* X, const float* Z,
                             double tol, int32_t max_cycles, void* ws, size_t ws_bytes, gmr_batch_result* res,
                             int32_t* sys_cycles, double* sys_rel_res, void* stream) {
  return solve_impl<double>("batch_gmres_solve", b, A64, A64, B, X, Z, tol, max_cycles, ws, ws_bytes, res,
                            sys_cycles, sys_rel_res, stream);
}

// Chooses the tiling by timing the block Gram-Schmidt contractions at three
// basis sizes, about (m+1)/8, (m+1)/2 and 7(m+1)/8 blocks, on the batch's own
// buffers (the workspace is the solve's; its contents are overwritten).
gmr_status batch_autotune(gmr_batch* b, void* ws, size_t ws_bytes, int32_t* best_tile_rows,
                          int32_t* best_group_blocks, double* best_ms, void* stream) {
  if (!b) return gmr::fail(GMR_ERR_INVALID, "batch_autotune: null batch");
  BRun R{b, layout(b, 4), (char*)ws, (hipStream_t)stream};
  if (!ws || ws_bytes < R.L.end) return gmr::fail(GMR_ERR_WORKSPACE, "batch_autotune: workspace too small");
  const int ns = b->nsys;
  std::vector<BState> hst(ns, BState{1, 0, 0, 0, 0, 0});
  BH(hipMemcpyAsync(R.at<BState>(R.L.st), hst.data(), ns * sizeof(BState), hipMemcpyHostToDevice, R.s));
  BH(hipMemsetAsync(R.at<float>(R.L.V), 0, (size_t)(b->m + 1) * R.L.vstride * 4, R.s));
  BH(hipMemsetAsync(R.at<float>(R.L.W), 0, R.L.vstride * 4, R.s));
  BH(hipMemsetAsync(R.at<float>(R.L.Cf), 0, (size_t)ns * R.L.cstride * 4, R.s));
  hipEvent_t e0, e1;
  BH(hipEventCreate(&e0));
  BH(hipEventCreate(&e1));
  // a block step of a cycle sees every basis size from 1 to m + 1: time the
  // pair at a small, a middle and a large one
  const int nbs[3] = {std::max(1, (b->m + 1) / 8), std::max(1, (b->m + 1) / 2), std::max(1, (b->m + 1) * 7 / 8)};
  const int cand_rows[] = {512, 1024, 2048, 4096};
  const int cand_gb[] = {4, 8, 16, kDotsW2x8, kDotsW4x4, kDotsW4x8, kDotsV8, kDotsV16};
  // The fastest of `reps` timed repetitions (after one warm-up) of the dots,
  // and with `upd` the block update too, at the three basis sizes.
  auto time_pair = [&](int reps, bool upd, float* out) -> gmr_status {
    float ms = 1e30f;
    for (int rep = 0; rep <= reps; ++rep) {
      if (hipEventRecord(e0, R.s) != hipSuccess) return GMR_ERR_HIP;
      for (int nb : nbs) {
        BT(dots<float>(R, R.at<float>(R.L.V), nb, R.at<float>(R.L.W), R.at<double>(R.L.Cd), R.at<float>(R.L.Cf)));
        if (upd) BT((gemm<float, kSub>(R, R.at<float>(R.L.V), nb, R.at<float>(R.L.Cf), R.at<float>(R.L.W))));
      }
      if (hipEventRecord(e1, R.s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return GMR_ERR_HIP;
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (rep > 0) ms = std::min(ms, t);
    }
    *out = ms;
    return GMR_OK;
  };
  // Two stages: the tile size by the dots and update together (with the staged
  // dots variant), then the dots variant at that tile size by the dots alone,
  // whose differences (a few per cent) the pair would blur with run-to-run noise.
  double best = 1e30;
  int bt = b->tile_rows, bg = kDotsV16;
  gmr_status status = GMR_OK;
  for (int tr : cand_rows) {
    build_tiles(b, tr);
    b->gb = kDotsV16;
    float ms = 0.f;
    if ((status = upload_tables(R)) != GMR_OK || (status = time_pair(5, true, &ms)) != GMR_OK) break;
    if (ms < best) {
      best = ms;
      bt = tr;
    }
  }
  if (status == GMR_OK) {
    build_tiles(b, bt);
    status = upload_tables(R);
    float best_d = 1e30f;
    for (int g : cand_gb) {
      if (status != GMR_OK) break;
      b->gb = g;
      float ms = 0.f;
      if ((status = time_pair(9, false, &ms)) != GMR_OK) break;
      if (ms < best_d) {
        best_d = ms;
        bg = g;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  build_tiles(b, bt);
  b->gb = bg;
  if (status != GMR_OK) return gmr::fail(status, "batch_autotune: a timed launch failed");
  if (best_tile_rows) *best_tile_rows = bt;
  if (best_group_blocks) *best_group_blocks = bg;
  if (best_ms) *best_ms = best;
  return GMR_OK;
}

// Block dots and block update on their own, for the parity tests:
// C[s][b] = V_b^T W (float64, ns x nblk x 16 x 16) and then W -= V C.
gmr_status batch_bcgs_step(gmr_batch* b, const float* Vin, int32_t nblk, float* W, double* C, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!b || !Vin || !W || !C || nblk < 1 || nblk > b->m + 1)
    return gmr::fail(GMR_ERR_INVALID, "batch_bcgs_step: bad arguments");
  BRun R{b, layout(b, 4), (char*)ws, (hipStream_t)stream};
  if (!ws || ws_bytes < R.L.end) return gmr::fail(GMR_ERR_WORKSPACE, "batch_bcgs_step: workspace too small");
  const int ns = b->nsys;
  std::vector<BState> hst(ns, BState{1, 0, 0, 0, 0, 0});
  BH(hipMemcpyAsync(R.at<BState>(R.L.st), hst.data(), ns * sizeof(BState), hipMemcpyHostToDevice, R.s));
  fill_tiles(b, b->tile_rows, std::vector<char>(ns, 1));
  BT(upload_tables(R));
  // the kernels read the caller's blocks in place when they are aligned as
  // the workspace basis is (256 bytes), a copy of them otherwise
  const float* V = Vin;
  if ((uintptr_t)Vin % 256 != 0) {
    BH(hipMemcpyAsync(R.at<float>(R.L.V), Vin, (size_t)nblk * R.L.vstride * 4, hipMemcpyDeviceToDevice, R.s));
    V = R.at<float>(R.L.V);
  }
  BT(dots<float>(R, V, nblk, W, R.at<double>(R.L.Cd), R.at<float>(R.L.Cf)));
  BH(hipMemcpy2DAsync(C, (size_t)nblk * PP * 8, R.at<double>(R.L.Cd), R.L.cstride * 8, (size_t)nblk * PP * 8, ns,
                      hipMemcpyDeviceToDevice, R.s));
  return gemm<float, kSub>(R, V, nblk, R.at<float>(R.L.Cf), W);
}

}  // extern "C"
