// GMRES-IR inner solve with the Krylov basis V stored in IEEE float16: the
// third precision that §VI names as future work.  Arithmetic stays float32
// (products, sums, w, the SpMV); only the stored basis vectors are rounded to
// float16, which halves the bytes of the basis that every CGS2 pass streams.
//
// A unit basis vector has entries of size about 1/sqrt(n), far below float16's
// normal range at large n, so column j is stored as half(sigma * v_j) with the
// power of two sigma ~ sqrt(n) (|sigma v_i| <= sigma <= 2^15 < 65504).  All
// scaling is by powers of two, hence exact:
//   dots    h = V^T w         = sum_r  Vs[r] * (w[r] / sigma)
//   update  w -= V h          = w - sum_c Vs[:, c] * (h[c] / sigma)
//   x      += gamma V y       = gamma * sum_c Vs[:, c] * (y[c] / sigma)
// The kernels mirror the float32 ones (same butterflies, fixed-order partial
// sums and float64 finish kernels), with two rows per lane where the float32
// form has one so that a wave still reads 256 contiguous bytes per column.
#pragma once

#include "kernels.hpp"

namespace gmr {

typedef _Float16 half_t;
typedef _Float16 hvec2_t __attribute__((ext_vector_type(2)));
typedef _Float16 hvec4_t __attribute__((ext_vector_type(4)));
typedef float fvec2_t __attribute__((ext_vector_type(2)));

// y = A (x * scale) as spmv_kernel<float>, with v_j = x * scale stored in the
// basis as half(sigma * v_j).
__global__ __launch_bounds__(kBlock) void spmv_hb_kernel(int n, const int* __restrict__ rp,
                                                         const int* __restrict__ ci,
                                                         const float* __restrict__ val,
                                                         const float* __restrict__ x,
                                                         const double* __restrict__ scale, float sigma,
                                                         half_t* __restrict__ vout, float* __restrict__ y,
                                                         const int* __restrict__ done) {
  __shared__ __align__(16) float s_prod[SpmvCfg<float>::kChunk];
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * kSpmvRows;
  const float s = float(*scale);
  float acc[kSpmvRpt];
  if (!spmv_rows<float, true>(n, r0, rp, ci, val, x, s, s_prod, acc, done)) return;
#pragma unroll
  for (int i = 0; i < kSpmvRpt; ++i) {
    const int r = r0 + threadIdx.x + i * kBlock;
    if (r < n) {
      vout[r] = half_t((x[r] * s) * sigma);
      y[r] = acc[i];
    }
  }
}

// Pass 1: h = V_j^T w, lane l of row group grp owning rows 128 grp + 2 l, +1.
template <int K, int NQ>
__global__ __launch_bounds__(kBlock) void hb_dots_kernel(int n, int j, const half_t* __restrict__ V,
                                                         int64_t ldv, const float* __restrict__ w,
                                                         float inv_sigma, double* partial,
                                                         const int* __restrict__ done, int rev) {
  constexpr int KO = Butterfly<K>::KOut;
  if (done && *done) return;
  const int lane = threadIdx.x % kWave;
  const int gw = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const int G = gridDim.x * kWavesPerBlock;
  const int ngrp = (n + 2 * kWave - 1) / (2 * kWave);
  float acc[NQ][KO];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < KO; ++i) acc[q][i] = 0.f;
  for (int it = gw; it < ngrp; it += G) {
    const int grp = rev ? ngrp - 1 - it : it;
    const int r = grp * 2 * kWave + 2 * lane;
    const bool one = r < n;
    const bool full = r + 1 < n;
    // branch-free loads: row r + 1 of a basis column lies inside the column
    // even past n (columns are padded to a multiple of 64 rows); the padding
    // is never written, so its value is replaced by zero, as is w's
    fvec2_t wv = {0.f, 0.f};
    if (one) wv = fvec2_t{w[r], full ? w[r + 1] : 0.f};
    wv *= inv_sigma;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (q * K < j) {
        float a[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
          const int col = q * K + c;
          hvec2_t v = {half_t(0), half_t(0)};
          if (col < j && one) v = *reinterpret_cast<const hvec2_t*>(V + (size_t)col * ldv + r);
          if (!full) v.y = half_t(0);
          a[c] = float(v.x) * wv.x + float(v.y) * wv.y;
        }
        Butterfly<K>::run(a, lane);
#pragma unroll
        for (int i = 0; i < KO; ++i) acc[q][i] += a[i];
      }
    }
  }
  publish_col_partials<K, float, NQ>(acc, j, partial);
}

// Pass-1 update fused with pass-2 dots (j <= K <= 64): w -= V_j h_in, then
// h_out = V_j^T w, with the row pair's j basis values kept in registers.
template <int K>
__global__ __launch_bounds__(kBlock) void hb_update_dots_kernel(int n, int j, const half_t* __restrict__ V,
                                                                int64_t ldv, const float* __restrict__ h_in,
                                                                float inv_sigma, float* __restrict__ w,
                                                                double* partial, const int* __restrict__ done,
                                                                int rev) {
  constexpr int KO = Butterfly<K>::KOut;
  __shared__ float s_h[K];
  if (done && *done) return;
  for (int c = threadIdx.x; c < K; c += kBlock) s_h[c] = (c < j) ? h_in[c] * inv_sigma : 0.f;
  __syncthreads();
  const int lane = threadIdx.x % kWave;
  const int gw = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  const int G = gridDim.x * kWavesPerBlock;
  const int ngrp = (n + 2 * kWave - 1) / (2 * kWave);
  float acc[1][KO];
#pragma unroll
  for (int i = 0; i < KO; ++i) acc[0][i] = 0.f;
  // rev: descending row groups, as in the float32 kernels
  for (int it = gw; it < ngrp; it += G) {
    const int grp = rev ? ngrp - 1 - it : it;
    const int r = grp * 2 * kWave + 2 * lane;
    const bool full = r + 1 < n;
    const bool one = r < n;
    // branch-free loads as in the dots pass (the padding row's values become
    // zero; its update is never stored)
    hvec2_t v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      v[c] = hvec2_t{half_t(0), half_t(0)};
      if (c < j && one) v[c] = *reinterpret_cast<const hvec2_t*>(V + (size_t)c * ldv + r);
      if (!full) v[c].y = half_t(0);
    }
    fvec2_t wv = {0.f, 0.f};
    if (one) wv = fvec2_t{w[r], full ? w[r + 1] : 0.f};
#pragma unroll
    for (int c = 0; c < K; ++c) {
      wv.x -= float(v[c].x) * s_h[c];
      wv.y -= float(v[c].y) * s_h[c];
    }
    if (full) *reinterpret_cast<fvec2_t*>(w + r) = wv;
    else if (one) w[r] = wv.x;
    // convert the packed values again for the dots rather than keep 2K float
    // copies live from the update (which would halve the resident waves)
#pragma unroll
    for (int c = 0; c < K; ++c) {
      unsigned u = __builtin_bit_cast(unsigned, v[c]);
      asm volatile("" : "+v"(u));
      v[c] = __builtin_bit_cast(hvec2_t, u);
    }
    const fvec2_t ws = wv * inv_sigma;
    float a[K];
#pragma unroll
    for (int c = 0; c < K; ++c) a[c] = float(v[c].x) * ws.x + float(v[c].y) * ws.y;
    Butterfly<K>::run(a, lane);
#pragma unroll
    for (int i = 0; i < KO; ++i) acc[0][i] += a[i];
  }
  publish_col_partials<K, float, 1>(acc, j, partial);
}

// w[r..r+3] -= sum_c Vs[c][r..r+3] s_h[c] (s_h already divided by sigma);
// eight-byte loads of four float16 values per column.
__device__ __forceinline__ void hb_update_rows4(int j, const half_t* __restrict__ V, int64_t ldv,
                                                const float* __restrict__ s_h, float* __restrict__ w, int r,
                                                float (&out)[4]) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4 wv = *reinterpret_cast<const f4*>(w + r);
  int c = 0;
  for (; c + 8 <= j; c += 8) {
    hvec4_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const hvec4_t*>(V + (size_t)(c + u) * ldv + r);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float h = s_h[c + u];
      wv.x -= float(v[u].x) * h;
      wv.y -= float(v[u].y) * h;
      wv.z -= float(v[u].z) * h;
      wv.w -= float(v[u].w) * h;
    }
  }
  for (; c < j; ++c) {
    const hvec4_t v = *reinterpret_cast<const hvec4_t*>(V + (size_t)c * ldv + r);
    const float h = s_h[c];
    wv.x -= float(v.x) * h;
    wv.y -= float(v.y) * h;
    wv.z -= float(v.z) * h;
    wv.w -= float(v.w) * h;
  }
  *reinterpret_cast<f4*>(w + r) = wv;
  out[0] = wv.x;
  out[1] = wv.y;
  out[2] = wv.z;
  out[3] = wv.w;
}

__device__ __forceinline__ float hb_update_row(int j, const half_t* __restrict__ V, int64_t ldv,
                                               const float* __restrict__ s_h, float* __restrict__ w, int r) {
  float wv = w[r];
  for (int c = 0; c < j; ++c) wv -= float(V[(size_t)c * ldv + r]) * s_h[c];
  w[r] = wv;
  return wv;
}

// w -= V_j h_in; with NORM, also the block's partial ||w||^2 in partial[blockIdx.x].
// With rev the row quads are taken in descending order.
template <bool NORM>
__global__ __launch_bounds__(kBlock) void hb_update_kernel(int n, int j, const half_t* __restrict__ V,
                                                           int64_t ldv, const float* __restrict__ h_in,
                                                           float inv_sigma, float* __restrict__ w,
                                                           double* partial, const int* __restrict__ done,
                                                           int rev) {
  __shared__ float s_h[kMaxCols];
  if (done && *done) return;
  for (int c = threadIdx.x; c < j; c += kBlock) s_h[c] = h_in[c] * inv_sigma;
  __syncthreads();
  float sq = 0.f;
  const int nq = n / 4;
  float o[4];
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < nq; q += gridDim.x * kBlock) {
    hb_update_rows4(j, V, ldv, s_h, w, 4 * (rev ? nq - 1 - q : q), o);
#pragma unroll
    for (int i = 0; i < 4; ++i) sq += o[i] * o[i];
  }
  for (int r = 4 * nq + blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    const float wv = hb_update_row(j, V, ldv, s_h, w, r);
    sq += wv * wv;
  }
  if constexpr (NORM) {
    sq = block_sum(sq);
    if (threadIdx.x == 0) partial[blockIdx.x] = double(sq);
  }
}

// With a right preconditioner: v_j = x * scale in float32 for the
// preconditioner (out), and half(sigma * v_j) into the basis.
__global__ __launch_bounds__(kBlock) void hb_scale_kernel(int n, const float* __restrict__ x,
                                                          const double* __restrict__ scale, float sigma,
                                                          half_t* __restrict__ vout, float* __restrict__ out,
                                                          const int* __restrict__ done) {
  if (done && *done) return;
  const float s = float(*scale);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const float v = x[i] * s;
    out[i] = v;
    vout[i] = half_t(v * sigma);
  }
}

// u = V_k y formed in float32 (k from the status); then x += gamma * double(u),
// or, when u_out is given, u is stored there (a preconditioner follows).
__global__ __launch_bounds__(kBlock) void hb_solution_update_kernel(int n, const half_t* __restrict__ V,
                                                                    int64_t ldv, const double* __restrict__ y,
                                                                    float inv_sigma, const Status* __restrict__ st,
                                                                    float* __restrict__ u_out,
                                                                    double* __restrict__ x) {
  __shared__ float s_y[kMaxCols];
  const int k = st->k;
  for (int c = threadIdx.x; c < k; c += kBlock) s_y[c] = float(y[c]) * inv_sigma;
  __syncthreads();
  const double gam = st->gamma;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    float s = 0.f;
    for (int c = 0; c < k; ++c) s += float(V[(size_t)c * ldv + r]) * s_y[c];
    if (u_out) u_out[r] = s;
    else x[r] += gam * double(s);
  }
}

}  // namespace gmr
