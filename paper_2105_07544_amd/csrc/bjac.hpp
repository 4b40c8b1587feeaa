// Block Jacobi right preconditioner (§III-D, used in §V-G): M = blockdiag(A)^-1
// with diagonal blocks of `k` consecutive rows (the last one may be shorter).
//
//  * Setup: one block of threads per diagonal block gathers A_bb from the CSR
//    rows into LDS and inverts it by Gauss-Jordan elimination with partial
//    pivoting, in the precision of A (float32 for the float32 copy: computed
//    and applied in float32).  The inverse is stored column-major in a k x k
//    slot per block, padded with zeros.
//  * Apply: y_b = inv_b x_b.  For small blocks (k < 8) a wave serves
//    floor(64 / k) blocks, k lanes per block, lane i forming row i; column c of
//    inv_b is one contiguous read and x_c is broadcast across the block's lanes
//    by a cross-lane shuffle.  For larger blocks a one-wave workgroup owns one
//    block: it copies the k x k slot into LDS with 16-byte loads, a few columns
//    at a time (the slot is one contiguous run, so every load is fully
//    coalesced), and lane i forms row i from LDS.
#pragma once

#include "device_common.hpp"

namespace gmr {

constexpr int kBjacMaxBlock = 64;

template <class T>
__global__ __launch_bounds__(kBlock) void bjac_invert_kernel(int n, int k, const int* __restrict__ rp,
                                                             const int* __restrict__ ci,
                                                             const T* __restrict__ val, T* __restrict__ inv,
                                                             int* __restrict__ singular) {
  __shared__ T s_a[kBjacMaxBlock][kBjacMaxBlock + 1];
  __shared__ T s_i[kBjacMaxBlock][kBjacMaxBlock + 1];
  __shared__ T s_f[kBjacMaxBlock];
  __shared__ int s_piv;
  __shared__ int s_bad;
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * k;
  const int kb = min(k, n - r0);
  for (int e = t; e < kb * kb; e += kBlock) {
    const int i = e / kb, c = e % kb;
    s_a[i][c] = T(0);
    s_i[i][c] = i == c ? T(1) : T(0);
  }
  if (t == 0) s_bad = 0;
  __syncthreads();
  for (int i = t; i < kb; i += kBlock) {
    for (int q = rp[r0 + i]; q < rp[r0 + i + 1]; ++q) {
      const int c = ci[q] - r0;
      if (c >= 0 && c < kb) s_a[i][c] += val[q];
    }
  }
  __syncthreads();
  for (int p = 0; p < kb; ++p) {
    // pivot: the largest |a_ip| for i >= p, the first such row on ties (one wave)
    if (t < kWave) {
      const int i = p + t;
      T v = i < kb ? fabs(s_a[i][p]) : T(-1);
      int at = i;
      for (int off = kWave / 2; off > 0; off >>= 1) {
        const T ov = __shfl_xor(v, off);
        const int oa = __shfl_xor(at, off);
        if (ov > v || (ov == v && oa < at)) {
          v = ov;
          at = oa;
        }
      }
      if (t == 0) {
        s_piv = at;
        if (!(v > T(0)) || !isfinite(v)) s_bad = 1;
      }
    }
    __syncthreads();
    if (s_bad) break;
    const int piv = s_piv;
    if (piv != p) {
      for (int c = t; c < kb; c += kBlock) {
        const T a = s_a[p][c], b = s_i[p][c];
        s_a[p][c] = s_a[piv][c];
        s_i[p][c] = s_i[piv][c];
        s_a[piv][c] = a;
        s_i[piv][c] = b;
      }
    }
    __syncthreads();
    const T d = T(1) / s_a[p][p];
    for (int i = t; i < kb; i += kBlock) s_f[i] = s_a[i][p];
    __syncthreads();
    for (int c = t; c < kb; c += kBlock) {
      s_a[p][c] *= d;
      s_i[p][c] *= d;
    }
    __syncthreads();
    for (int e = t; e < kb * kb; e += kBlock) {
      const int i = e / kb, c = e % kb;
      if (i != p) {
        const T f = s_f[i];
        s_a[i][c] -= f * s_a[p][c];
        s_i[i][c] -= f * s_i[p][c];
      }
    }
    __syncthreads();
  }
  if (s_bad) {
    if (t == 0) singular[0] = 1;
    return;
  }
  T* out = inv + (size_t)blockIdx.x * k * k;
  for (int e = t; e < k * k; e += kBlock) {
    const int c = e / k, i = e % k;
    out[e] = (i < kb && c < kb) ? s_i[i][c] : T(0);
  }
}

// y = blockdiag(inv) x; skipped once the cycle has ended (done set).
template <class T>
__global__ __launch_bounds__(kBlock) void bjac_apply_kernel(int n, int k, const T* __restrict__ inv,
                                                            const T* __restrict__ x, T* __restrict__ y,
                                                            const int* __restrict__ done) {
  if (done && *done) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
  const int bpw = kWave / k;
  const int g = lane / k, i = lane - (lane / k) * k;
  const int nblk = (n + k - 1) / k;
  const int b = wave * bpw + g;
  const bool active = g < bpw && b < nblk;
  const int r0 = b * k;
  const int kb = active ? min(k, n - r0) : 0;
  const bool row = i < kb;
  const T xv = row ? x[r0 + i] : T(0);
  const T* col = inv + (size_t)(active ? b : 0) * k * k + i;
  const int src0 = min(g * k, kWave - 1);
  T acc = T(0);
#pragma unroll 8
  for (int c = 0; c < k; ++c) {
    const T xc = __shfl(xv, min(src0 + c, kWave - 1));
    if (row && c < kb) acc += col[(size_t)c * k] * xc;
  }
  if (row) y[r0 + i] = acc;
}

constexpr int kBjacStagedMin = 8;

// One block per one-wave workgroup; the k x k slot is staged through LDS in
// chunks of `ch` columns (dynamic LDS: ch * k + 64 values of T), so the LDS
// per workgroup stays near 8 KB and many workgroups stay resident per CU: one
// wave's loads overlap another's arithmetic.  ch is even; for even k every
// chunk is a contiguous run of whole 16-byte vectors.
template <class T>
__global__ __launch_bounds__(kWave) void bjac_apply_staged_kernel(int n, int k, int ch, const T* __restrict__ inv,
                                                                  const T* __restrict__ x, T* __restrict__ y,
                                                                  const int* __restrict__ done) {
  extern __shared__ __align__(16) unsigned char bjac_smem[];
  if (done && *done) return;
  const int lane = threadIdx.x;
  T* s_inv = reinterpret_cast<T*>(bjac_smem);
  T* s_x = s_inv + (size_t)ch * k;
  const int b = blockIdx.x;
  const int r0 = b * k;
  const int kb = min(k, n - r0);
  const T* src = inv + (size_t)b * k * k;
  constexpr int V = 16 / sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(16 / sizeof(T))));
  const bool vec = (k % 2) == 0;
  if (lane < kb) s_x[lane] = x[r0 + lane];
  T acc = T(0);
  for (int c0 = 0; c0 < kb; c0 += ch) {
    const int len = min(ch, k - c0) * k;
    const T* cs = src + (size_t)c0 * k;
    if (vec) {
      const vec_t* s4 = reinterpret_cast<const vec_t*>(cs);
      vec_t* d4 = reinterpret_cast<vec_t*>(s_inv);
      for (int e = lane; e < len / V; e += kWave) d4[e] = __builtin_nontemporal_load(s4 + e);
    } else {
      for (int e = lane; e < len; e += kWave) s_inv[e] = cs[e];
    }
    __syncthreads();
    if (lane < kb) {
      const int cols = min(ch, kb - c0);
      for (int c = 0; c < cols; ++c) acc += s_inv[c * k + lane] * s_x[c0 + c];
    }
    __syncthreads();
  }
  if (lane < kb) y[r0 + lane] = acc;
}

}  // namespace gmr
