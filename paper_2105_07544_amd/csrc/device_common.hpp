// Device-side building blocks for gfx950 (CDNA4, wave64): cross-lane
// reductions with DPP / ds_swizzle, a butterfly that reduces many columns at
// once, and the XCD-aware block remap.
//
// Global sums are two-stage: every block of a pass writes its float64
// partials, and a small follow-up kernel adds them in a fixed order.  The
// kernel boundary makes the partials of all eight XCDs visible; an in-kernel
// "last block" protocol would need an agent-scope fence per block, which
// writes back the whole L2 of the block's XCD each time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gmr {

constexpr int kWave = 64;
constexpr int kBlock = 256;               // threads per block for every kernel here
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kNumXcd = 8;                // MI355X: 8 XCDs, blocks dispatched round-robin

// ---------------------------------------------------------------------------
// 32-bit lane moves.  DPP for the in-row patterns, ds_swizzle (bit-mask mode,
// groups of 32 lanes) for xor 4/8/16, ds_bpermute for xor 32.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int S>
__device__ __forceinline__ int xor_lane_i32(int v) {
  static_assert(S == 1 || S == 2 || S == 4 || S == 8 || S == 16 || S == 32, "xor offset");
  if constexpr (S == 1) {
    return dpp_i32<0xB1>(v);                           // quad_perm [1,0,3,2]
  } else if constexpr (S == 2) {
    return dpp_i32<0x4E>(v);                           // quad_perm [2,3,0,1]
  } else if constexpr (S == 32) {
    return __shfl_xor(v, 32, kWave);
  } else {
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (S << 10));  // and 0x1f, or 0, xor S
  }
}

template <int S>
__device__ __forceinline__ float xor_lane(float v) {
  return __builtin_bit_cast(float, xor_lane_i32<S>(__builtin_bit_cast(int, v)));
}

template <int S>
__device__ __forceinline__ double xor_lane(double v) {
  uint64_t b = __builtin_bit_cast(uint64_t, v);
  int lo = xor_lane_i32<S>((int)(uint32_t)b);
  int hi = xor_lane_i32<S>((int)(uint32_t)(b >> 32));
  return __builtin_bit_cast(double, (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32));
}

// Sum over the 64 lanes; every lane receives the total.  The order of the
// additions is fixed, so the result is deterministic.
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  v += xor_lane<1>(v);
  v += xor_lane<2>(v);
  v += xor_lane<4>(v);
  v += xor_lane<8>(v);
  v += xor_lane<16>(v);
  v += xor_lane<32>(v);
  return v;
}

// ---------------------------------------------------------------------------
// Butterfly transpose-reduction.  Each lane holds K per-column values a[0..K)
// (K a power of two, 1..128).  After the call the column sums over all 64
// lanes are spread across the lanes: lane l holds in a[i] (i < KOut) the sum
// of column  col_of(l, i).  For K = 64 that is column l; for K = 128 lane l
// holds columns 2l and 2l+1; for K < 64 each column sum appears on 64/K
// lanes.  It costs K-1 (+ a few) lane moves instead of 6 per column.
// ---------------------------------------------------------------------------
template <int K>
struct Butterfly {
  static constexpr int KOut = (K > 64) ? K / 64 : 1;

  template <class T, int S, int KC>
  __device__ __forceinline__ static void step(T (&a)[K], int lane) {
    if constexpr (S >= 1) {
      if constexpr (KC > KOut) {
        constexpr int H = KC / 2;
        const bool up = (lane & S) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
          T send = up ? a[i] : a[i + H];
          T keep = up ? a[i + H] : a[i];
          a[i] = keep + xor_lane<S>(send);
        }
        step<T, S / 2, H>(a, lane);
      } else {
#pragma unroll
        for (int i = 0; i < KC; ++i) a[i] += xor_lane<S>(a[i]);
        step<T, S / 2, KC>(a, lane);
      }
    }
  }

  template <class T>
  __device__ __forceinline__ static void run(T (&a)[K], int lane) {
    step<T, 32, K>(a, lane);
  }

  // Column whose sum lane `lane` holds in a[i] after run().
  __device__ __forceinline__ static int col_of(int lane, int i) {
    int col = 0;
    int kc = K;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      if (kc > KOut) {
        kc >>= 1;
        if (lane & s) col += kc;
      }
    }
    return col + i;
  }

  // True on exactly one of the lanes that hold the same column sums.
  __device__ __forceinline__ static bool owner(int lane) {
    int dup_bits = 0;
    int kc = K;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      if (kc > KOut) kc >>= 1;
      else dup_bits |= s;
    }
    return (lane & dup_bits) == 0;
  }
};

// ---------------------------------------------------------------------------
// XCD-aware block order.  The hardware hands block b to XCD b % 8; this maps
// it to a logical block so that every XCD works on one contiguous range of
// rows (better reuse of gathered x entries in that XCD's L2).  A bijection on
// [0, nb).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int xcd = b % kNumXcd;
  const int local = b / kNumXcd;
  const int q = nb / kNumXcd;
  const int rem = nb % kNumXcd;
  return xcd * q + (xcd < rem ? xcd : rem) + local;
}

// Block-wide sum of one value per thread; result valid on every thread.
template <class T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T s_part[kWavesPerBlock];
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) s_part[wave] = v;
  __syncthreads();
  T t = s_part[0];
#pragma unroll
  for (int i = 1; i < kWavesPerBlock; ++i) t += s_part[i];
  return t;
}

}  // namespace gmr
