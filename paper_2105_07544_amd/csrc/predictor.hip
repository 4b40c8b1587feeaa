// Learned parameter predictor: cheap matrix statistics on the GPU, and the
// forward pass, backward pass and Adam step of a 16-64-64-11 MLP whose three
// heads choose the restart length, the polynomial degree and the inner
// precision of GMRES-IR.  The paper gives guidance for these choices from
// its experiments (§V-E restart length, §V-C and §V-F polynomial degree,
// §V-B inner precision); the network learns it from solver runs instead.
//
// The network is tiny (5,963 parameters), so one block of 64 threads (one
// per hidden unit) handles one sample in the forward and backward passes;
// per-sample gradients are then added in sample order (deterministic), and
// Adam runs element-wise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/gmres_ir.h"
#include "device_common.hpp"
#include "host_common.hpp"

namespace gmr {
namespace mlp {

constexpr int IN = 16, H1 = 64, H2 = 64, OUT = 11;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H1 * IN, OFF_W2 = OFF_B1 + H1, OFF_B2 = OFF_W2 + H2 * H1,
              OFF_W3 = OFF_B2 + H2, OFF_B3 = OFF_W3 + OUT * H2, NPARAM = OFF_B3 + OUT;
constexpr int ACT = IN + H1 + H2;  // saved per sample: z0, a1, a2 (pre-activations)

__device__ __forceinline__ int head_off(int h) { return h == 0 ? 0 : (h == 1 ? 4 : 9); }
__device__ __forceinline__ int head_size(int h) { return h == 0 ? 4 : (h == 1 ? 5 : 2); }

// Forward pass of sample blockIdx.x: logits (and the saved activations).
__global__ __launch_bounds__(64) void mlp_forward_kernel(const float* __restrict__ th,
                                                         const float* __restrict__ X,
                                                         const float* __restrict__ mu,
                                                         const float* __restrict__ sd, int B,
                                                         float* __restrict__ logits,
                                                         float* __restrict__ act) {
  __shared__ float z0[IN], h1[H1], h2[H2];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  if (b >= B) return;
  if (t < IN) z0[t] = (X[b * IN + t] - mu[t]) / sd[t];
  __syncthreads();
  float a1 = th[OFF_B1 + t];
  for (int k = 0; k < IN; ++k) a1 += th[OFF_W1 + t * IN + k] * z0[k];
  h1[t] = a1 > 0.f ? a1 : 0.f;
  __syncthreads();
  float a2 = th[OFF_B2 + t];
  for (int k = 0; k < H1; ++k) a2 += th[OFF_W2 + t * H1 + k] * h1[k];
  h2[t] = a2 > 0.f ? a2 : 0.f;
  __syncthreads();
  if (t < OUT) {
    float o = th[OFF_B3 + t];
    for (int k = 0; k < H2; ++k) o += th[OFF_W3 + t * H2 + k] * h2[k];
    logits[b * OUT + t] = o;
  }
  if (act) {
    float* a = act + (size_t)b * ACT;
    if (t < IN) a[t] = z0[t];
    a[IN + t] = a1;
    a[IN + H1 + t] = a2;
  }
}

// Backward pass of sample blockIdx.x for the mean over B samples of the summed
// head cross-entropies: the sample's gradient into gs[b][NPARAM] and its loss.
__global__ __launch_bounds__(64) void mlp_backward_kernel(const float* __restrict__ th,
                                                          const float* __restrict__ act,
                                                          const float* __restrict__ logits,
                                                          const int* __restrict__ labels, int B,
                                                          float* __restrict__ gs,
                                                          float* __restrict__ lossv) {
  __shared__ float z0[IN], a1[H1], a2[H2], dl[OUT], da2[H2], da1[H1], s_l[3];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  if (b >= B) return;
  const float* a = act + (size_t)b * ACT;
  if (t < IN) z0[t] = a[t];
  a1[t] = a[IN + t];
  a2[t] = a[IN + H1 + t];
  if (t < 3) {
    // softmax cross-entropy of head t
    const int o = head_off(t), k = head_size(t);
    const float* z = logits + b * OUT + o;
    float zmax = z[0];
    for (int i = 1; i < k; ++i) zmax = fmaxf(zmax, z[i]);
    float se = 0.f;
    for (int i = 0; i < k; ++i) se += expf(z[i] - zmax);
    const int y = min(max(labels[b * 3 + t], 0), k - 1);  // out-of-range labels are clamped
    for (int i = 0; i < k; ++i) dl[o + i] = (expf(z[i] - zmax) / se - (i == y ? 1.f : 0.f)) / B;
    s_l[t] = logf(se) - (z[y] - zmax);
  }
  __syncthreads();
  if (t == 0) lossv[b] = s_l[0] + s_l[1] + s_l[2];
  float* g = gs + (size_t)b * NPARAM;
  // output layer
  const float h2t = a2[t] > 0.f ? a2[t] : 0.f;
  for (int o = 0; o < OUT; ++o) g[OFF_W3 + o * H2 + t] = dl[o] * h2t;
  if (t < OUT) g[OFF_B3 + t] = dl[t];
  float dh2 = 0.f;
  for (int o = 0; o < OUT; ++o) dh2 += dl[o] * th[OFF_W3 + o * H2 + t];
  da2[t] = a2[t] > 0.f ? dh2 : 0.f;
  __syncthreads();
  // second hidden layer
  const float h1t = a1[t] > 0.f ? a1[t] : 0.f;
  for (int j = 0; j < H2; ++j) g[OFF_W2 + j * H1 + t] = da2[j] * h1t;
  g[OFF_B2 + t] = da2[t];
  float dh1 = 0.f;
  for (int j = 0; j < H2; ++j) dh1 += da2[j] * th[OFF_W2 + j * H1 + t];
  da1[t] = a1[t] > 0.f ? dh1 : 0.f;
  __syncthreads();
  // first hidden layer
  for (int k = 0; k < IN; ++k) g[OFF_W1 + t * IN + k] = da1[t] * z0[k];
  g[OFF_B1 + t] = da1[t];
}

// grad[p] = sum over samples (in sample order) of gs[b][p]; loss = mean of lossv.
__global__ __launch_bounds__(kBlock) void mlp_reduce_kernel(const float* __restrict__ gs, int B,
                                                            const float* __restrict__ lossv,
                                                            float* __restrict__ grad,
                                                            float* __restrict__ loss) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p < NPARAM) {
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += gs[(size_t)b * NPARAM + p];
    grad[p] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    float l = 0.f;
    for (int b = 0; b < B; ++b) l += lossv[b];
    *loss = l / B;
  }
}

// Adam (Kingma & Ba) with bias correction, element-wise.
__global__ __launch_bounds__(kBlock) void mlp_adam_kernel(float* __restrict__ th,
                                                          const float* __restrict__ g,
                                                          float* __restrict__ m,
                                                          float* __restrict__ v, int n, float lr,
                                                          float b1, float b2, float eps, float c1,
                                                          float c2) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= n) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  th[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

}  // namespace mlp

// ---------------------------------------------------------------------------
// Matrix statistics: one pass over the CSR rows.  Per block partials of
//  0 sum |a_ii| / sum_{j != i} |a_ij|   (diagonal dominance ratio, rows with
//                                          off-diagonal entries)
//  1 min of that ratio     2 rows with ratio >= 1   3 rows with off-diagonals
//  4 min (a_ii - r_i)      5 max (a_ii + r_i)       6 max r_i      7 max |a_ii|
//  8 sum a_ii              9 sum a_ii^2            10 max nnz in a row
// 11 ||A||_F^2            12 sum (a_ij - a_ji)^2 (a_ji found by binary search
//                            in row j: columns must ascend within a row)
// ---------------------------------------------------------------------------
namespace feat {
constexpr int NS = 13;

template <class T>
__global__ __launch_bounds__(kBlock) void stats_kernel(int n, const int* __restrict__ rp,
                                                       const int* __restrict__ ci,
                                                       const T* __restrict__ val,
                                                       double* __restrict__ part) {
  __shared__ double s[NS][kBlock];
  double acc[NS];
  acc[0] = 0; acc[1] = INFINITY; acc[2] = 0; acc[3] = 0; acc[4] = INFINITY; acc[5] = -INFINITY;
  acc[6] = 0; acc[7] = 0; acc[8] = 0; acc[9] = 0; acc[10] = 0; acc[11] = 0; acc[12] = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double d = 0.0, r = 0.0, f = 0.0, ns = 0.0;
    const int k0 = rp[i], k1 = rp[i + 1];
    for (int k = k0; k < k1; ++k) {
      const int j = ci[k];
      const double v = double(val[k]);
      f += v * v;
      if (j == i) {
        d = v;
      } else {
        r += fabs(v);
        // a_ji by binary search in row j; when row j stores no a_ji, the
        // unstored entry (j, i) of A - A^T contributes a_ij^2 as well
        int lo = rp[j], hi = rp[j + 1] - 1;
        double vt = 0.0;
        bool found = false;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int cm = ci[mid];
          if (cm == i) { vt = double(val[mid]); found = true; break; }
          if (cm < i) lo = mid + 1; else hi = mid - 1;
        }
        ns += found ? (v - vt) * (v - vt) : 2.0 * v * v;
      }
    }
    if (r > 0.0) {
      const double q = fabs(d) / r;
      acc[0] += q;
      acc[1] = fmin(acc[1], q);
      acc[2] += q >= 1.0 ? 1.0 : 0.0;
      acc[3] += 1.0;
    }
    acc[4] = fmin(acc[4], d - r);
    acc[5] = fmax(acc[5], d + r);
    acc[6] = fmax(acc[6], r);
    acc[7] = fmax(acc[7], fabs(d));
    acc[8] += d;
    acc[9] += d * d;
    acc[10] = fmax(acc[10], double(k1 - k0));
    acc[11] += f;
    acc[12] += ns;
  }
  for (int q = 0; q < NS; ++q) s[q][threadIdx.x] = acc[q];
  __syncthreads();
  if (threadIdx.x < NS) {
    const int q = threadIdx.x;
    double v = s[q][0];
    for (int t = 1; t < kBlock; ++t) {
      const double w = s[q][t];
      if (q == 1 || q == 4) v = fmin(v, w);
      else if (q == 5 || q == 6 || q == 7 || q == 10) v = fmax(v, w);
      else v += w;
    }
    part[blockIdx.x * NS + q] = v;
  }
}

__global__ void stats_finish_kernel(int nparts, const double* __restrict__ part, double* out) {
  const int q = threadIdx.x;
  if (q >= NS) return;
  double v = part[q];
  for (int b = 1; b < nparts; ++b) {
    const double w = part[b * NS + q];
    if (q == 1 || q == 4) v = fmin(v, w);
    else if (q == 5 || q == 6 || q == 7 || q == 10) v = fmax(v, w);
    else v += w;
  }
  out[q] = v;
}
// Steps of the Arnoldi run whose Ritz values enter the features (at most n).
constexpr int kArnoldiSteps = 5;

// The 16 features from the 13 row statistics (matrix_stats order), the
// (k+1) x k Hessenberg matrix H of the k-step Arnoldi run (column-major, ld k+1)
// and the Ritz values theta (eigenvalues of its leading k x k block):
//  0 log10 n            1 nonzeros per row        2 max nonzeros in a row
//  3 min dominance      4 mean dominance          5 dominant-row fraction
//  6-8 Gershgorin min (a_ii - r_i), max (a_ii + r_i), max r_i, each over max |a_ii|
//  9 ||A - A^T||_F / ||A||_F                      10 std / |mean| of the diagonal
// 11 max |theta|, 12 min |theta| (over max |a_ii|), 13 log10 of their ratio,
// 14 max |Im theta| / max |theta|, 15 h_{k+1,k} / max |theta|.
// Dominance is |a_ii| / sum_{j != i} |a_ij| over rows with off-diagonal
// entries (10 when there are none).  Non-finite values become 0, +1e6, -1e6.
inline void features_from(int n, int nnz, const double* s, int k, const double* H, const double* re,
                          const double* im, double* f) {
  const double maxd = std::max(s[7], 1e-300);
  const double rows_off = std::max(s[3], 1.0);
  const double mean_d = s[8] / n;
  const double var_d = std::max(s[9] / n - mean_d * mean_d, 0.0);
  double amax = 0.0, amin = INFINITY, imax = 0.0;
  for (int i = 0; i < k; ++i) {
    const double a = std::hypot(re[i], im[i]);
    amax = std::max(amax, a);
    amin = std::min(amin, a);
    imax = std::max(imax, std::fabs(im[i]));
  }
  f[0] = std::log10((double)n);
  f[1] = (double)nnz / n;
  f[2] = s[10];
  f[3] = s[3] > 0 ? s[1] : 10.0;
  f[4] = s[0] / rows_off;
  f[5] = s[2] / n;
  f[6] = s[4] / maxd;
  f[7] = s[5] / maxd;
  f[8] = s[6] / maxd;
  f[9] = std::sqrt(s[12] / std::max(s[11], 1e-300));
  f[10] = std::sqrt(var_d) / std::max(std::fabs(mean_d), 1e-300);
  f[11] = amax / maxd;
  f[12] = amin / maxd;
  f[13] = std::log10(amax / std::max(amin, 1e-300));
  f[14] = imax / amax;
  f[15] = H[(size_t)(k - 1) * (k + 1) + k] / amax;
  for (int i = 0; i < 16; ++i) {
    if (std::isnan(f[i])) f[i] = 0.0;
    else if (std::isinf(f[i])) f[i] = f[i] > 0 ? 1e6 : -1e6;
  }
}

}  // namespace feat
}  // namespace gmr

using namespace gmr;

namespace {
gmr_status lchk(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return gmr::fail(GMR_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return GMR_OK;
}
}  // namespace

extern "C" {

int32_t mlp_param_count(void) { return mlp::NPARAM; }

size_t mlp_workspace_bytes(int32_t batch) {
  if (batch <= 0) return 0;
  return (size_t)batch * (mlp::NPARAM + mlp::ACT + mlp::OUT + 1) * sizeof(float);
}

gmr_status mlp_forward(const float* params, const float* X, const float* mu, const float* sigma,
                       int32_t batch, float* logits, void* stream) {
  if (!params || !X || !mu || !sigma || !logits || batch <= 0)
    return gmr::fail(GMR_ERR_INVALID, "mlp_forward: bad arguments");
  mlp::mlp_forward_kernel<<<batch, 64, 0, (hipStream_t)stream>>>(params, X, mu, sigma, batch, logits, nullptr);
  return lchk("mlp_forward_kernel");
}

gmr_status mlp_loss_grad(const float* params, const float* X, const float* mu, const float* sigma,
                         const int32_t* labels, int32_t batch, float* grad, float* loss, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!params || !X || !mu || !sigma || !labels || !grad || batch <= 0)
    return gmr::fail(GMR_ERR_INVALID, "mlp_loss_grad: bad arguments");
  if (!ws || ws_bytes < mlp_workspace_bytes(batch)) return gmr::fail(GMR_ERR_WORKSPACE, "mlp_loss_grad: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  float* gs = (float*)ws;
  float* act = gs + (size_t)batch * mlp::NPARAM;
  float* logits = act + (size_t)batch * mlp::ACT;
  float* lossv = logits + (size_t)batch * mlp::OUT;
  mlp::mlp_forward_kernel<<<batch, 64, 0, s>>>(params, X, mu, sigma, batch, logits, act);
  gmr_status st = lchk("mlp_forward_kernel");
  if (st != GMR_OK) return st;
  mlp::mlp_backward_kernel<<<batch, 64, 0, s>>>(params, act, logits, labels, batch, gs, lossv);
  if ((st = lchk("mlp_backward_kernel")) != GMR_OK) return st;
  mlp::mlp_reduce_kernel<<<(mlp::NPARAM + kBlock - 1) / kBlock, kBlock, 0, s>>>(gs, batch, lossv, grad, loss);
  return lchk("mlp_reduce_kernel");
}

gmr_status mlp_adam_step(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                         float beta1, float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1) return gmr::fail(GMR_ERR_INVALID, "mlp_adam_step: bad arguments");
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  mlp::mlp_adam_kernel<<<(mlp::NPARAM + kBlock - 1) / kBlock, kBlock, 0, (hipStream_t)stream>>>(
      params, grad, m, v, mlp::NPARAM, lr, beta1, beta2, eps, c1, c2);
  return lchk("mlp_adam_kernel");
}

gmr_status matrix_stats(const gmr_csr* A, double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!A || !out || A->n <= 0 || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return gmr::fail(GMR_ERR_INVALID, "matrix_stats: bad arguments");
  const int G = std::min((A->n + kBlock - 1) / kBlock, 1024);
  const size_t need = (size_t)(G + 1) * feat::NS * sizeof(double);
  if (!ws || ws_bytes < need) return gmr::fail(GMR_ERR_WORKSPACE, "matrix_stats: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  double* part = (double*)ws;
  double* res = part + (size_t)G * feat::NS;
  if (A->dtype == GMR_F64)
    feat::stats_kernel<double><<<G, kBlock, 0, s>>>(A->n, A->row_ptr, A->col_idx, (const double*)A->val, part);
  else
    feat::stats_kernel<float><<<G, kBlock, 0, s>>>(A->n, A->row_ptr, A->col_idx, (const float*)A->val, part);
  gmr_status st = lchk("stats_kernel");
  if (st != GMR_OK) return st;
  feat::stats_finish_kernel<<<1, 64, 0, s>>>(G, part, res);
  if ((st = lchk("stats_finish_kernel")) != GMR_OK) return st;
  if (hipMemcpyAsync(out, res, feat::NS * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return gmr::fail(GMR_ERR_HIP, "matrix_stats: copy failed");
  return GMR_OK;
}

size_t matrix_features_workspace_bytes(int32_t n, int32_t dtype) {
  if (n <= 0 || (dtype != GMR_F32 && dtype != GMR_F64)) return 0;
  const gmr_params p{feat::kArnoldiSteps, 1e-10, 1, 0, 0, 0, 0};
  const size_t arnoldi = gmres_workspace_bytes(n, &p, dtype, 0);
  const size_t stats = (size_t)(std::min((n + kBlock - 1) / kBlock, 1024) + 1) * feat::NS * sizeof(double);
  return std::max(arnoldi, stats);
}

gmr_status matrix_features(const gmr_csr* A, const void* v0, double* out, void* ws, size_t ws_bytes,
                           void* stream) {
  if (!A || !v0 || !out) return gmr::fail(GMR_ERR_INVALID, "matrix_features: null pointer");
  if (A->n <= 0 || (A->dtype != GMR_F32 && A->dtype != GMR_F64))
    return gmr::fail(GMR_ERR_INVALID, "matrix_features: bad matrix");
  if (!ws || ws_bytes < matrix_features_workspace_bytes(A->n, A->dtype))
    return gmr::fail(GMR_ERR_WORKSPACE, "matrix_features: workspace too small");
  double st[feat::NS];
  gmr_status rc = matrix_stats(A, st, ws, ws_bytes, stream);
  if (rc != GMR_OK) return rc;
  // the Arnoldi run of a degree-(steps-1) polynomial setup: its Hessenberg matrix
  gmr_poly* P = nullptr;
  rc = poly_prec_setup(A, std::min(feat::kArnoldiSteps, A->n) - 1, v0, ws, ws_bytes, &P, stream);
  if (rc != GMR_OK) return rc;
  const int k = poly_prec_degree(P) + 1;  // fewer steps after a lucky breakdown
  std::vector<double> H((size_t)(k + 1) * k), Hk((size_t)k * k), re(k), im(k);
  rc = poly_prec_hessenberg(P, H.data());
  poly_prec_destroy(P);
  if (rc != GMR_OK) return rc;
  for (int c = 0; c < k; ++c)
    for (int r = 0; r < k; ++r) Hk[(size_t)c * k + r] = H[(size_t)c * (k + 1) + r];
  if ((rc = gmr_hessenberg_eigvals(k, Hk.data(), re.data(), im.data())) != GMR_OK) return rc;
  feat::features_from(A->n, A->nnz, st, k, H.data(), re.data(), im.data(), out);
  return GMR_OK;
}

}  // extern "C"
