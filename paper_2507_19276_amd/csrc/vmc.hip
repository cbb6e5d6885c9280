// Kernels of one VMC step (Sec. 2.1 Eq. (7); Sec. 2.3 Eq. (19); AdamW):
// the reweighted gradient's cotangent over the unique samples and the AdamW
// update of the packed parameters.  Both reduce in a fixed order, so a step
// is bit-reproducible.
#include "internal.h"
#include <cmath>

namespace nqs {
namespace {

constexpr int kBlock = 1024;

// block-wide sum in a fixed order (strided partial sums, then a tree in LDS)
__device__ double block_sum(double x, double* sh) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void k_i64_to_f64(int64_t n, const int64_t* a, double* b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) b[i] = double(a[i]);
}

// one workgroup: S = sum c |f|^2, E = sum c Etilde_num / S,
// cot_n = 2 c_n (Etilde_num(n) - |f_n|^2 E) / S; out = {E, S}
__global__ __launch_bounds__(kBlock) void k_vmc_cotangent(int64_t N, const double* c, const double* etnum,
                                                          const double* fsq, double* cot, double* out) {
  __shared__ double sh[kBlock];
  double a = 0.0, b = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += kBlock) {
    a += c[n] * fsq[n];
    b += c[n] * etnum[n];
  }
  const double S = block_sum(a, sh);
  const double T = block_sum(b, sh);
  const double E = T / S;
  for (int64_t n = threadIdx.x; n < N; n += kBlock) cot[n] = 2.0 * c[n] * (etnum[n] - fsq[n] * E) / S;
  if (threadIdx.x == 0) {
    out[0] = E;
    out[1] = S;
  }
}

// complex parameters: E from Re Etilde_num, cot from Re, cotp_n =
// 2 c_n Im Etilde_num(n) / S (the phase cotangent of 2 Re <(E_loc - E)^* d ln Psi>)
__global__ __launch_bounds__(kBlock) void k_vmc_cotangent_cx(int64_t N, const double* c, const double* etnum,
                                                             const double* etnum_im, const double* fsq,
                                                             double* cot, double* cotp, double* out) {
  __shared__ double sh[kBlock];
  double a = 0.0, b = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += kBlock) {
    a += c[n] * fsq[n];
    b += c[n] * etnum[n];
  }
  const double S = block_sum(a, sh);
  const double T = block_sum(b, sh);
  const double E = T / S;
  for (int64_t n = threadIdx.x; n < N; n += kBlock) {
    cot[n] = 2.0 * c[n] * (etnum[n] - fsq[n] * E) / S;
    cotp[n] = 2.0 * c[n] * etnum_im[n] / S;
  }
  if (threadIdx.x == 0) {
    out[0] = E;
    out[1] = S;
  }
}

// AdamW with decoupled weight decay (the formulation of PyTorch's AdamW)
__global__ void k_adamw(int64_t n, double* p, const double* g, double* m, double* v, double lr, double b1, double b2,
                        double eps, double wd, double c1, double c2) {
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double gk = g[k];
  double pk = p[k] * (1.0 - lr * wd);
  const double mk = b1 * m[k] + (1.0 - b1) * gk;
  const double vk = b2 * v[k] + (1.0 - b2) * gk * gk;
  pk -= lr * (mk / c1) / (sqrt(vk / c2) + eps);
  p[k] = pk;
  m[k] = mk;
  v[k] = vk;
}

// projection onto eta >= 0: one workgroup per site, one thread per unit; a
// NaN stays NaN (the re-bind then refuses it)
__global__ void k_project_eta(int chi, const int64_t* off, double* p) {
  const int u = threadIdx.x;
  if (u >= chi) return;
  double* e = p + off[blockIdx.x] + u;
  if (*e < 0.0) *e = 0.0;
}

// one workgroup: out = sum g^2
__global__ __launch_bounds__(kBlock) void k_sumsq(int64_t n, const double* g, double* out) {
  __shared__ double sh[kBlock];
  double a = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += kBlock) a += g[k] * g[k];
  const double s = block_sum(a, sh);
  if (threadIdx.x == 0) *out = s;
}

inline unsigned blocks_for(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

hipError_t launch_i64_to_f64(int64_t n, const int64_t* a, double* b, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_i64_to_f64, dim3(blocks_for(n)), dim3(256), 0, st, n, a, b);
  return hipGetLastError();
}

hipError_t launch_vmc_cotangent(int64_t N, const double* c, const double* etnum, const double* fsq, double* cot,
                                double* out, hipStream_t st) {
  if (N <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vmc_cotangent, dim3(1), dim3(kBlock), 0, st, N, c, etnum, fsq, cot, out);
  return hipGetLastError();
}

hipError_t launch_vmc_cotangent_cx(int64_t N, const double* c, const double* etnum, const double* etnum_im,
                                   const double* fsq, double* cot, double* cotp, double* out, hipStream_t st) {
  if (N <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_vmc_cotangent_cx, dim3(1), dim3(kBlock), 0, st, N, c, etnum, etnum_im, fsq, cot, cotp, out);
  return hipGetLastError();
}

hipError_t launch_adamw(int64_t n, double* p, const double* g, double* m, double* v, int64_t t, double lr, double b1,
                        double b2, double eps, double wd, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const double c1 = 1.0 - std::pow(b1, double(t)), c2 = 1.0 - std::pow(b2, double(t));
  hipLaunchKernelGGL(k_adamw, dim3(blocks_for(n)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps, wd, c1, c2);
  return hipGetLastError();
}

hipError_t launch_project_eta(int K, int chi, const int64_t* off, double* p, hipStream_t st) {
  if (K <= 0 || chi <= 0 || chi > 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_project_eta, dim3(K), dim3(chi), 0, st, chi, off, p);
  return hipGetLastError();
}

hipError_t launch_sumsq(int64_t n, const double* g, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(1), dim3(kBlock), 0, st, n, g, out);
  return hipGetLastError();
}

}  // namespace nqs
