// Energy side of the local energy on gfx950 (arXiv:2507.19276):
//   * the cos-RBM correlator (Sec. 2.3, Eq. (15)) and the Ising-RBM
//     correlator (Eq. (16));
//   * the per-sample local-energy reduction (Eqs. (6), (18), (22)) and the
//     batch sums of Sec. 2.3.
#include "internal.h"
#include <algorithm>
#include <cmath>

namespace nqs {
namespace {

__device__ inline double tlog(double x) { return log(x); }
__device__ inline float tlog(float x) { return logf(x); }

// ---------------------------------------------------------------------------
// cos-RBM correlator
// ---------------------------------------------------------------------------

__device__ inline bool bit_at(uint64_t lo, uint64_t hi, int P) {
  return P < 64 ? ((lo >> P) & 1ull) : ((hi >> (P - 64)) & 1ull);
}

// theta_k(n) = b_k + sum_P W_kP x_P, one thread per (sample, k)
__global__ void k_corr_theta(CorrParams C, const uint64_t* samples, int64_t N, double* theta) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= N * C.nh) return;
  const int64_t n = t / C.nh;
  const int k = int(t % C.nh);
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  const int nv = 2 * C.K;
  double th = C.b[k];
  for (int P = 0; P < nv; ++P)
    if (bit_at(lo, hi, P)) th += C.W[size_t(k) * nv + P];
  theta[t] = th;
}

__device__ inline double tcos(double x) { return cos(x); }
__device__ inline float tcos(float x) { return cosf(x); }
__device__ inline double tabs(double x) { return fabs(x); }
__device__ inline float tabs(float x) { return fabsf(x); }

// cos in FP64 for |x| < 2^20 as a sine: x = (2q+1) pi/2 + r with |r| <= pi/2
// by a Cody-Waite reduction with a two-constant FMA split of pi/2 (the first
// FMA is exact, so r carries an absolute error near 2^-105 |q|), and
// cos x = (-1)^(q+1) sin r with sin r from its Taylor series to r^21 (the
// truncation term stays below 2^-59): r + r z (-1/6 + z P(z)), z = r^2, the
// high-order terms of P by pairs.  Within 2 ulp of the true cosine and within
// 2.3e-16 relative, also near its zeros (where r is small), against a
// long-double cosine on the host.  Larger or non-finite arguments take the
// library cosine.
__device__ inline double cos_cw(double x) {
  if (!(fabs(x) < 1048576.0)) return cos(x);
  const double q = floor(x * 0.31830988618379067154);
  const double q2 = fma(2.0, q, 1.0);
  double r = fma(-q2, 1.5707963267948966, x);
  r = fma(-q2, 6.123233995736766e-17, r);
  const double z = r * r, z2 = z * z, z4 = z2 * z2;
  const double p23 = fma(-1.0 / 5040.0, z, 1.0 / 120.0);
  const double p45 = fma(-1.0 / 39916800.0, z, 1.0 / 362880.0);
  const double p67 = fma(-1.0 / 1307674368000.0, z, 1.0 / 6227020800.0);
  const double p89 = fma(-1.0 / 121645100408832000.0, z, 1.0 / 355687428096000.0);
  const double p810 = fma(1.0 / 51090942171709440000.0, z2, p89);
  const double P = fma(fma(p810, z2, p67), z4, fma(p45, z2, p23));
  const double sn = fma(r * z, fma(P, z, -1.0 / 6.0), r);
  return (int(q) & 1) ? sn : -sn;
}

// The same in FP32 for |x| < 2^15 (a two-constant FMA split of pi/2 in FP32,
// sin r to r^13: the truncation term stays below 2^-30): within 1.9 x 2^-24
// absolute of the true cosine of the FP32 argument, against an FP64 cosine
// on the host.  Larger or non-finite arguments take the library cosine.
__device__ inline float cos_cw(float x) {
  if (!(fabsf(x) < 32768.0f)) return cosf(x);
  const float q = floorf(x * 0.318309886f);
  const float q2 = fmaf(2.0f, q, 1.0f);
  float r = fmaf(-q2, 1.57079637f, x);
  r = fmaf(-q2, -4.37113883e-8f, r);
  const float z = r * r;
  float p = fmaf(1.0f / 6227020800.0f, z, -1.0f / 39916800.0f);
  p = fmaf(p, z, 1.0f / 362880.0f);
  p = fmaf(p, z, -1.0f / 5040.0f);
  p = fmaf(p, z, 1.0f / 120.0f);
  const float sn = fmaf(r * z, fmaf(p, z, -1.0f / 6.0f), r);
  return (int(q) & 1) ? sn : -sn;
}

// theta(m) = theta(n) + sum_{created P} W_:P - sum_{annihilated P} W_:P; one
// thread per row, theta in FP64.  The cosines are multiplied in FP64 with a
// power of two split off every 8 factors (|cos| of a rounded angle stays far
// above 2^-128, so 8 factors cannot underflow), and one FP64 log per row:
// log |prod_k cos| = log |mantissa| + exponent log 2.  The FP32 form takes
// each cosine in FP32 from theta rounded to FP32 (the form the FP32 error
// bound is stated for: the product and the log add only FP64 roundings).
//
// A row of the local energy differs from its sample by at most two created
// and two annihilated spin orbitals, and their weights are read without
// branches: an absent change reads a zero (theta + 0 is theta), and the loads
// of hidden unit k + 1 are issued before the cosine of unit k.  With LDS, a
// persistent workgroup per CU stages W as [k][2K + 1] with a zero last column
// (the index of an absent change), so the only vector-memory load per hidden
// unit is theta(n); without (W too large for LDS), W is read through a buffer
// resource where an absent change takes the offset of W's end, which the range
// check turns into a zero read.  Other rows take a plain loop over the changed
// orbitals.
template <typename T>
struct CorrAcc {
  double pm = 1.0;
  int pe = 0;
  __device__ void add(double th) { pm *= double(cos_cw(T(th))); }
  __device__ void split() {
    int e;
    pm = frexp(pm, &e);
    pe += e;
  }
  __device__ void finish(double& lfo, int8_t& sfo) {
    int e;
    const double m = frexp(pm, &e);
    lfo = log(fabs(m)) + double(pe + e) * 0.69314718055994530942;
    sfo = int8_t(m < 0.0 ? -1 : 1);
  }
};

__device__ inline int low_bit(uint64_t lo, uint64_t hi) {
  return lo ? __ffsll((unsigned long long)lo) - 1 : 64 + __ffsll((unsigned long long)hi) - 1;
}

constexpr int kCorrLdsThreads = 1024;
constexpr size_t kCorrLdsMax = 128 * 1024;   // largest LDS copy of W

template <typename T, bool LDS>
__global__ __launch_bounds__(LDS ? kCorrLdsThreads : 256) void k_corr_rows(
    CorrParams C, const uint64_t* m, const int32_t* owner, const uint64_t* samples, const double* theta, int64_t R,
    double* lf, int8_t* sf) {
  extern __shared__ double wl[];
  const int nv = 2 * C.K, nh = C.nh, ws = nv + 1;
  if constexpr (LDS) {
    for (int u = threadIdx.x; u < nh * ws; u += blockDim.x) {
      const int k = u / ws, P = u - k * ws;
      wl[u] = P < nv ? C.W[size_t(k) * nv + P] : 0.0;
    }
    __syncthreads();
  }
  const uint32_t wbytes = uint32_t(nh) * uint32_t(nv) * 8u;
  const __amdgpu_buffer_rsrc_t wr =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(C.W), short(0), int(wbytes), 0x00020000);
  const int64_t step = LDS ? int64_t(gridDim.x) * blockDim.x : R;
  for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < R; r += step) {
    const int64_t o = owner[r];
    const uint64_t mlo = m[2 * r], mhi = m[2 * r + 1];
    const uint64_t nlo = samples[2 * o], nhi = samples[2 * o + 1];
    uint64_t alo = mlo & ~nlo, ahi = mhi & ~nhi, rlo = nlo & ~mlo, rhi = nhi & ~mhi;
    const int na = __popcll(alo) + __popcll(ahi), nr = __popcll(rlo) + __popcll(rhi);
    const double* th0 = theta + o * nh;
    CorrAcc<T> A;
    if (na > 2 || nr > 2) {
      for (int k = 0; k < nh; ++k) {
        double th = th0[k];
        for (uint64_t x = alo, y = ahi; x | y;) {
          th += C.W[size_t(k) * nv + low_bit(x, y)];
          if (x) x &= x - 1; else y &= y - 1;
        }
        for (uint64_t x = rlo, y = rhi; x | y;) {
          th -= C.W[size_t(k) * nv + low_bit(x, y)];
          if (x) x &= x - 1; else y &= y - 1;
        }
        A.add(th);
        if ((k & 7) == 7) A.split();
      }
      A.finish(lf[r], sf[r]);
      continue;
    }
    // created a0 < a1 and annihilated r0 < r1: LDS element offsets (absent:
    // the zero column), or byte offsets into a row of W (absent: W's end)
    const uint32_t absent = LDS ? uint32_t(nv) : wbytes;
    const uint32_t unit = LDS ? 1u : 8u;
    const uint32_t a0 = na > 0 ? uint32_t(low_bit(alo, ahi)) * unit : absent;
    if (alo) alo &= alo - 1; else ahi &= ahi - 1;
    const uint32_t a1 = na > 1 ? uint32_t(low_bit(alo, ahi)) * unit : absent;
    const uint32_t r0 = nr > 0 ? uint32_t(low_bit(rlo, rhi)) * unit : absent;
    if (rlo) rlo &= rlo - 1; else rhi &= rhi - 1;
    const uint32_t r1 = nr > 1 ? uint32_t(low_bit(rlo, rhi)) * unit : absent;
    auto ld = [&](uint32_t off, int k) -> double {
      if constexpr (LDS) {
        return wl[k * ws + int(off)];
      } else {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(wr, off, k * nv * 8, 0));
      }
    };
    double t = th0[0], wa0 = ld(a0, 0), wa1 = ld(a1, 0), wr0 = ld(r0, 0), wr1 = ld(r1, 0);
    for (int k8 = 0; k8 < nh; k8 += 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = k8 + j;
        if (k >= nh) break;
        const double th = (((t + wa0) + wa1) - wr0) - wr1;
        if (k + 1 < nh) {
          t = th0[k + 1];
          wa0 = ld(a0, k + 1); wa1 = ld(a1, k + 1); wr0 = ld(r0, k + 1); wr1 = ld(r1, k + 1);
        }
        A.add(th);
      }
      A.split();
    }
    A.finish(lf[r], sf[r]);
  }
}

// direct evaluation for arbitrary ONVs (no owner): theta = b + W x
__global__ void k_corr_direct(CorrParams C, const uint64_t* m, int64_t R, double* lf, int8_t* sf) {
  const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const uint64_t lo = m[2 * r], hi = m[2 * r + 1];
  const int nv = 2 * C.K;
  double acc = 0.0;
  int s = 1;
  for (int k = 0; k < C.nh; ++k) {
    double th = C.b[k];
    for (int P = 0; P < nv; ++P)
      if (bit_at(lo, hi, P)) th += C.W[size_t(k) * nv + P];
    const double c = cos(th);
    acc += log(fabs(c));
    if (c < 0) s = -s;
  }
  lf[r] = acc;
  sf[r] = int8_t(s);
}

// ---------------------------------------------------------------------------
// Ising-RBM correlator: theta_k = b_k + sum_P W_kP x_P + (1/2) x^T W2_k x.
// Only S_k = (W2_k + W2_k^T) / 2 enters.  S is kept as [P][Q][k] and W^T as
// [P][k]: a wavefront with one hidden unit per lane reads them coalesced.
//
// A row m of sample n changes the occupations by delta (at most four spin
// orbitals, +1 created, -1 annihilated), so
//   theta_k(m) = theta_k(n) + sum_a [delta_a (W_kPa + G_kPa(n)) + S_kPaPa / 2]
//                + sum_{a<b} delta_a delta_b S_kPaPb,   G_k(n) = S_k x(n).
// An orbital is created in m only if empty in n and annihilated only if
// occupied, so delta_a = 1 - 2 x_Pa(n) is fixed by (n, P): the first sum reads
// one per-sample table E[n][P][k] = (1 - 2 x_P) (W_kP + G_kP) + S_kPP / 2.
// ---------------------------------------------------------------------------

template <typename F>
__device__ inline void for_each_bit(uint64_t lo, uint64_t hi, F f) {
  for (uint64_t x = lo; x; x &= x - 1) f(__ffsll((unsigned long long)x) - 1);
  for (uint64_t x = hi; x; x &= x - 1) f(64 + __ffsll((unsigned long long)x) - 1);
}

__device__ inline double ising_theta(const CorrParams& C, uint64_t lo, uint64_t hi, int k) {
  const int nv = 2 * C.K, nh = C.nh;
  double lin = 0.0, quad = 0.0;
  for_each_bit(lo, hi, [&](int P) {
    lin += C.W1t[size_t(P) * nh + k];
    double row = 0.0;
    for_each_bit(lo, hi, [&](int Q) { row += C.S[(size_t(P) * nv + Q) * nh + k]; });
    quad += row;
  });
  return C.b[k] + lin + 0.5 * quad;
}

__device__ inline double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}

// theta of N ONVs: one wavefront per ONV, lanes over hidden units
__global__ __launch_bounds__(256) void k_ising_theta(CorrParams C, const uint64_t* samples, int64_t N,
                                                     double* theta) {
  const int64_t n = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (n >= N) return;
  const uint64_t lo = samples[2 * n], hi = samples[2 * n + 1];
  for (int k = lane; k < C.nh; k += 64) theta[n * C.nh + k] = ising_theta(C, lo, hi, k);
}

// E[n][P][k] for a tile of 32 samples (block x) and 256 columns c = P nh + k of
// one sample's table (block y): G = S x sums the rows S[Q][P][.] (= S[P][Q][.])
// of the occupied Q, read once per tile
constexpr int kIsingTile = 32;
template <typename TT>
__global__ __launch_bounds__(256) void k_ising_E(CorrParams C, const uint64_t* samples, int64_t N, TT* E) {
  __shared__ uint64_t slo[kIsingTile], shi[kIsingTile];
  const int nv = 2 * C.K, nh = C.nh;
  const int64_t cols = int64_t(nv) * nh;
  const int64_t n0 = int64_t(blockIdx.x) * kIsingTile;
  const int64_t c = int64_t(blockIdx.y) * blockDim.x + threadIdx.x;
  if (threadIdx.x < kIsingTile) {
    const int64_t n = n0 + threadIdx.x;
    slo[threadIdx.x] = n < N ? samples[2 * n] : 0ull;
    shi[threadIdx.x] = n < N ? samples[2 * n + 1] : 0ull;
  }
  __syncthreads();
  if (c >= cols) return;
  const int P = int(c / nh), k = int(c % nh);
  double acc[kIsingTile];
#pragma unroll
  for (int t = 0; t < kIsingTile; ++t) acc[t] = 0.0;
  for (int Q = 0; Q < nv; ++Q) {
    const double v = C.S[size_t(Q) * cols + c];
#pragma unroll
    for (int t = 0; t < kIsingTile; ++t)
      if (bit_at(slo[t], shi[t], Q)) acc[t] += v;
  }
  const double w = C.W1t[c], d = 0.5 * C.S[size_t(P) * cols + c];
#pragma unroll
  for (int t = 0; t < kIsingTile; ++t) {
    const int64_t n = n0 + t;
    if (n < N) E[n * cols + c] = TT((bit_at(slo[t], shi[t], P) ? -(w + acc[t]) : (w + acc[t])) + d);
  }
}

// log|f(m)| and sign f(m) of the rows: a wavefront takes kIsingRowsPerWave
// consecutive rows, kIsingBatch at a time, with hidden units across lanes; a
// batch's rows are decoded with scalar loads and their table reads issued
// together, so the wavefront keeps several rows' loads in flight.  Tables E and
// S in precision TT (FP32 for the FP32/BF16 paths: they then round like the
// FP32 cos that follows), theta accumulated in FP64, cos and log in precision
// T, the sum of logs in FP64.
constexpr int kIsingRowsPerWave = 16, kIsingBatch = 2;

// lowest set bit of the 128-bit (lo, hi), cleared; -1 if none
__device__ inline int pop_lowest(uint64_t& lo, uint64_t& hi) {
  if (lo) {
    const int P = __ffsll((unsigned long long)lo) - 1;
    lo &= lo - 1;
    return P;
  }
  if (hi) {
    const int P = 64 + __ffsll((unsigned long long)hi) - 1;
    hi &= hi - 1;
    return P;
  }
  return -1;
}

template <typename T, typename TT>
__global__ __launch_bounds__(256) void k_ising_rows(CorrParams C, const TT* S, const uint64_t* m,
                                                    const int32_t* owner, const uint64_t* samples,
                                                    const double* theta, const TT* E, int64_t R, double* lf,
                                                    int8_t* sf) {
  const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + __builtin_amdgcn_readfirstlane(threadIdx.x)) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t r0 = wave * kIsingRowsPerWave;
  if (r0 >= R) return;
  const int64_t r1 = r0 + kIsingRowsPerWave < R ? r0 + kIsingRowsPerWave : R;
  const int nv = 2 * C.K, nh = C.nh;
  for (int64_t rb = r0; rb < r1; rb += kIsingBatch) {
    // per row four fixed slots: the two created orbitals (delta +1), then the
    // two annihilated ones (delta -1); an absent slot has delta 0 and points
    // at orbital 0, so every row issues the same loads and adds exact zeros
    int ch[kIsingBatch][4];
    double dl[kIsingBatch][4];
    const TT* Eo[kIsingBatch];
    const double* To[kIsingBatch];
#pragma unroll
    for (int j = 0; j < kIsingBatch; ++j) {
      const int64_t r = rb + j < r1 ? rb + j : r1 - 1;
      const int64_t o = owner[r];
      const uint64_t mlo = m[2 * r], mhi = m[2 * r + 1];
      const uint64_t nlo = samples[2 * o], nhi = samples[2 * o + 1];
      uint64_t clo = mlo & ~nlo, chi = mhi & ~nhi, alo = nlo & ~mlo, ahi = nhi & ~mhi;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int P = a < 2 ? pop_lowest(clo, chi) : pop_lowest(alo, ahi);
        ch[j][a] = P < 0 ? 0 : P;
        dl[j][a] = P < 0 ? 0.0 : (a < 2 ? 1.0 : -1.0);
      }
      Eo[j] = E + size_t(o) * nv * nh;
      To[j] = theta + size_t(o) * nh;
    }
    double acc[kIsingBatch];
    int neg[kIsingBatch];
#pragma unroll
    for (int j = 0; j < kIsingBatch; ++j) { acc[j] = 0.0; neg[j] = 0; }
    for (int k = lane; k < nh; k += 64) {
#pragma unroll
      for (int j = 0; j < kIsingBatch; ++j) {
        double th = To[j][k];
#pragma unroll
        for (int a = 0; a < 4; ++a) th += (dl[j][a] * dl[j][a]) * double(Eo[j][size_t(ch[j][a]) * nh + k]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = a + 1; b < 4; ++b)
            th += (dl[j][a] * dl[j][b]) * double(S[(size_t(ch[j][a]) * nv + ch[j][b]) * nh + k]);
        const T cv = tcos(T(th));
        acc[j] += double(tlog(tabs(cv)));
        neg[j] ^= cv < T(0) ? 1 : 0;
      }
    }
#pragma unroll
    for (int j = 0; j < kIsingBatch; ++j) {
      const double sum = wave_sum(acc[j]);
      const int odd = __popcll(__ballot(neg[j])) & 1;
      if (lane == 0 && rb + j < r1) {
        lf[rb + j] = sum;
        sf[rb + j] = int8_t(odd ? -1 : 1);
      }
    }
  }
}

// direct evaluation for arbitrary ONVs (no owner), FP64
__global__ __launch_bounds__(256) void k_ising_direct(CorrParams C, const uint64_t* m, int64_t R, double* lf,
                                                      int8_t* sf) {
  const int64_t r = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= R) return;
  const uint64_t lo = m[2 * r], hi = m[2 * r + 1];
  double acc = 0.0;
  int neg = 0;
  for (int k = lane; k < C.nh; k += 64) {
    const double cv = cos(ising_theta(C, lo, hi, k));
    acc += log(fabs(cv));
    neg ^= cv < 0.0 ? 1 : 0;
  }
  acc = wave_sum(acc);
  const int odd = __popcll(__ballot(neg)) & 1;
  if (lane == 0) {
    lf[r] = acc;
    sf[r] = int8_t(odd ? -1 : 1);
  }
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

// Per sample n (one wavefront): E_loc(n) = H_nn + sum_rows coef * Psi(m)/Psi(n)
// and Etilde_num(n) = |f_n|^2 H_nn + f_n sum_rows coef f_m Phi(m)/Phi(n).
// CORR = false: no correlator (log|f| = 0, sign f = +1; the same arithmetic
// with the zero terms left out, which changes no bit)
template <bool CORR>
__global__ __launch_bounds__(256) void k_reduce(int64_t n0, int64_t n1, const int64_t* rowptr,
                                                int64_t row_base, const double* coef,
                                                const double* lphi, const int8_t* sphi,
                                                const double* lf, const int8_t* sf,
                                                const double* hdiag, double* eloc, double* etnum,
                                                double* logabs, int8_t* sign, double* fsq) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n = n0 + int64_t(blockIdx.x) * 4 + wv;
  if (n >= n1) return;
  const int64_t r0 = rowptr[n] - row_base, r1 = rowptr[n + 1] - row_base;
  const double lpn = lphi[r0], lfn = CORR ? lf[r0] : 0.0;
  const int sn = CORR ? int(sphi[r0]) * int(sf[r0]) : int(sphi[r0]);
  double se = 0.0, st = 0.0;
  for (int64_t r = r0 + 1 + lane; r < r1; r += 64) {
    if (CORR) {
      const double s = double(int(sphi[r]) * int(sf[r]) * sn);
      se += coef[r] * s * exp(lphi[r] + lf[r] - lpn - lfn);
      st += coef[r] * s * exp(lfn + lf[r] + lphi[r] - lpn);
    } else {
      const double s = double(int(sphi[r]) * sn);
      const double x = coef[r] * s * exp(lphi[r] - lpn);
      se += x;
      st += x;
    }
  }
  se = wave_sum(se);
  st = wave_sum(st);
  if (lane == 0) {
    const double la = lpn + lfn;
    const bool valid = sn != 0 && isfinite(la);
    const double f2 = exp(2.0 * lfn);
    const double hd = hdiag[n];
    if (eloc) eloc[n] = valid ? hd + se : NAN;
    if (etnum) etnum[n] = valid ? f2 * hd + st : NAN;
    if (logabs) logabs[n] = la;
    if (sign) sign[n] = int8_t(sn);
    if (fsq) fsq[n] = f2;
  }
}

// Per sample n (one wavefront), complex amplitudes: Psi(m)/Psi(n) =
// s e^{ln|Psi(m)| - ln|Psi(n)|} e^{i (phase_m - phase_n)} with the real signs s
// of the correlator; E_loc and Etilde_num as (re, im).  phs == nullptr: real
// parameters, the phase factor is the sign product (imaginary parts exactly 0).
template <bool CORR>
__global__ __launch_bounds__(256) void k_reduce_cx(int64_t n0, int64_t n1, const int64_t* rowptr,
                                                   int64_t row_base, const double* coef, const double* lphi,
                                                   const int8_t* sphi, const double* phs, const double* lf,
                                                   const int8_t* sf, const double* hdiag, double* eloc,
                                                   double* eloc_im, double* etnum, double* etnum_im,
                                                   double* logabs, double* phase, double* fsq) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n = n0 + int64_t(blockIdx.x) * 4 + wv;
  if (n >= n1) return;
  const int64_t r0 = rowptr[n] - row_base, r1 = rowptr[n + 1] - row_base;
  const double lpn = lphi[r0], lfn = CORR ? lf[r0] : 0.0;
  const int spn = int(sphi[r0]), sfn = CORR ? int(sf[r0]) : 1;
  const double phn = phs ? phs[r0] : 0.0;
  double se = 0.0, sei = 0.0, st = 0.0, sti = 0.0;
  for (int64_t r = r0 + 1 + lane; r < r1; r += 64) {
    const double s = CORR ? double(int(sf[r]) * sfn) : 1.0;
    const double x = CORR ? coef[r] * s * exp(lphi[r] + lf[r] - lpn - lfn) : coef[r] * exp(lphi[r] - lpn);
    const double xt = CORR ? coef[r] * s * exp(lfn + lf[r] + lphi[r] - lpn) : x;
    double cr, ci;
    if (phs) {
      const double d = phs[r] - phn;
      cr = cos(d);
      ci = sin(d);
    } else {
      cr = double(int(sphi[r]) * spn);
      ci = 0.0;
    }
    se += x * cr;
    sei += x * ci;
    st += xt * cr;
    sti += xt * ci;
  }
  se = wave_sum(se);
  sei = wave_sum(sei);
  st = wave_sum(st);
  sti = wave_sum(sti);
  if (lane == 0) {
    const double la = lpn + lfn;
    const bool valid = spn != 0 && isfinite(la);
    const double f2 = exp(2.0 * lfn);
    const double hd = hdiag[n];
    const double pi = 3.14159265358979323846;
    const double ph = phs ? phn : (spn < 0 ? pi : 0.0);
    if (eloc) eloc[n] = valid ? hd + se : NAN;
    if (eloc_im) eloc_im[n] = valid ? sei : NAN;
    if (etnum) etnum[n] = valid ? f2 * hd + st : NAN;
    if (etnum_im) etnum_im[n] = valid ? sti : NAN;
    if (logabs) logabs[n] = la;
    if (phase) phase[n] = valid ? remainder(ph + (sfn < 0 ? pi : 0.0), 2.0 * pi) : 0.0;
    if (fsq) fsq[n] = f2;
  }
}

// Batch sums with weights c_n (NaN local energies are left out and counted):
// out = {sum c, sum c|f|^2, sum c Etilde_num, E, B, var, n_nan, E_im}; with
// complex local energies the variance takes |E_loc - E|^2 and
// E_im = sum c Im Etilde_num / sum c|f|^2 (else 0)
__global__ __launch_bounds__(1024) void k_batch_sums(int64_t N, const double* counts, const double* eloc,
                                                     const double* etnum, const double* fsq,
                                                     const double* eloc_im, const double* etnum_im,
                                                     double* out) {
  __shared__ double red[4][1024];
  __shared__ double E_sh;
  const int tid = threadIdx.x;
  double sc = 0, sf2 = 0, se = 0, sei = 0, nn = 0;
  for (int64_t n = tid; n < N; n += 1024) {
    const double c = counts ? counts[n] : 1.0;
    if (isnan(eloc[n])) { nn += 1; continue; }
    sc += c;
    sf2 += c * fsq[n];
    se += c * etnum[n];
    if (etnum_im) sei += c * etnum_im[n];
  }
  red[0][tid] = sc; red[1][tid] = sf2; red[2][tid] = se; red[3][tid] = sei;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o)
      for (int k = 0; k < 4; ++k) red[k][tid] += red[k][tid + o];
    __syncthreads();
  }
  if (tid == 0) E_sh = red[2][0] / red[1][0];
  const double tsc = red[0][0], tsf = red[1][0], tse = red[2][0], tsei = red[3][0];
  __syncthreads();
  const double E = E_sh;
  double sv = 0;
  for (int64_t n = tid; n < N; n += 1024) {
    const double c = counts ? counts[n] : 1.0;
    if (isnan(eloc[n])) continue;
    const double d = eloc[n] - E;
    const double di = eloc_im ? eloc_im[n] : 0.0;
    sv += c * fsq[n] * (d * d + di * di);
  }
  __syncthreads();
  red[0][tid] = sv;
  red[1][tid] = nn;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) { red[0][tid] += red[0][tid + o]; red[1][tid] += red[1][tid + o]; }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = tsc; out[1] = tsf; out[2] = tse; out[3] = E; out[4] = tsf / tsc;
    out[5] = red[0][0] / tsf; out[6] = red[1][0]; out[7] = etnum_im ? tsei / tsf : 0.0;
  }
}

__global__ void k_gather_logpsi_phase(int64_t N, const double* lphi, const int8_t* sphi, const double* phs,
                                      const double* lf, const int8_t* sf, double* logabs, double* phase) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double pi = 3.14159265358979323846;
  const double ph = phs ? phs[n] : (sphi[n] < 0 ? pi : 0.0);
  const bool neg_f = sf && sf[n] < 0;
  if (logabs) logabs[n] = lphi[n] + (lf ? lf[n] : 0.0);
  if (phase) phase[n] = sphi[n] == 0 ? 0.0 : remainder(ph + (neg_f ? pi : 0.0), 2.0 * pi);
}

__global__ void k_gather_logpsi(int64_t N, const double* lphi, const int8_t* sphi, const double* lf,
                                const int8_t* sf, double* logabs, int8_t* sign) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double l = lphi[n] + (lf ? lf[n] : 0.0);
  const int s = int(sphi[n]) * (sf ? int(sf[n]) : 1);
  if (logabs) logabs[n] = l;
  if (sign) sign[n] = int8_t(s);
}

inline unsigned grid_for(int64_t units, int per_block) {
  return unsigned((units + per_block - 1) / per_block);
}

}  // namespace

hipError_t launch_corr_theta(const CorrParams& C, const uint64_t* samples, int64_t N, double* theta,
                             void* E, int precision, hipStream_t st) {
  if (N <= 0 || C.nh <= 0) return hipSuccess;
  if (!C.ising) {
    hipLaunchKernelGGL(k_corr_theta, dim3(grid_for(N * C.nh, 256)), dim3(256), 0, st, C, samples, N, theta);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_ising_theta, dim3(grid_for(N, 4)), dim3(256), 0, st, C, samples, N, theta);
  if (E) {
    const int64_t cols = int64_t(2 * C.K) * C.nh;
    if (precision == 0)
      hipLaunchKernelGGL(k_ising_E<double>, dim3(grid_for(N, kIsingTile), grid_for(cols, 256)), dim3(256), 0, st,
                         C, samples, N, (double*)E);
    else
      hipLaunchKernelGGL(k_ising_E<float>, dim3(grid_for(N, kIsingTile), grid_for(cols, 256)), dim3(256), 0, st,
                         C, samples, N, (float*)E);
  }
  return hipGetLastError();
}

hipError_t launch_corr_rows(const CorrParams& C, const uint64_t* m, const int32_t* owner,
                            const uint64_t* samples, const double* theta, const void* E, int64_t R,
                            int precision, double* lf, int8_t* sf, hipStream_t st) {
  if (R <= 0) return hipSuccess;
  if (C.ising) {
    if (!E) return hipErrorInvalidValue;
    if (precision == 0)
      hipLaunchKernelGGL((k_ising_rows<double, double>), dim3(grid_for(R, 4 * kIsingRowsPerWave)), dim3(256), 0,
                         st, C, C.S, m, owner, samples, theta, (const double*)E, R, lf, sf);
    else
      hipLaunchKernelGGL((k_ising_rows<float, float>), dim3(grid_for(R, 4 * kIsingRowsPerWave)), dim3(256), 0,
                         st, C, C.S32, m, owner, samples, theta, (const float*)E, R, lf, sf);
    return hipGetLastError();
  }
  // W in LDS when it fits: one persistent workgroup per CU (the device's CU
  // count, read once per device); else a thread per row with W from L2
  const size_t lds = size_t(C.nh) * (2 * C.K + 1) * sizeof(double);
  if (lds <= kCorrLdsMax) {
    static int cus[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    if (!cus[dev] && hipDeviceGetAttribute(&cus[dev], hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return hipErrorInvalidDevice;
    const unsigned blocks = unsigned(std::min<int64_t>((R + kCorrLdsThreads - 1) / kCorrLdsThreads, cus[dev]));
    if (precision == 0)
      hipLaunchKernelGGL((k_corr_rows<double, true>), dim3(blocks), dim3(kCorrLdsThreads), lds, st, C, m, owner,
                         samples, theta, R, lf, sf);
    else
      hipLaunchKernelGGL((k_corr_rows<float, true>), dim3(blocks), dim3(kCorrLdsThreads), lds, st, C, m, owner,
                         samples, theta, R, lf, sf);
  } else if (precision == 0) {
    hipLaunchKernelGGL((k_corr_rows<double, false>), dim3(grid_for(R, 256)), dim3(256), 0, st, C, m, owner, samples,
                       theta, R, lf, sf);
  } else {
    hipLaunchKernelGGL((k_corr_rows<float, false>), dim3(grid_for(R, 256)), dim3(256), 0, st, C, m, owner, samples,
                       theta, R, lf, sf);
  }
  return hipGetLastError();
}

hipError_t launch_corr_direct(const CorrParams& C, const uint64_t* m, int64_t R, double* lf, int8_t* sf,
                              hipStream_t st) {
  if (R <= 0) return hipSuccess;
  if (C.ising)
    hipLaunchKernelGGL(k_ising_direct, dim3(grid_for(R, 4)), dim3(256), 0, st, C, m, R, lf, sf);
  else
    hipLaunchKernelGGL(k_corr_direct, dim3(grid_for(R, 256)), dim3(256), 0, st, C, m, R, lf, sf);
  return hipGetLastError();
}

hipError_t launch_reduce(int64_t n0, int64_t n1, const int64_t* rowptr, int64_t row_base, const double* coef,
                         const double* lphi, const int8_t* sphi, const double* lf, const int8_t* sf,
                         const double* hdiag, double* eloc, double* etnum, double* logabs, int8_t* sign,
                         double* fsq, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (lf && sf)
    hipLaunchKernelGGL(k_reduce<true>, dim3(grid_for(n1 - n0, 4)), dim3(256), 0, st, n0, n1, rowptr, row_base,
                       coef, lphi, sphi, lf, sf, hdiag, eloc, etnum, logabs, sign, fsq);
  else
    hipLaunchKernelGGL(k_reduce<false>, dim3(grid_for(n1 - n0, 4)), dim3(256), 0, st, n0, n1, rowptr, row_base,
                       coef, lphi, sphi, lf, sf, hdiag, eloc, etnum, logabs, sign, fsq);
  return hipGetLastError();
}

hipError_t launch_batch_sums(int64_t N, const double* counts, const double* eloc, const double* etnum,
                             const double* fsq, double* out, hipStream_t st, const double* eloc_im,
                             const double* etnum_im) {
  hipLaunchKernelGGL(k_batch_sums, dim3(1), dim3(1024), 0, st, N, counts, eloc, etnum, fsq, eloc_im, etnum_im,
                     out);
  return hipGetLastError();
}

hipError_t launch_reduce_cx(int64_t n0, int64_t n1, const int64_t* rowptr, int64_t row_base, const double* coef,
                            const double* lphi, const int8_t* sphi, const double* phs, const double* lf,
                            const int8_t* sf, const double* hdiag, double* eloc, double* eloc_im, double* etnum,
                            double* etnum_im, double* logabs, double* phase, double* fsq, hipStream_t st) {
  if (n1 <= n0) return hipSuccess;
  if (lf && sf)
    hipLaunchKernelGGL(k_reduce_cx<true>, dim3(grid_for(n1 - n0, 4)), dim3(256), 0, st, n0, n1, rowptr, row_base,
                       coef, lphi, sphi, phs, lf, sf, hdiag, eloc, eloc_im, etnum, etnum_im, logabs, phase, fsq);
  else
    hipLaunchKernelGGL(k_reduce_cx<false>, dim3(grid_for(n1 - n0, 4)), dim3(256), 0, st, n0, n1, rowptr, row_base,
                       coef, lphi, sphi, phs, lf, sf, hdiag, eloc, eloc_im, etnum, etnum_im, logabs, phase, fsq);
  return hipGetLastError();
}

hipError_t launch_gather_logpsi_phase(int64_t N, const double* lphi, const int8_t* sphi, const double* phs,
                                      const double* lf, const int8_t* sf, double* logabs, double* phase,
                                      hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_logpsi_phase, dim3(grid_for(N, 256)), dim3(256), 0, st, N, lphi, sphi, phs, lf, sf,
                     logabs, phase);
  return hipGetLastError();
}

hipError_t launch_gather_logpsi(int64_t N, const double* lphi, const int8_t* sphi, const double* lf,
                                const int8_t* sf, double* logabs, int8_t* sign, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_logpsi, dim3(grid_for(N, 256)), dim3(256), 0, st, N, lphi, sphi, lf, sf,
                     logabs, sign);
  return hipGetLastError();
}

}  // namespace nqs
