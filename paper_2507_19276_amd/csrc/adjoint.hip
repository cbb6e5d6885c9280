// Hand-written adjoint of log|Psi(n)| (the gradient factor of Sec. 2.1
// Eq. (7) and Sec. 2.3 Eq. (19)) for the BDG-RNN / MPS-RNN amplitude and the
// cos-RBM correlator on gfx950.
//
// Forward: the amplitude kernel stores the carried state h_i^{s_i} of every
// row and site (Hbuf[i][row][chip]).  Backward: a reverse sweep over sites,
// per site i
//   A. recompute the four candidates h_i^s = sum_j M_ij^s h_j + v_i^s on MFMA
//      from the stored parents, then
//        dcand^s = g eta h^s ([s = s_i] / P^{s_i} - [s allowed] / Z) + [s = s_i] dcarry_i
//        deta    = g/2 (h^{s_i}^2 / P^{s_i} - sum_allowed h^s^2 / Z)
//      and push dcarry_j += sum_s M_ij^s^T dcand^s to every parent j (MFMA);
//   B. dM_ij^s = sum_rows dcand^s (x) h_j and dv, deta as column sums over row
//      splits, each split writing its own slice of a partial-gradient buffer.
// The partial buffer is summed in a fixed order at the end, so the gradient is
// bit-reproducible from run to run.
//
// Complex parameters run on the realified 2chi-unit state.  The phase term
// gp arg(z_i), z_i = (w^T x + c) + i (w2^T x + c2) of the row's state x = h_i^{s_i},
// adds (alpha w + beta w2) to dcand^{s_i} with alpha = -gp Im z / |z|^2 and
// beta = gp Re z / |z|^2, and the column sums dw = sum_rows alpha x,
// dw2 = sum beta x, dc = sum alpha, dc2 = sum beta.  k_cx_* map the realified
// gradient back onto the packed complex parameters.
//
// MFMA k-permutation: in the 16x16x4 output layout lane (row j, group g)
// holds units 16t + 4g + v of tile t in register v.  A contraction over those
// units uses k-step (t, v) and lets lane group g supply unit 16t + 4g + v,
// so values already in registers are valid A/B operands without a transpose.
#include "internal.h"
#include <cmath>

namespace nqs {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct V4;
template <> struct V4<double> { typedef d4 type; };
template <> struct V4<float> { typedef f4 type; };

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// row of the 16x16 output tile held in register v of lane group g
template <typename T> __device__ inline int out_row(int g, int v);
template <> __device__ inline int out_row<float>(int g, int v) { return 4 * g + v; }
template <> __device__ inline int out_row<double>(int g, int v) { return g + 4 * v; }

__device__ inline bool allowed(int a_prev, int b_prev, int s, int rest, int na, int nb) {
  const int a = a_prev + (s & 1), b = b_prev + (s >> 1);
  return a <= na && a + rest >= na && b <= nb && b + rest >= nb;
}

__device__ inline int site_state(uint64_t lo, uint64_t hi, int i) {
  const int P = 2 * i;
  const uint64_t w = P < 64 ? (lo >> P) : (hi >> (P - 64));
  return int(w & 3ull);
}

// electrons of each spin on sites < i
__device__ inline void counts_below(uint64_t lo, uint64_t hi, int i, int& ca, int& cb) {
  const uint64_t ev = 0x5555555555555555ull;
  const int P = 2 * i;
  uint64_t mlo, mhi;
  if (P >= 128) { mlo = ~0ull; mhi = ~0ull; }
  else if (P >= 64) { mlo = ~0ull; mhi = P == 64 ? 0ull : ((1ull << (P - 64)) - 1ull); }
  else { mlo = P == 0 ? 0ull : ((1ull << P) - 1ull); mhi = 0ull; }
  ca = __popcll(lo & mlo & ev) + __popcll(hi & mhi & ev);
  cb = __popcll(lo & mlo & (ev << 1)) + __popcll(hi & mhi & (ev << 1));
}

// Kernel A: one wavefront = 16 rows of site i.
template <typename T, int CH, bool CPLX>
__global__ __launch_bounds__(256) void k_bwd_site(AdjParams<T> P, int i, const uint64_t* m, int64_t R,
                                                  int64_t Rpad, const double* cot, const T* Hbuf,
                                                  T* dcarry, T* Dc, T* Eeta) {
  typedef typename V4<T>::type V;
  constexpr int TPC = CH / 16, NT = 4 * TPC, KS = CH / 4;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  const int64_t tile = int64_t(blockIdx.x) * 4 + wv;
  const int64_t row0 = tile * 16;
  if (row0 >= Rpad) return;
  const int64_t row = row0 + j;
  const bool live = row < R;
  const int64_t rr = live ? row : (R - 1);
  const uint64_t lo = m[2 * rr], hi = m[2 * rr + 1];
  const double gd = live ? cot[row] : 0.0;
  const T gg = T(gd);
  const int e0 = P.pptr[i], e1 = P.pptr[i + 1];
  // recompute the candidates (A operand: W^T with the k-permutation, B: own
  // row's stored parent state, units 16t + 4g + v in component v)
  V acc[NT];
#pragma unroll
  for (int ot = 0; ot < NT; ++ot) acc[ot] = V{0, 0, 0, 0};
  for (int e = e0; e < e1; ++e) {
    const int pj = P.pidx[e];
    const T* hp = Hbuf + (size_t(pj) * Rpad + row) * CH + 4 * g;
    const T* Ae = P.AF + P.afoff[i] + size_t(e - e0) * (KS * NT * 64) + lane;
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      const V hb = *reinterpret_cast<const V*>(hp + 16 * t);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = 4 * t + v;
        const T b = hb[v];
#pragma unroll
        for (int ot = 0; ot < NT; ++ot) acc[ot] = mfma(Ae[(q * NT + ot) * 64], b, acc[ot]);
      }
    }
  }
  const T* vi = P.v + size_t(i) * 4 * CH;
  const T* ei = P.eta + size_t(i) * CH;
  T ps[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    T p = 0;
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      const int u0 = 16 * t + 4 * g;
      const V vv = *reinterpret_cast<const V*>(vi + s * CH + u0);
      const V ee = *reinterpret_cast<const V*>(ei + u0);
      V x = acc[s * TPC + t] + vv;
      if (P.tadd) x += *reinterpret_cast<const V*>(P.tadd + (size_t(row) * 4 + s) * CH + u0);
      acc[s * TPC + t] = x;
      p += ee.x * x.x * x.x + ee.y * x.y * x.y + ee.z * x.z * x.z + ee.w * x.w * x.w;
    }
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    ps[s] = p;
  }
  int ca, cb;
  counts_below(lo, hi, i, ca, cb);
  const int si = site_state(lo, hi, i);
  const int rest = P.K - 1 - i;
  bool ok[4];
  T Z = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    ok[s] = allowed(ca, cb, s, rest, P.na, P.nb);
    if (ok[s]) Z += ps[s];
  }
  const T psi_ = si == 0 ? ps[0] : si == 1 ? ps[1] : si == 2 ? ps[2] : ps[3];
  const T inv_p = T(1) / psi_, inv_z = T(1) / Z;
  // phase term (complex parameters): alpha, beta of this row
  T al = T(0), be = T(0);
  if (CPLX) {
    T zr = T(0), zi = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (s != si) continue;
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        const int u0 = 16 * t + 4 * g;
        const V wa = *reinterpret_cast<const V*>(P.w + size_t(i) * CH + u0);
        const V wb = *reinterpret_cast<const V*>(P.w2 + size_t(i) * CH + u0);
        const V x = acc[s * TPC + t];
        zr += wa.x * x.x + wa.y * x.y + wa.z * x.z + wa.w * x.w;
        zi += wb.x * x.x + wb.y * x.y + wb.z * x.z + wb.w * x.w;
      }
    }
    zr += __shfl_xor(zr, 16);
    zr += __shfl_xor(zr, 32);
    zi += __shfl_xor(zi, 16);
    zi += __shfl_xor(zi, 32);
    zr += P.c[i];
    zi += P.c2[i];
    const T z2 = zr * zr + zi * zi;
    const T gp = live ? T(P.cotp[row]) : T(0);
    if (z2 > T(0)) {
      al = -gp * zi / z2;
      be = gp * zr / z2;
    }
    if (g == 0) {
      P.ab[2 * row] = al;
      P.ab[2 * row + 1] = be;
    }
  }
  // d eta and dcand (in place of acc)
  const T* dci = dcarry + (size_t(i) * Rpad + row) * CH + 4 * g;
  V de[TPC];
#pragma unroll
  for (int t = 0; t < TPC; ++t) de[t] = V{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      const int u0 = 16 * t + 4 * g;
      const V ee = *reinterpret_cast<const V*>(ei + u0);
      const V x = acc[s * TPC + t];
      V d = V{0, 0, 0, 0};
      if (ok[s]) {
        const T f = (s == si ? inv_p : T(0)) - inv_z;
        d = gg * f * ee * x;
        de[t] -= T(0.5) * gg * inv_z * x * x;
      }
      if (s == si) {
        d += *reinterpret_cast<const V*>(dci + 16 * t);
        de[t] += T(0.5) * gg * inv_p * x * x;
        if (CPLX) {
          const V wa = *reinterpret_cast<const V*>(P.w + size_t(i) * CH + u0);
          const V wb = *reinterpret_cast<const V*>(P.w2 + size_t(i) * CH + u0);
          d += al * wa + be * wb;
        }
      }
      acc[s * TPC + t] = d;
      *reinterpret_cast<V*>(Dc + size_t(row) * 4 * CH + s * CH + u0) = d;
    }
  }
#pragma unroll
  for (int t = 0; t < TPC; ++t)
    *reinterpret_cast<V*>(Eeta + size_t(row) * CH + 16 * t + 4 * g) = de[t];
  // parents: dcarry_j[row][kk] += sum_{s,u} dcand[row][s,u] M_ij^s[u][kk]
  // A = dcand (rows x (s,u)), own registers; B = BT-packed M, k-step (s,t,v)
  for (int e = e0; e < e1; ++e) {
    const int pj = P.pidx[e];
    const T* Be = P.BT + P.btoff[i] + size_t(e - e0) * (4 * KS * TPC * 64) + lane;
#pragma unroll
    for (int ot = 0; ot < TPC; ++ot) {
      V o = V{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < TPC; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int q = (s * TPC + t) * 4 + v;
            o = mfma(acc[s * TPC + t][v], Be[(q * TPC + ot) * 64], o);
          }
      // o: rows out_row(g, v) of the tile, column kk = 16 ot + j
      T* dcp = dcarry + size_t(pj) * Rpad * CH;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + out_row<T>(g, v);
        dcp[size_t(r) * CH + 16 * ot + j] += o[v];
      }
    }
  }
}

// Kernel B: dM_ij^s[u][kk] = sum_{rows in split} Dc[row][s,u] Hbuf[j][row][kk]
// One wavefront per (edge, output tile of (s,u) x kk, split).
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_bwd_dm(AdjParams<T> P, int i, int64_t Rpad, int rows_per_split,
                                                int nsplit, const T* Hbuf, const T* Dc, double* gpart,
                                                int64_t n_params) {
  typedef typename V4<T>::type V;
  constexpr int MT = 4 * CH / 16, KT = CH / 16;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int e0 = P.pptr[i], d = P.pptr[i + 1] - e0;
  const int64_t unit = int64_t(blockIdx.x) * 4 + wv;
  const int64_t total = int64_t(d) * MT * KT * nsplit;
  if (unit >= total) return;
  const int split = int(unit % nsplit);
  int64_t rest = unit / nsplit;
  const int kt = int(rest % KT); rest /= KT;
  const int mt = int(rest % MT); rest /= MT;
  const int el = int(rest);
  const int pj = P.pidx[e0 + el];
  const int mrow = lane & 15, kq = lane >> 4;
  // the f64 output keeps rows g + 4v in register v: load A rows permuted so
  // that register v of group g again holds unit 4g + v
  const int mperm = sizeof(T) == 8 ? 4 * (mrow & 3) + (mrow >> 2) : mrow;
  const int64_t r0 = int64_t(split) * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < Rpad ? r0 + rows_per_split : Rpad;
  V acc = V{0, 0, 0, 0};
  const T* Ap = Dc + size_t(mt) * 16 + mperm;
  const T* Bp = Hbuf + size_t(pj) * Rpad * CH + size_t(kt) * 16 + mrow;
  for (int64_t r = r0 + kq; r < r1; r += 4) {
    const T a = Ap[size_t(r) * 4 * CH];
    const T b = Bp[size_t(r) * CH];
    acc = mfma(a, b, acc);
  }
  const int g = lane >> 4, n = lane & 15;
  const int kk = kt * 16 + n;
  double* out = gpart + size_t(split) * n_params;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int o = mt * 16 + 4 * g + v;          // unit index (s, u) = (o / CH, o % CH)
    const int s = o / CH, u = o % CH;
    if (u < P.chi && kk < P.chi)
      out[P.offM[e0 + el] + (int64_t(s) * P.chi + u) * P.chi + kk] = double(acc[v]);
  }
}

// dv and deta: column sums over the rows of each split (one thread per unit)
template <typename T, int CH>
__global__ void k_bwd_colsum(AdjParams<T> P, int i, int64_t Rpad, int rows_per_split, int nsplit,
                             const T* Dc, const T* Eeta, double* gpart, int64_t n_params) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int ncol = 5 * CH;   // 4 CH of v, CH of eta
  if (t >= int64_t(ncol) * nsplit) return;
  const int split = int(t / ncol);
  const int col = int(t % ncol);
  const int64_t r0 = int64_t(split) * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < Rpad ? r0 + rows_per_split : Rpad;
  double acc = 0.0;
  if (col < 4 * CH) {
    for (int64_t r = r0; r < r1; ++r) acc += double(Dc[size_t(r) * 4 * CH + col]);
    const int s = col / CH, u = col % CH;
    if (u < P.chi) gpart[size_t(split) * n_params + P.offV[i] + s * P.chi + u] = acc;
  } else {
    const int u = col - 4 * CH;
    for (int64_t r = r0; r < r1; ++r) acc += double(Eeta[size_t(r) * CH + u]);
    if (u < P.chi) gpart[size_t(split) * n_params + P.offEta[i] + u] = acc;
  }
}

// complex parameters: dw[u] = sum_rows alpha x[u], dw2[u] = sum beta x[u],
// dc = sum alpha, dc2 = sum beta over the rows of each split (one thread per
// column: 2 CH units, then c and c2)
template <typename T, int CH>
__global__ void k_bwd_phase_colsum(AdjParams<T> P, int i, int64_t Rpad, int rows_per_split, int nsplit,
                                   const T* Hbuf, double* gpart, int64_t n_params) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int ncol = 2 * CH + 2;
  if (t >= int64_t(ncol) * nsplit) return;
  const int split = int(t / ncol);
  const int col = int(t % ncol);
  const int64_t r0 = int64_t(split) * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < Rpad ? r0 + rows_per_split : Rpad;
  const int which = col < 2 * CH ? col / CH : col - 2 * CH;    // 0: alpha (w, c), 1: beta (w2, c2)
  const int u = col % CH;
  const T* x = Hbuf + size_t(i) * Rpad * CH + u;
  double acc = 0.0;
  if (col < 2 * CH) {
    for (int64_t r = r0; r < r1; ++r) acc += double(P.ab[2 * r + which]) * double(x[size_t(r) * CH]);
    if (u < P.chi) gpart[size_t(split) * n_params + (which ? P.offW2[i] : P.offW[i]) + u] = acc;
  } else {
    for (int64_t r = r0; r < r1; ++r) acc += double(P.ab[2 * r + which]);
    gpart[size_t(split) * n_params + (which ? P.offC2[i] : P.offC[i])] = acc;
  }
}

// realified -> packed complex gradient.  M_r = [[Re M, -Im M], [Im M, Re M]]
// per state: d Re M = G[u][k] + G[u+chi][k+chi], d Im M = G[u+chi][k] - G[u][k+chi]
__global__ void k_cx_grad_edges(CxMap M, const double* gr, double* grad) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int chi = M.chi, c2 = 2 * chi;
  const int64_t per = int64_t(4) * chi * chi;
  if (t >= per * M.n_edges) return;
  const int e = int(t / per);
  const int r = int(t % per);
  const int s = r / (chi * chi), u = (r / chi) % chi, k = r % chi;
  const double* G = gr + M.rM[e] + size_t(s) * c2 * c2;
  const double dre = G[size_t(u) * c2 + k] + G[size_t(u + chi) * c2 + k + chi];
  const double dim = G[size_t(u + chi) * c2 + k] - G[size_t(u) * c2 + k + chi];
  double* out = grad + M.cM[e] + 2 * ((size_t(s) * chi + u) * chi + k);
  out[0] += dre;
  out[1] += dim;
}

// per site: v_r = [Re v; Im v], eta_r = [eta; eta], w_r = [Re w; -Im w],
// w2 = [Im w; Re w], c_r = Re c, c2 = Im c
__global__ void k_cx_grad_sites(CxMap M, const double* gr, double* grad) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int chi = M.chi, c2 = 2 * chi;
  const int per = 6 * chi + 1;
  if (t >= int64_t(per) * M.K) return;
  const int i = int(t / per);
  const int r = int(t % per);
  if (r < 4 * chi) {
    const int s = r / chi, u = r % chi;
    double* out = grad + M.cV[i] + 2 * (s * chi + u);
    out[0] += gr[M.rV[i] + s * c2 + u];
    out[1] += gr[M.rV[i] + s * c2 + chi + u];
  } else if (r < 5 * chi) {
    const int u = r - 4 * chi;
    grad[M.cEta[i] + u] += gr[M.rEta[i] + u] + gr[M.rEta[i] + chi + u];
  } else if (r < 6 * chi) {
    const int u = r - 5 * chi;
    double* out = grad + M.cW[i] + 2 * u;
    out[0] += gr[M.rW[i] + u] + gr[M.rW2[i] + chi + u];
    out[1] += gr[M.rW2[i] + u] - gr[M.rW[i] + chi + u];
  } else {
    double* out = grad + M.cC[i];
    out[0] += gr[M.rC[i]];
    out[1] += gr[M.rC2[i]];
  }
}

__global__ void k_cx_grad_corr(CxMap M, const double* gr, double* grad) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < M.n_corr) grad[M.c_corr + t] += gr[M.r_corr + t];
}

__device__ inline bool bit_at(uint64_t lo, uint64_t hi, int P) {
  return P < 64 ? ((lo >> P) & 1ull) : ((hi >> (P - 64)) & 1ull);
}

// d log|f| / d theta_k = -tan(theta_k), scaled by the cotangent
__global__ void k_corr_dtheta(CorrParams C, const uint64_t* m, int64_t R, const double* cot,
                              double* dth) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= R * C.nh) return;
  const int64_t r = t / C.nh;
  const int k = int(t % C.nh);
  const uint64_t lo = m[2 * r], hi = m[2 * r + 1];
  const int nv = 2 * C.K;
  double th = C.b[k];
  for (int P = 0; P < nv; ++P)
    if (bit_at(lo, hi, P)) th += C.W[size_t(k) * nv + P];
  dth[t] = -cot[r] * tan(th);
}

// db_k and dW_kP over the rows of one split: block (split, k), thread P (P = 2K -> db)
__global__ void k_corr_grad(CorrParams C, const uint64_t* m, int64_t R, int rows_per_split,
                            const double* dth, int64_t offB, int64_t offW, double* gpart,
                            int64_t n_params) {
  const int split = blockIdx.x / C.nh, k = blockIdx.x % C.nh;
  const int P = threadIdx.x;
  const int nv = 2 * C.K;
  if (P > nv) return;
  const int64_t r0 = int64_t(split) * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < R ? r0 + rows_per_split : R;
  double acc = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double d = dth[r * C.nh + k];
    if (P == nv) acc += d;
    else if (bit_at(m[2 * r], m[2 * r + 1], P)) acc += d;
  }
  double* out = gpart + size_t(split) * n_params;
  if (P == nv) out[offB + k] = acc;
  else out[offW + int64_t(k) * nv + P] = acc;
}

// Ising-RBM: dth = -cot tan(theta) from theta of the rows (written in place)
__global__ void k_dth_from_theta(int64_t R, int nh, const double* cot, double* dth) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= R * nh) return;
  dth[t] = -cot[t / nh] * tan(dth[t]);
}

// Ising-RBM quadratic couplings: d theta_k / d W2_kPQ = x_P x_Q / 2; block
// (split, k, P), thread Q
__global__ void k_ising_grad_W2(CorrParams C, const uint64_t* m, int64_t R, int rows_per_split,
                                const double* dth, int64_t offW2, double* gpart, int64_t n_params) {
  const int nv = 2 * C.K, nh = C.nh;
  const int64_t b = blockIdx.x;
  const int split = int(b / (int64_t(nh) * nv));
  const int k = int((b / nv) % nh), P = int(b % nv);
  const int Q = threadIdx.x;
  if (Q >= nv) return;
  const int64_t r0 = int64_t(split) * rows_per_split;
  const int64_t r1 = r0 + rows_per_split < R ? r0 + rows_per_split : R;
  double acc = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const uint64_t lo = m[2 * r], hi = m[2 * r + 1];
    if (bit_at(lo, hi, P) && bit_at(lo, hi, Q)) acc += dth[r * nh + k];
  }
  gpart[size_t(split) * n_params + offW2 + (int64_t(k) * nv + P) * nv + Q] = 0.5 * acc;
}

// grad[p] += sum_split gpart[split][p], splits in ascending order
__global__ void k_sum_parts(int64_t n_params, int nsplit, const double* gpart, double* grad) {
  const int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= n_params) return;
  double acc = 0.0;
  for (int s = 0; s < nsplit; ++s) acc += gpart[size_t(s) * n_params + p];
  grad[p] += acc;
}

inline unsigned grid_for(int64_t units, int per_block) {
  return unsigned((units + per_block - 1) / per_block);
}

template <typename T, int CH>
hipError_t run_site(const AdjParams<T>& P, int i, const uint64_t* m, int64_t R, int64_t Rpad,
                    const double* cot, const T* Hbuf, T* dcarry, T* Dc, T* Eeta, int rows_per_split,
                    int nsplit, double* gpart, int64_t n_params, hipStream_t st) {
  const int64_t tiles = Rpad / 16;
  if (P.cotp)
    hipLaunchKernelGGL((k_bwd_site<T, CH, true>), dim3(grid_for(tiles, 4)), dim3(256), 0, st, P, i, m, R, Rpad,
                       cot, Hbuf, dcarry, Dc, Eeta);
  else
    hipLaunchKernelGGL((k_bwd_site<T, CH, false>), dim3(grid_for(tiles, 4)), dim3(256), 0, st, P, i, m, R, Rpad,
                       cot, Hbuf, dcarry, Dc, Eeta);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (P.cotp) {
    hipLaunchKernelGGL((k_bwd_phase_colsum<T, CH>), dim3(grid_for(int64_t(2 * CH + 2) * nsplit, 256)), dim3(256),
                       0, st, P, i, Rpad, rows_per_split, nsplit, Hbuf, gpart, n_params);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int d = P.pptr_host[i + 1] - P.pptr_host[i];
  if (d > 0) {
    const int64_t units = int64_t(d) * (4 * CH / 16) * (CH / 16) * nsplit;
    hipLaunchKernelGGL((k_bwd_dm<T, CH>), dim3(grid_for(units, 4)), dim3(256), 0, st, P, i, Rpad,
                       rows_per_split, nsplit, Hbuf, Dc, gpart, n_params);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_bwd_colsum<T, CH>), dim3(grid_for(int64_t(5 * CH) * nsplit, 256)), dim3(256), 0, st,
                     P, i, Rpad, rows_per_split, nsplit, Dc, Eeta, gpart, n_params);
  return hipGetLastError();
}

template <typename T>
hipError_t run_sweep(const AdjParams<T>& P0, const uint64_t* m, int64_t R, int64_t Rpad, const double* cot,
                     const T* Hbuf, T* dcarry, T* Dc, T* Eeta, int rows_per_split, int nsplit, double* gpart,
                     int64_t n_params, hipStream_t st, const TnAdj<T>* tn) {
  for (int i = P0.K - 1; i >= 0; --i) {
    hipError_t e;
    // a tensor site: its term t^s of every row first (added to the recomputed
    // candidates), its own gradient and the parents' cotangents after dcand
    const bool tsite = tn && tn->tq_host[i] > 0;
    AdjParams<T> P = P0;
    P.tadd = tsite ? tn->TT : nullptr;
    if (tsite && (e = launch_tn_bwd_site(*tn, P0.pidx, i, 0, Rpad, Hbuf, Dc, dcarry, rows_per_split, nsplit, gpart,
                                         n_params, st)) != hipSuccess)
      return e;
    switch (P.chip) {
      case 16: e = run_site<T, 16>(P, i, m, R, Rpad, cot, Hbuf, dcarry, Dc, Eeta, rows_per_split, nsplit, gpart, n_params, st); break;
      case 32: e = run_site<T, 32>(P, i, m, R, Rpad, cot, Hbuf, dcarry, Dc, Eeta, rows_per_split, nsplit, gpart, n_params, st); break;
      case 48: e = run_site<T, 48>(P, i, m, R, Rpad, cot, Hbuf, dcarry, Dc, Eeta, rows_per_split, nsplit, gpart, n_params, st); break;
      case 64: e = run_site<T, 64>(P, i, m, R, Rpad, cot, Hbuf, dcarry, Dc, Eeta, rows_per_split, nsplit, gpart, n_params, st); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (tsite && (e = launch_tn_bwd_site(*tn, P0.pidx, i, 1, Rpad, Hbuf, Dc, dcarry, rows_per_split, nsplit, gpart,
                                         n_params, st)) != hipSuccess)
      return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_bwd_sweep_f64(const AdjParams<double>& P, const uint64_t* m, int64_t R, int64_t Rpad,
                                const double* cot, const double* Hbuf, double* dcarry, double* Dc,
                                double* Eeta, int rows_per_split, int nsplit, double* gpart,
                                int64_t n_params, hipStream_t st, const TnAdj<double>* tn) {
  return run_sweep<double>(P, m, R, Rpad, cot, Hbuf, dcarry, Dc, Eeta, rows_per_split, nsplit, gpart,
                           n_params, st, tn);
}

hipError_t launch_bwd_sweep_f32(const AdjParams<float>& P, const uint64_t* m, int64_t R, int64_t Rpad,
                                const double* cot, const float* Hbuf, float* dcarry, float* Dc,
                                float* Eeta, int rows_per_split, int nsplit, double* gpart,
                                int64_t n_params, hipStream_t st, const TnAdj<float>* tn) {
  return run_sweep<float>(P, m, R, Rpad, cot, Hbuf, dcarry, Dc, Eeta, rows_per_split, nsplit, gpart,
                          n_params, st, tn);
}

hipError_t launch_corr_backward(const CorrParams& C, const uint64_t* m, int64_t R, const double* cot,
                                double* dth, int rows_per_split, int nsplit, int64_t offB, int64_t offW,
                                int64_t offW2, double* gpart, int64_t n_params, hipStream_t st) {
  if (C.nh <= 0 || R <= 0) return hipSuccess;
  hipError_t e;
  if (C.ising) {
    if ((e = launch_corr_theta(C, m, R, dth, nullptr, 0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dth_from_theta, dim3(grid_for(R * C.nh, 256)), dim3(256), 0, st, R, C.nh, cot, dth);
  } else {
    hipLaunchKernelGGL(k_corr_dtheta, dim3(grid_for(R * C.nh, 256)), dim3(256), 0, st, C, m, R, cot, dth);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (C.ising) {
    const int nv = 2 * C.K;
    hipLaunchKernelGGL(k_ising_grad_W2, dim3(unsigned(int64_t(nsplit) * C.nh * nv)), dim3((nv + 63) / 64 * 64),
                       0, st, C, m, R, rows_per_split, dth, offW2, gpart, n_params);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int threads = ((2 * C.K + 1 + 63) / 64) * 64;
  hipLaunchKernelGGL(k_corr_grad, dim3(unsigned(nsplit * C.nh)), dim3(threads), 0, st, C, m, R, rows_per_split,
                     dth, offB, offW, gpart, n_params);
  return hipGetLastError();
}

hipError_t launch_cx_grad_map(const CxMap& M, const double* gr, double* grad, hipStream_t st) {
  const int64_t ne = int64_t(4) * M.chi * M.chi * M.n_edges;
  if (ne > 0) {
    hipLaunchKernelGGL(k_cx_grad_edges, dim3(grid_for(ne, 256)), dim3(256), 0, st, M, gr, grad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_cx_grad_sites, dim3(grid_for(int64_t(6 * M.chi + 1) * M.K, 256)), dim3(256), 0, st, M, gr,
                     grad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || M.n_corr == 0) return e;
  hipLaunchKernelGGL(k_cx_grad_corr, dim3(grid_for(M.n_corr, 256)), dim3(256), 0, st, M, gr, grad);
  return hipGetLastError();
}

hipError_t launch_sum_parts(int64_t n_params, int nsplit, const double* gpart, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_parts, dim3(grid_for(n_params, 256)), dim3(256), 0, st, n_params, nsplit, gpart,
                     grad);
  return hipGetLastError();
}

}  // namespace nqs
