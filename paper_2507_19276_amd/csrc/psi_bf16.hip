// BDG-RNN / MPS-RNN forward with BF16 bond contractions on gfx950
// (arXiv:2507.19276, Sec. 2.1 Eqs. (9)-(10); the reduced-precision form of
// the amplitude evaluation): BF16 operands on the 16x16x32 MFMA with FP32
// accumulation and per-row power-of-two scaled hidden states.
#include "device.h"

namespace nqs {
namespace {

// ---------------------------------------------------------------------------
// BF16 bond contractions (16x16x32 MFMA, FP32 accumulate) with scaled hidden
// states: the ring keeps h_j / 2^e_j in BF16 with a per-row exponent e_j per
// slot.  At site i the parents are brought to the common exponent
// e_ref = max_j e_j (exact power-of-two rescaling), the MFMA result is
// h_i / 2^e_ref, and v, c are scaled alike.  The conditional ratios
// P^s / sum P and the sign of w^T h + c do not depend on the common scale, so
// the scaling is exact in exact arithmetic and keeps every operand near 1.
// ---------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

__device__ inline f4 mfma_bf16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int CH>
__global__ __launch_bounds__(256) void k_psi_bf16(BF16Params P, const uint64_t* m, int64_t R,
                                                  double* lphi, int8_t* sphi, int rs, int wpb) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int TPC = CH / 16;
  constexpr int NT = 4 * TPC;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = lane & 15, g = lane >> 4;
  const size_t ring_elems = size_t(P.W) * 16 * rs;
  unsigned char* base = smem + size_t(wv) * (ring_elems * 2 + size_t(P.W) * 16 * 4);
  __bf16* ring = reinterpret_cast<__bf16*>(base);
  int* exps = reinterpret_cast<int*>(base + ring_elems * 2);
  const int64_t tile = int64_t(blockIdx.x) * wpb + wv;
  if (tile * 16 >= R) return;   // surplus wavefront of the last block (no block barrier below)
  const int64_t row = tile * 16 + j;
  const bool live = row < R;
  const int64_t rr = live ? row : (R - 1);
  const uint64_t lo = m[2 * rr], hi = m[2 * rr + 1];
  const bf8* Abase = reinterpret_cast<const bf8*>(P.A);
  double logacc = 0.0;
  int sgn = 1, ca = 0, cb = 0;
  bool bad = false;
  for (int i = 0; i < P.K; ++i) {
    f4 acc[NT];
#pragma unroll
    for (int ot = 0; ot < NT; ++ot) acc[ot] = f4{0, 0, 0, 0};
    const int e0 = P.pptr[i], d = P.pptr[i + 1] - e0;
    int eref = 0;
    if (d > 0) {
      eref = -100000;
      for (int e = 0; e < d; ++e) eref = max(eref, exps[(P.pidx[e0 + e] % P.W) * 16 + j]);
    }
    const int KQ = (d * CH + 31) / 32;
    const bf8* A = Abase + P.aoff[i] / 8 + lane;
    for (int q = 0; q < KQ; ++q) {
      const int k0 = 32 * q + 8 * g;
      const int el = k0 / CH, kk = k0 % CH;
      bf8 b;
      if (el < d) {
        const int slot = P.pidx[e0 + el] % P.W;
        b = *reinterpret_cast<const bf8*>(ring + (slot * 16 + j) * rs + kk);
        const int sh = exps[slot * 16 + j] - eref;
        if (sh != 0) {
#pragma unroll
          for (int t = 0; t < 8; ++t) b[t] = (__bf16)ldexpf(float(b[t]), sh);
        }
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) b[t] = (__bf16)0.0f;
      }
#pragma unroll
      for (int ot = 0; ot < NT; ++ot) acc[ot] = mfma_bf16(A[(q * NT + ot) * 64], b, acc[ot]);
    }
    const float sc = ldexpf(1.0f, -eref);
    const float* vi = P.v + size_t(i) * 4 * CH;
    const float* ei = P.eta + size_t(i) * CH;
    float ps[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      float p = 0;
#pragma unroll
      for (int t = 0; t < TPC; ++t) {
        const int u0 = 16 * t + 4 * g;
        const f4 vv = *reinterpret_cast<const f4*>(vi + s * CH + u0);
        const f4 ee = *reinterpret_cast<const f4*>(ei + u0);
        const f4 x = acc[s * TPC + t] + vv * sc;
        acc[s * TPC + t] = x;
        p += ee.x * x.x * x.x + ee.y * x.y * x.y + ee.z * x.z * x.z + ee.w * x.w * x.w;
      }
      p += __shfl_xor(p, 16);
      p += __shfl_xor(p, 32);
      ps[s] = p;
    }
    const int si = site_state(lo, hi, i);
    const int rest = P.K - 1 - i;
    float Z = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
      if (allowed(ca, cb, s, rest, P.na, P.nb)) Z += ps[s];
    if (!allowed(ca, cb, si, rest, P.na, P.nb)) bad = true;
    const float psi_ = si == 0 ? ps[0] : si == 1 ? ps[1] : si == 2 ? ps[2] : ps[3];
    logacc += 0.5 * (double(logf(psi_)) - double(logf(Z)));
    f4 sel[TPC];
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      sel[t] = acc[t];
#pragma unroll
      for (int s = 1; s < 4; ++s)
        if (si == s) sel[t] = acc[s * TPC + t];
    }
    const float* wi = P.w + size_t(i) * CH;
    float dot = 0, mx = 0;
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      const f4 ww = *reinterpret_cast<const f4*>(wi + 16 * t + 4 * g);
      dot += ww.x * sel[t].x + ww.y * sel[t].y + ww.z * sel[t].z + ww.w * sel[t].w;
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(sel[t].x), fabsf(sel[t].y)), fmaxf(fabsf(sel[t].z), fabsf(sel[t].w))));
    }
    dot += __shfl_xor(dot, 16);
    dot += __shfl_xor(dot, 32);
    dot += P.c[i] * sc;
    if (dot < 0) sgn = -sgn;
    mx = fmaxf(mx, __shfl_xor(mx, 16));
    mx = fmaxf(mx, __shfl_xor(mx, 32));
    int en = 0;
    if (mx > 0.0f) frexpf(mx, &en);
    const int slot_i = i % P.W;
    __bf16* wp = ring + (slot_i * 16 + j) * rs + 4 * g;
#pragma unroll
    for (int t = 0; t < TPC; ++t) {
      bf4 o;
      o[0] = (__bf16)ldexpf(sel[t].x, -en);
      o[1] = (__bf16)ldexpf(sel[t].y, -en);
      o[2] = (__bf16)ldexpf(sel[t].z, -en);
      o[3] = (__bf16)ldexpf(sel[t].w, -en);
      *reinterpret_cast<bf4*>(wp + 16 * t) = o;
    }
    if (g == 0) exps[slot_i * 16 + j] = eref + en;
    wave_sync();
    ca += si & 1;
    cb += si >> 1;
  }
  if (live && g == 0) {
    lphi[row] = bad ? -INFINITY : logacc;
    sphi[row] = int8_t(bad ? 0 : sgn);
  }
}

template <int CH>
hipError_t run_psi_bf16(const BF16Params& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                        hipStream_t st) {
  if (R <= 0) return hipSuccess;
  const int rs = CH + 8;
  const size_t per_wave = size_t(P.W) * 16 * rs * 2 + size_t(P.W) * 16 * 4;
  int wpb = 4;
  while (wpb > 1 && per_wave * wpb > 64 * 1024) wpb >>= 1;
  if (per_wave * wpb > 160 * 1024) return hipErrorInvalidValue;
  const int64_t tiles = (R + 15) / 16;
  const int64_t blocks = (tiles + wpb - 1) / wpb;
  hipLaunchKernelGGL((k_psi_bf16<CH>), dim3(unsigned(blocks)), dim3(64 * wpb), per_wave * wpb, st, P, m, R,
                     lphi, sphi, rs, wpb);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_psi_bf16(const BF16Params& P, const uint64_t* m, int64_t R, double* lphi,
                           int8_t* sphi, hipStream_t st) {
  switch (P.chip) {
    case 16: return run_psi_bf16<16>(P, m, R, lphi, sphi, st);
    case 32: return run_psi_bf16<32>(P, m, R, lphi, sphi, st);
    case 48: return run_psi_bf16<48>(P, m, R, lphi, sphi, st);
    case 64: return run_psi_bf16<64>(P, m, R, lphi, sphi, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nqs
