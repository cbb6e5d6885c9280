// Host runtime and C ABI of libnqs (include/nqs.h): contexts with a device
// workspace pool, resident Hamiltonian instances and ansatz parameter
// layouts, and the orchestration of the local-energy pipeline
// (enumerate -> screen -> draw -> rows -> amplitudes -> reduce) on one
// HIP stream.
#include "nqs.h"
#include "internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <limits>
#include <map>
#include <type_traits>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

using namespace nqs;

namespace {

thread_local std::string g_err;

// Allocation size classes of the workspace pool: multiples of 256 B up to
// 64 KiB, above that the power-of-two octave split in 8 steps (<= 12.5%
// rounding).  Blocks are reused only within the same class, so the bytes a
// call holds are exactly the sum of the classes of its requests.
size_t size_class(size_t bytes) {
  size_t b = std::max<size_t>(256, (bytes + 255) & ~size_t(255));
  if (b <= 65536) return b;
  int k = 63 - __builtin_clzll(b);            // 2^k <= b < 2^(k+1)
  const size_t step = size_t(1) << (k - 3);   // octave / 8
  return (b + step - 1) / step * step;
}

nqs_status fail(nqs_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(NQS_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(_e));               \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// context and workspace pool
// ---------------------------------------------------------------------------
struct nqs_ctx {
  int device = 0;
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;   // cached blocks by size
  std::map<void*, size_t> sizes;              // every block we own
  size_t in_use = 0, cached = 0, peak = 0;
  size_t cap = 0;                             // 0 = no limit on in_use + cached
  void* arena = nullptr;                      // this device's static workspace (nqs_eloc_noalloc)
  hipError_t arena_err = hipSuccess;          // its lookup's result
  int64_t fail_at = 0;                        // test hook: k-th acquire fails
  std::atomic<double> node_cap_scale{1.0};    // test hook: scales the node capacities
  // blocks handed back with work still queued on their stream: they count as
  // in use until the event recorded after that work has completed
  std::vector<std::pair<hipEvent_t, std::vector<void*>>> pending;

  void free_block_locked(void* p) {
    auto it = sizes.find(p);
    if (it == sizes.end()) return;
    in_use -= it->second;
    cached += it->second;
    free_blocks.emplace(it->second, p);
  }
  // move the pending blocks whose work has completed to the free list
  // (wait: block until all of them have)
  void reclaim_locked(bool wait) {
    for (size_t k = 0; k < pending.size();) {
      const hipError_t e = wait ? hipEventSynchronize(pending[k].first) : hipEventQuery(pending[k].first);
      if (e == hipErrorNotReady) {
        (void)hipGetLastError();   // not an error: keep it out of the next launch check
        ++k;
        continue;
      }
      if (e != hipSuccess) (void)hipGetLastError();
      (void)hipEventDestroy(pending[k].first);
      for (void* p : pending[k].second) free_block_locked(p);
      pending[k] = std::move(pending.back());
      pending.pop_back();
    }
  }
  void reclaim(bool wait) {
    std::lock_guard<std::mutex> lk(mu);
    reclaim_locked(wait);
  }
  void drop_cache() {
    for (auto& kv : free_blocks) { (void)hipFree(kv.second); sizes.erase(kv.second); }
    free_blocks.clear();
    cached = 0;
  }
  void* acquire(size_t bytes) {
    bytes = size_class(bytes);
    std::lock_guard<std::mutex> lk(mu);
    if (fail_at > 0 && --fail_at == 0) return nullptr;
    if (!pending.empty()) reclaim_locked(false);
    auto it = free_blocks.find(bytes);
    if (it != free_blocks.end()) {
      void* p = it->second;
      size_t sz = it->first;
      free_blocks.erase(it);
      cached -= sz;
      in_use += sz;
      peak = std::max(peak, in_use);
      return p;
    }
    while (cap && in_use + cached + bytes > cap && !free_blocks.empty()) {
      auto big = std::prev(free_blocks.end());          // release the largest cached block
      (void)hipFree(big->second);
      sizes.erase(big->second);
      cached -= big->first;
      free_blocks.erase(big);
    }
    if (cap && in_use + bytes > cap && !pending.empty()) {
      reclaim_locked(true);   // wait for the pending blocks, then try the cache again
      it = free_blocks.find(bytes);
      if (it != free_blocks.end()) {
        void* p = it->second;
        const size_t sz = it->first;
        free_blocks.erase(it);
        cached -= sz;
        in_use += sz;
        peak = std::max(peak, in_use);
        return p;
      }
      while (in_use + cached + bytes > cap && !free_blocks.empty()) {
        auto big = std::prev(free_blocks.end());
        (void)hipFree(big->second);
        sizes.erase(big->second);
        cached -= big->first;
        free_blocks.erase(big);
      }
    }
    if (cap && in_use + bytes > cap) return nullptr;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      reclaim_locked(true);
      drop_cache();   // release the cache and retry once
      if (hipMalloc(&p, bytes) != hipSuccess) { (void)hipGetLastError(); return nullptr; }
    }
    sizes[p] = bytes;
    in_use += bytes;
    peak = std::max(peak, in_use);
    return p;
  }
  void release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    free_block_locked(p);
  }
  // hand back blocks that work queued on `st` may still use: they return to
  // the free list once everything queued on `st` so far has completed
  void release_after(std::vector<void*>& ps, hipStream_t st) {
    if (ps.empty()) return;
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, st) != hipSuccess) {
      (void)hipGetLastError();
      if (ev) (void)hipEventDestroy(ev);
      (void)hipStreamSynchronize(st);   // no event: wait for the stream instead
      (void)hipGetLastError();
      std::lock_guard<std::mutex> lk(mu);
      for (void* p : ps) free_block_locked(p);
      ps.clear();
      return;
    }
    std::lock_guard<std::mutex> lk(mu);
    pending.emplace_back(ev, std::move(ps));
    ps.clear();
  }
  ~nqs_ctx() {
    for (auto& pe : pending) {
      (void)hipEventSynchronize(pe.first);
      (void)hipEventDestroy(pe.first);
    }
    for (auto& kv : sizes) (void)hipFree(kv.first);
  }
};

namespace {

// Bump allocator over a fixed device array (the static workspace of the
// allocation-free entry point): one per call; the workspaces of the call
// take consecutive 256-byte aligned pieces and give them back in reverse
// order.  Reuse of a piece by a later phase of the same call is ordered by
// the call's stream.
struct Arena {
  unsigned char* base = nullptr;
  size_t size = 0, off = 0;
  bool overflow = false;
};

// Workspace of one call on one stream: when the call returns (on any path,
// errors included) its blocks go back to the pool behind the work queued on
// that stream, so no other call is handed a block a queued kernel may still
// write.  With an arena the blocks come from it instead and nothing is
// allocated.
struct Scratch {
  nqs_ctx* ctx;
  hipStream_t st;
  Arena* arena;
  size_t arena_start = 0;
  std::vector<void*> blocks;
  bool oom = false;
  Scratch(nqs_ctx* c, hipStream_t s, Arena* a = nullptr) : ctx(c), st(s), arena(a) {
    if (arena) arena_start = arena->off;
  }
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  template <typename T>
  T* get(size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    if (arena) {
      const size_t need = (bytes + 255) / 256 * 256;
      if (arena->overflow || arena->size - arena->off < need) {
        arena->overflow = true;
        oom = true;
        return nullptr;
      }
      void* p = arena->base + arena->off;
      arena->off += need;
      return static_cast<T*>(p);
    }
    void* p = ctx->acquire(bytes);
    if (!p) { oom = true; return nullptr; }
    blocks.push_back(p);
    return static_cast<T*>(p);
  }
  ~Scratch() {
    if (arena) arena->off = arena_start;
    else ctx->release_after(blocks, st);
  }
};

uint64_t magic(uint64_t d) { return d == 0 ? 0 : ((uint64_t(1) << 32) + d - 1) / d; }

int64_t choose2(int64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }

}  // namespace

// ---------------------------------------------------------------------------
// instance
// ---------------------------------------------------------------------------
struct nqs_instance {
  nqs_ctx* ctx = nullptr;
  int device = 0;           // the context's device, kept for destruction after the context
  int K = 0, na = 0, nb = 0;
  double ecore = 0;
  double* d_h = nullptr;
  double* d_eri = nullptr;
  double* d_jk = nullptr;
  double* d_s3 = nullptr;
  HamDev H{};
  ~nqs_instance() {
    if (d_h) (void)hipFree(d_h);
    if (d_eri) (void)hipFree(d_eri);
    if (d_jk) (void)hipFree(d_jk);
    if (d_s3) (void)hipFree(d_s3);
  }
};

// ---------------------------------------------------------------------------
// ansatz
// ---------------------------------------------------------------------------
template <typename T>
struct PsiLayout {
  T* A = nullptr;           // forward: per forward edge, then one zero edge
  T* v = nullptr;
  T* eta = nullptr;
  T* w = nullptr;
  T* c = nullptr;
  T* w2 = nullptr;          // complex parameters: [K][chip] vector of Im z, (folded like w)
  T* c2 = nullptr;          // [K]
  T* TA = nullptr;          // BDG-TensorRNN term on MFMA (PsiParams::TA)
  T* AF = nullptr;          // adjoint: recompute operands (k-permuted)
  int64_t* afoff = nullptr;
  T* BT = nullptr;          // adjoint: M^T operands
  int64_t* btoff = nullptr;
  bool folded = false;      // operands carry sqrt(eta)
  void free_all() {
    for (void* p : {(void*)A, (void*)v, (void*)eta, (void*)w, (void*)c, (void*)w2, (void*)c2, (void*)TA,
                    (void*)AF, (void*)afoff, (void*)BT, (void*)btoff})
      if (p) (void)hipFree(p);
    A = nullptr; v = eta = w = c = w2 = c2 = TA = nullptr;
    AF = nullptr; afoff = nullptr; BT = nullptr; btoff = nullptr;
  }
};

struct nqs_ansatz {
  nqs_ctx* ctx = nullptr;
  int device = 0;           // the context's device, kept for destruction after the context
  int K = 0, na = 0, nb = 0, chi = 0, chip = 0, nh = 0, W = 1;
  bool d1 = false;          // every site has exactly one forward edge (a chain: the single-edge kernels)
  std::vector<int32_t> pptr, pidx;
  std::vector<int64_t> offM, offV, offEta, offW, offC;
  int64_t offB = 0, offWc = 0, n_params = 0;
  int* d_pptr = nullptr;
  int* d_pidx = nullptr;
  int* d_slot = nullptr;    // ring slot of each parent edge (pidx % W)
  int* d_fptr = nullptr;    // forward edge CSR: every parentless site gets one zero-weight edge
  int* d_fslot = nullptr;   // forward edge: ring slot of the parent's state (ring: the zero edge)
  int ring = 1;             // LDS ring slots of the forward kernels (states live at once)
  int* d_wsl = nullptr;     // [K] ring slot receiving site i's state
  uint64_t* d_live = nullptr;   // [K+1] bit s: the state of site s < i is read by a site >= i
  bool bound = false;
  PsiLayout<double> L64, F64;   // F*: sqrt(eta)-folded forward layouts (when every eta > 0)
  PsiLayout<float> L32, F32;
  bool has_fold = false;
  uint16_t* bfA = nullptr;  // BF16 forward A stream (folded when has_fold)
  uint16_t* bfAlo = nullptr;  // its lo parts: bf16(x - bf16(x)), for the split BF16 form
  double* d_cb = nullptr;   // correlator b
  double* d_cW = nullptr;   // correlator W
  bool ising = false;       // Ising-RBM correlator (quadratic couplings W2)
  int64_t offW2 = 0;
  double* d_cW1t = nullptr; // Ising-RBM: W transposed [2K][nh]
  double* d_cS = nullptr;   // Ising-RBM: (W2 + W2^T)/2 as [2K][2K][nh]
  float* d_cS32 = nullptr;  // the same in FP32
  // BDG-TensorRNN: per site chi' (0: no tensor term) and the packed offsets of
  // the factor matrices and cores; kernel tables and per-precision layouts
  bool tensor = false;
  std::vector<int> tq;
  std::vector<int64_t> offTK, offTU;
  int* d_tn_edge = nullptr;
  int* d_tn_site = nullptr;
  double* tn64 = nullptr;
  float* tn32 = nullptr;
  int64_t tn_size = 0;
  int tn_qp = 16;           // 8 when every chi' <= 8
  bool tn_f64_ok = true;    // the FP64 ring fits the LDS
  std::vector<int> tn_edge_host, tn_site_host;
  // the tensor term on the MFMA forward (chip <= 32 and every chi' <= 8): per
  // site {chi', offsets of projections, core, output factor} in PsiLayout::TA
  bool tn_mfma = false;
  std::vector<int> tsite_host;
  int64_t ta_size = 0;
  int* d_tsite = nullptr;
  int64_t* d_offM = nullptr;
  int64_t* d_offV = nullptr;
  int64_t* d_offEta = nullptr;
  // Complex parameters: the kernels see the realified ansatz (chi = 2 chi_c
  // real units, block matrices); its packed vector (nr_params) is the real
  // layout, the correlator, then per site w2 (2 chi_c) and c2 at offW2x /
  // offC2x.  n_params and cx_* describe the caller's packed complex layout.
  bool cplx = false;
  int chi_c = 0;
  int64_t nr_params = 0;
  std::vector<int64_t> offW2x, offC2x, cx_offM, cx_offV, cx_offEta, cx_offW, cx_offC;
  int64_t cx_offB = 0;
  int64_t* d_cx = nullptr;  // device: rW, rC, rW2, rC2, cV, cEta, cW, cC ([K] each), then cM ([edges])
  ~nqs_ansatz() {
    L64.free_all();
    L32.free_all();
    F64.free_all();
    F32.free_all();
    for (void* p : {(void*)d_pptr, (void*)d_pidx, (void*)d_slot, (void*)d_fptr, (void*)d_fslot, (void*)d_wsl,
                    (void*)d_live, (void*)bfA,
                    (void*)bfAlo,
                    (void*)d_cb, (void*)d_cW, (void*)d_cW1t, (void*)d_cS, (void*)d_cS32, (void*)d_tn_edge,
                    (void*)d_tn_site, (void*)tn64, (void*)tn32, (void*)d_offM, (void*)d_offV,
                    (void*)d_offEta, (void*)d_cx, (void*)d_tsite})
      if (p) (void)hipFree(p);
  }
  template <typename T>
  AdjParams<T> adj(const PsiLayout<T>& L) const {
    AdjParams<T> P;
    P.K = K; P.chi = chi; P.chip = chip; P.na = na; P.nb = nb;
    P.pptr = d_pptr; P.pidx = d_pidx; P.pptr_host = pptr.data();
    P.AF = L.AF; P.afoff = L.afoff; P.BT = L.BT; P.btoff = L.btoff;
    P.v = L.v; P.eta = L.eta;
    P.offM = d_offM; P.offV = d_offV; P.offEta = d_offEta;
    return P;
  }
  template <typename T>
  PsiParams<T> params(const PsiLayout<T>& L) const {
    PsiParams<T> P;
    P.K = K; P.chi = chi; P.chip = chip; P.na = na; P.nb = nb; P.W = ring;
    P.d1 = d1;
    P.pptr = d_fptr; P.slot = d_fslot; P.wsl = d_wsl; P.live = d_live;
    P.A = L.A; P.v = L.v; P.eta = L.eta; P.w = L.w; P.c = L.c;
    P.folded = L.folded;
    P.w2 = L.w2; P.c2 = L.c2;
    P.TA = tn_mfma ? L.TA : nullptr;
    P.tsite = d_tsite;
    return P;
  }
  CxMap cxmap() const {
    CxMap M;
    M.K = K; M.chi = chi_c; M.n_edges = pptr[K];
    M.pptr = d_pptr;
    M.rM = d_offM; M.rV = d_offV; M.rEta = d_offEta;
    M.rW = d_cx; M.rC = d_cx + K; M.rW2 = d_cx + 2 * K; M.rC2 = d_cx + 3 * K;
    M.cV = d_cx + 4 * K; M.cEta = d_cx + 5 * K; M.cW = d_cx + 6 * K; M.cC = d_cx + 7 * K;
    M.cM = d_cx + 8 * K;
    M.r_corr = offB; M.c_corr = cx_offB; M.n_corr = n_params - cx_offB;
    return M;
  }
  // forward layout for amplitudes without a carried-state store
  const PsiLayout<double>& fwd64() const { return has_fold ? F64 : L64; }
  const PsiLayout<float>& fwd32() const { return has_fold ? F32 : L32; }
  template <typename T>
  TnParams<T> tn(const T* prm) const {
    TnParams<T> P;
    P.K = K; P.chi = chi; P.chip = chip; P.rw = (chi + 3) / 4 * 4; P.na = na; P.nb = nb; P.W = W; P.qp = tn_qp;
    P.prm = prm; P.pptr = d_pptr; P.edge = d_tn_edge; P.site = d_tn_site;
    return P;
  }
  CorrParams corr() const {
    CorrParams C;
    C.K = K; C.nh = nh; C.b = d_cb; C.W = d_cW;
    C.ising = ising ? 1 : 0; C.W1t = d_cW1t; C.S = d_cS; C.S32 = d_cS32;
    return C;
  }
};

namespace {

template <typename T>
nqs_status upload(T** dst, const std::vector<T>& src) {
  HIPCHK(hipMalloc((void**)dst, std::max<size_t>(src.size(), 1) * sizeof(T)));
  if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return NQS_OK;
}

// Forward MFMA A operands: W_i^T tiles over the forward edges (the parents of
// each site in order; a parentless site gets one zero edge), then one more
// zero edge so that the kernel's one-edge-ahead fetch stays in bounds.  Per
// edge [k-step q][output tile ot][lane]: lane l holds W^T[o][k] = M_ij^s[u][k]
// with s = o / chip, u = o % chip (zero outside chi), tile row m = l%16 and
// parent unit k = 16 (q/4) + 4 (l/16) + q%4.  The 16x16x4 f32 MFMA returns
// row m = 4 g + v of the tile in register v of lane group g = lane/16; the f64
// MFMA returns row m = g + 4 v.  Tile row m therefore carries unit
// o = 16 ot + m for f32 and o = 16 ot + 4 (m%4) + m/4 for f64, so that in both
// cases lane group g ends up with units 16 ot + 4 g + v, and k-step q of lane
// group g reads the parent unit that the same lane produced in register q%4 of
// output tile q/4.
//
// fold = true: every operand carries sigma = sqrt(eta) (requires eta > 0):
// A' = sigma_i[u] M[u][k] / sigma_j[k], v' = sigma_i v, w' = w / sigma_i, so the
// forward kernel carries sigma h and P^s = sum x'^2.  The adjoint operands are
// built only for the unfolded layout.
template <typename T>
nqs_status build_layout(nqs_ansatz* a, const std::vector<double>& prm, PsiLayout<T>& L, bool fold) {
  const int K = a->K, chi = a->chi, CH = a->chip;
  const int KS = CH / 4, NT = CH / 4;
  const size_t ES = size_t(KS) * NT * 64;
  std::vector<double> sig(size_t(K) * chi, 1.0);
  if (fold)
    for (int i = 0; i < K; ++i)
      for (int u = 0; u < chi; ++u) sig[size_t(i) * chi + u] = std::sqrt(prm[a->offEta[i] + u]);
  std::vector<T> A;
  for (int i = 0; i < K; ++i) {
    if (a->pptr[i + 1] == a->pptr[i]) A.resize(A.size() + ES, T(0));   // zero edge
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) {
      const double* M = prm.data() + a->offM[e];
      const double* sj = sig.data() + size_t(a->pidx[e]) * chi;
      const double* si = sig.data() + size_t(i) * chi;
      for (int q = 0; q < KS; ++q)
        for (int ot = 0; ot < NT; ++ot)
          for (int l = 0; l < 64; ++l) {
            const int mrow = l & 15;
            const int o = ot * 16 + (sizeof(T) == 8 ? 4 * (mrow & 3) + (mrow >> 2) : mrow);
            const int k = 16 * (q >> 2) + 4 * (l >> 4) + (q & 3);
            const int s = o / CH, u = o % CH;
            double val = 0.0;
            if (u < chi && k < chi) val = si[u] * M[(size_t(s) * chi + u) * chi + k] / sj[k];
            A.push_back(T(val));
          }
    }
  }
  A.resize(A.size() + ES, T(0));   // fetch-ahead edge
  std::vector<T> v(size_t(K) * 4 * CH, T(0)), eta(size_t(K) * CH, T(0)), w(size_t(K) * CH, T(0)), c(K);
  for (int i = 0; i < K; ++i) {
    const double* si = sig.data() + size_t(i) * chi;
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < chi; ++u)
        v[(size_t(i) * 4 + s) * CH + u] = T(si[u] * prm[a->offV[i] + s * chi + u]);
    for (int u = 0; u < chi; ++u) {
      eta[size_t(i) * CH + u] = T(prm[a->offEta[i] + u]);
      w[size_t(i) * CH + u] = T(prm[a->offW[i] + u] / si[u]);
    }
    c[i] = T(prm[a->offC[i]]);
  }
  std::vector<T> w2, c2;
  if (a->cplx) {
    w2.assign(size_t(K) * CH, T(0));
    c2.resize(K);
    for (int i = 0; i < K; ++i) {
      const double* si = sig.data() + size_t(i) * chi;
      for (int u = 0; u < chi; ++u) w2[size_t(i) * CH + u] = T(prm[a->offW2x[i] + u] / si[u]);
      c2[i] = T(prm[a->offC2x[i]]);
    }
  }
  // the tensor term's MFMA operands (see PsiParams::TA); A row m of a tile
  // carries logical row o(m) so that lane group g holds rows 4g + v in its
  // output registers v (f64 MFMA rows g + 4v)
  std::vector<T> TA;
  if (a->tn_mfma) {
    TA.assign(a->ta_size, T(0));
    auto orow = [](int m) { return sizeof(T) == 8 ? 4 * (m & 3) + (m >> 2) : m; };
    const int KSq = CH / 4, TPCq = CH / 16;
    for (int i = 0; i < K; ++i) {
      const int Q = a->tsite_host[4 * i];
      if (!Q) continue;
      const int d = a->pptr[i + 1] - a->pptr[i];
      const double* si = sig.data() + size_t(i) * chi;
      T* P0 = TA.data() + a->tsite_host[4 * i + 1];
      T* C0 = TA.data() + a->tsite_host[4 * i + 2];
      T* K0s = TA.data() + a->tsite_host[4 * i + 3];
      const double* Kp = prm.data() + a->offTK[i];            // K^(0..d), chi x chi' each
      const double* Up = prm.data() + a->offTU[i];            // U^s, chi'^(d+1) each
      // projections: output row o -> p index a = 2 (o / 4) + o % 4 for o % 4 < 2
      for (int jx = 0; jx < d; ++jx) {
        const double* sj = sig.data() + size_t(a->pidx[a->pptr[i] + jx]) * chi;
        for (int q = 0; q < KSq; ++q)
          for (int l = 0; l < 64; ++l) {
            const int o = orow(l & 15), pa = 2 * (o >> 2) + (o & 3);
            const int k = 16 * (q >> 2) + 4 * (l >> 4) + (q & 3);
            double val = 0.0;
            if ((o & 3) < 2 && pa < Q && k < chi) val = Kp[size_t(jx + 1) * chi * Q + size_t(k) * Q + pa] / sj[k];
            P0[(size_t(jx) * KSq + q) * 64 + l] = T(val);
          }
      }
      // core: k-step kk = (a_1 [, a_2]) * 2 + v, lane group g supplies a_d = 2 g + v;
      // tile mt row o holds (s, i') = ((16 mt + o) / 8, (16 mt + o) % 8)
      int nlead = 1;
      for (int k = 0; k < d - 1; ++k) nlead *= Q;
      size_t qd = 1;
      for (int k = 0; k < d; ++k) qd *= Q;
      for (int kk = 0; kk < nlead * 2; ++kk)
        for (int mt = 0; mt < 2; ++mt)
          for (int l = 0; l < 64; ++l) {
            const int row = 16 * mt + orow(l & 15), s_ = row / 8, ip = row % 8;
            const int ad = 2 * (l >> 4) + (kk & 1), lead = kk >> 1;
            double val = 0.0;
            if (ip < Q && ad < Q) val = Up[(size_t(s_) * Q + ip) * qd + size_t(lead) * Q + ad];
            C0[(size_t(kk) * 2 + mt) * 64 + l] = T(val);
          }
      // output factor: for state s, tile tt, k-step v, lane group g supplies the q
      // row 4g + v of core tile s / 2, i.e. (s', i') = (2 (s / 2) + g / 2, 4 (g % 2) + v)
      for (int s_ = 0; s_ < 4; ++s_)
        for (int tt = 0; tt < TPCq; ++tt)
          for (int v = 0; v < 4; ++v)
            for (int l = 0; l < 64; ++l) {
              const int u = 16 * tt + orow(l & 15), g = l >> 4;
              const int sq = 2 * (s_ / 2) + g / 2, ip = 4 * (g % 2) + v;
              double val = 0.0;
              if (sq == s_ && ip < Q && u < chi) val = si[u] * Kp[size_t(u) * Q + ip];
              K0s[((size_t(s_) * TPCq + tt) * 4 + v) * 64 + l] = T(val);
            }
    }
  }
  auto upload_cx = [&]() -> nqs_status {
    nqs_status st;
    if (a->tn_mfma && (st = upload(&L.TA, TA)) != NQS_OK) return st;
    if (!a->cplx) return NQS_OK;
    if ((st = upload(&L.w2, w2)) != NQS_OK) return st;
    return upload(&L.c2, c2);
  };
  if (fold) {
    L.free_all();
    L.folded = true;
    nqs_status st;
    if ((st = upload(&L.A, A)) != NQS_OK) return st;
    if ((st = upload(&L.v, v)) != NQS_OK) return st;
    if ((st = upload(&L.eta, eta)) != NQS_OK) return st;
    if ((st = upload(&L.w, w)) != NQS_OK) return st;
    if ((st = upload(&L.c, c)) != NQS_OK) return st;
    return upload_cx();
  }
  // adjoint operands.  AF: like A but k-step q = 4t + v pairs lane group k'
  // with parent unit 16t + 4k' + v.  BT: k-step q = (s*TPC + t)*4 + v over the
  // candidate units (s, 16t + 4k' + v) and output tiles ot over the parent
  // unit kk = 16 ot + n: B[k'][n] = M_ij^s[u][kk].
  const int TPC = CH / 16;
  std::vector<int64_t> afoff(K), btoff(K);
  std::vector<T> AF, BT;
  for (int i = 0; i < K; ++i) {
    afoff[i] = int64_t(AF.size());
    btoff[i] = int64_t(BT.size());
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) {
      const double* M = prm.data() + a->offM[e];
      for (int q = 0; q < KS; ++q)
        for (int ot = 0; ot < NT; ++ot)
          for (int l = 0; l < 64; ++l) {
            const int mrow = l & 15;
            const int o = ot * 16 + (sizeof(T) == 8 ? 4 * (mrow & 3) + (mrow >> 2) : mrow);
            const int k = 16 * (q >> 2) + 4 * (l >> 4) + (q & 3);
            const int s = o / CH, u = o % CH;
            double val = 0.0;
            if (u < chi && k < chi) val = M[(size_t(s) * chi + u) * chi + k];
            AF.push_back(T(val));
          }
      for (int q = 0; q < 4 * KS; ++q)
        for (int ot = 0; ot < TPC; ++ot)
          for (int l = 0; l < 64; ++l) {
            const int v = q & 3, t = (q >> 2) % TPC, s = (q >> 2) / TPC;
            const int u = 16 * t + 4 * (l >> 4) + v;
            const int kk = 16 * ot + (l & 15);
            double val = 0.0;
            if (u < chi && kk < chi) val = M[(size_t(s) * chi + u) * chi + kk];
            BT.push_back(T(val));
          }
    }
  }
  L.free_all();
  nqs_status st;
  if ((st = upload(&L.AF, AF)) != NQS_OK) return st;
  if ((st = upload(&L.afoff, afoff)) != NQS_OK) return st;
  if ((st = upload(&L.BT, BT)) != NQS_OK) return st;
  if ((st = upload(&L.btoff, btoff)) != NQS_OK) return st;
  if ((st = upload(&L.A, A)) != NQS_OK) return st;
  if ((st = upload(&L.v, v)) != NQS_OK) return st;
  if ((st = upload(&L.eta, eta)) != NQS_OK) return st;
  if ((st = upload(&L.w, w)) != NQS_OK) return st;
  if ((st = upload(&L.c, c)) != NQS_OK) return st;
  return upload_cx();
}

// round-to-nearest-even FP32 -> BF16 bit pattern (finite inputs)
uint16_t to_bf16(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return uint16_t(b >> 16);
}

// BF16 forward A stream (psi_bf16.hip): per forward edge (a parentless site
// has one zero edge; one more zero edge at the end), TPC/2 pair k-steps of
// [output tile ot][lane][8] then, when TPC = chip/16 is odd, one k-step of
// [ot][lane][4].  Lane l holds tile row m = l%16 (output unit o = 16 ot + m,
// the FP32 output layout) and, for lane group g = l/16, the parent units
// k = 16 (2q + e/4) + 4 g + e%4 (pair step q, element e) or 16 (TPC-1) + 4 g + e
// (odd step): each lane's own quads of the parent state.  With fold the
// operands carry sigma = sqrt(eta) as in build_layout.  Round to nearest even.
// A second stream of the same layout holds the lo parts of the split form:
// bf16(x - bf16(x)) with the difference taken in FP64.
nqs_status build_bf16(nqs_ansatz* a, const std::vector<double>& prm, bool fold) {
  const int K = a->K, chi = a->chi, CH = a->chip, NT = CH / 4, TPC = CH / 16, NP = TPC / 2;
  const size_t EQ = size_t(NP) * NT * 64 * 8 + size_t(TPC & 1) * NT * 64 * 4;   // bf16 values per edge
  std::vector<double> sig(size_t(K) * chi, 1.0);
  if (fold)
    for (int i = 0; i < K; ++i)
      for (int u = 0; u < chi; ++u) sig[size_t(i) * chi + u] = std::sqrt(prm[a->offEta[i] + u]);
  std::vector<uint16_t> A, Alo;
  auto value = [&](int e, int i, int o, int k) {
    const int s = o / CH, u = o % CH;
    if (u >= chi || k >= chi) {
      Alo.push_back(0);
      return uint16_t(0);
    }
    const double* M = prm.data() + a->offM[e];
    const double v = sig[size_t(i) * chi + u] * M[(size_t(s) * chi + u) * chi + k] /
                     sig[size_t(a->pidx[e]) * chi + k];
    const uint16_t hi = to_bf16(float(v));
    uint32_t bits = uint32_t(hi) << 16;
    float fhi;
    std::memcpy(&fhi, &bits, 4);
    Alo.push_back(to_bf16(float(v - double(fhi))));
    return hi;
  };
  for (int i = 0; i < K; ++i) {
    if (a->pptr[i + 1] == a->pptr[i]) {   // zero edge
      A.resize(A.size() + EQ, 0);
      Alo.resize(Alo.size() + EQ, 0);
    }
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) {
      for (int q = 0; q < NP; ++q)
        for (int ot = 0; ot < NT; ++ot)
          for (int l = 0; l < 64; ++l)
            for (int el = 0; el < 8; ++el)
              A.push_back(value(e, i, 16 * ot + (l & 15), 16 * (2 * q + el / 4) + 4 * (l >> 4) + el % 4));
      if (TPC & 1)
        for (int ot = 0; ot < NT; ++ot)
          for (int l = 0; l < 64; ++l)
            for (int el = 0; el < 4; ++el)
              A.push_back(value(e, i, 16 * ot + (l & 15), 16 * (TPC - 1) + 4 * (l >> 4) + el));
    }
  }
  A.resize(A.size() + EQ, 0);   // fetch-ahead edge
  Alo.resize(Alo.size() + EQ, 0);
  if (a->bfA) { (void)hipFree(a->bfA); a->bfA = nullptr; }
  if (a->bfAlo) { (void)hipFree(a->bfAlo); a->bfAlo = nullptr; }
  nqs_status st = upload(&a->bfA, A);
  return st != NQS_OK ? st : upload(&a->bfAlo, Alo);
}

// algorithmic flops of one site of one row: 8 chi^2 d (four candidates, d
// parents); with a tensor term also the projections (d chi chi' MACs), the
// core (4 chi'^(d+1)) and the output factor (4 chi chi')
double site_flops(const nqs_ansatz& a, int i) {
  const int d = a.pptr[i + 1] - a.pptr[i];
  double f = 8.0 * a.chi * a.chi * d;
  const int q = a.tensor ? a.tq[i] : 0;
  if (q) {
    double qd = 1;
    for (int k = 0; k <= d; ++k) qd *= q;
    f += 2.0 * (double(d) * a.chi * q + 4.0 * qd + 4.0 * a.chi * q);
  }
  return f;
}

// BDG-TensorRNN kernel layout (see TnParams) in FP64 and FP32, zero-padded to
// chip units and to 16 projection columns
nqs_status build_tn(nqs_ansatz* a, const std::vector<double>& prm) {
  const int K = a->K, chi = a->chi, cp = a->chip;
  std::vector<double> L(size_t(a->tn_size), 0.0);
  for (int i = 0; i < K; ++i) {
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) {
      double* Mt = L.data() + a->tn_edge_host[2 * e];
      for (int s = 0; s < 4; ++s)
        for (int u = 0; u < chi; ++u)
          for (int k = 0; k < chi; ++k)
            Mt[(size_t(s) * cp + k) * cp + u] = prm[a->offM[e] + (size_t(s) * chi + u) * chi + k];
    }
    const int* st8 = a->tn_site_host.data() + 8 * i;
    for (int s = 0; s < 4; ++s)
      for (int u = 0; u < chi; ++u) L[st8[0] + s * cp + u] = prm[a->offV[i] + s * chi + u];
    for (int u = 0; u < chi; ++u) {
      L[st8[1] + u] = prm[a->offEta[i] + u];
      L[st8[2] + u] = prm[a->offW[i] + u];
    }
    L[st8[3]] = prm[a->offC[i]];
    const int q = a->tq[i], d = a->pptr[i + 1] - a->pptr[i];
    if (!q) continue;
    const double* Kp = prm.data() + a->offTK[i];   // K^(0..d), each [chi][q]
    for (int ip = 0; ip < q; ++ip)
      for (int u = 0; u < chi; ++u) L[st8[5] + size_t(ip) * cp + u] = Kp[size_t(u) * q + ip];
    const int qp = a->tn_qp;
    for (int j = 0; j < d; ++j)
      for (int v = 0; v < chi; ++v)
        for (int b = 0; b < q; ++b)
          L[st8[6] + (size_t(j) * cp + v) * qp + b] = Kp[size_t(j + 1) * chi * q + size_t(v) * q + b];
    int64_t qd = 1;
    for (int k = 0; k <= d; ++k) qd *= q;
    for (int64_t f = 0; f < 4 * qd; ++f) L[st8[7] + (f / q) * qp + f % q] = prm[a->offTU[i] + f];
  }
  if (a->tn64) { (void)hipFree(a->tn64); a->tn64 = nullptr; }
  if (a->tn32) { (void)hipFree(a->tn32); a->tn32 = nullptr; }
  nqs_status st;
  if ((st = upload(&a->tn64, L)) != NQS_OK) return st;
  std::vector<float> L32(L.begin(), L.end());
  return upload(&a->tn32, L32);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* nqs_last_error(void) { return g_err.c_str(); }
const char* nqs_version(void) { return "nqs-eloc gfx950 0.1"; }

nqs_status nqs_ctx_create(int device, nqs_ctx** out) {
  if (!out) return fail(NQS_EINVAL, "out is NULL");
  int n = 0;
  HIPCHK(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(NQS_EINVAL, "device %d out of range (%d devices)", device, n);
  DeviceGuard g(device);
  HIPCHK(hipFree(nullptr));
  auto* c = new nqs_ctx();
  c->device = device;
  // this device's static workspace (once per device; only nqs_eloc_noalloc uses it)
  c->arena_err = static_workspace_setup(device);
  if (c->arena_err == hipSuccess) c->arena = static_workspace(device);
  *out = c;
  return NQS_OK;
}

int nqs_ctx_device(const nqs_ctx* ctx) { return ctx ? ctx->device : -1; }

nqs_status nqs_ctx_destroy(nqs_ctx* ctx) {
  if (!ctx) return NQS_OK;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  delete ctx;
  return NQS_OK;
}

nqs_status nqs_ctx_fail_alloc_at(nqs_ctx* ctx, int64_t k) {
  if (!ctx || k < 0) return fail(NQS_EINVAL, "bad arguments");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->fail_at = k;
  return NQS_OK;
}

nqs_status nqs_ctx_set_node_capacity(nqs_ctx* ctx, double scale) {
  if (!ctx || !(scale > 0.0 && scale <= 1.0)) return fail(NQS_EINVAL, "scale must be in (0, 1]");
  ctx->node_cap_scale.store(scale);
  return NQS_OK;
}

nqs_status nqs_ctx_pool_bytes(const nqs_ctx* ctx, size_t* in_use, size_t* cached) {
  if (!ctx) return fail(NQS_EINVAL, "ctx is NULL");
  auto* c = const_cast<nqs_ctx*>(ctx);
  std::lock_guard<std::mutex> lk(c->mu);
  c->reclaim_locked(true);   // blocks still behind queued work count once that work is done
  if (in_use) *in_use = c->in_use;
  if (cached) *cached = c->cached;
  return NQS_OK;
}

nqs_status nqs_ctx_pool_peak(nqs_ctx* ctx, size_t* peak, int reset) {
  if (!ctx) return fail(NQS_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->reclaim_locked(true);   // a reset starts from the blocks still in use, not those behind finished work
  if (peak) *peak = ctx->peak;
  if (reset) ctx->peak = ctx->in_use;
  return NQS_OK;
}

nqs_status nqs_ctx_set_pool_limit(nqs_ctx* ctx, size_t bytes) {
  if (!ctx) return fail(NQS_EINVAL, "ctx is NULL");
  DeviceGuard g(ctx->device);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->cap = bytes;
  if (bytes && ctx->in_use + ctx->cached > bytes) ctx->drop_cache();
  return NQS_OK;
}

nqs_status nqs_instance_create(nqs_ctx* ctx, int K, int n_alpha, int n_beta, const double* h1,
                               const double* eri, double e_core, nqs_instance** out) {
  if (!ctx || !h1 || !eri || !out) return fail(NQS_EINVAL, "NULL argument");
  if (K < 1 || K > 64) return fail(NQS_EINVAL, "K=%d outside [1,64]", K);
  if (n_alpha < 0 || n_alpha > K || n_beta < 0 || n_beta > K)
    return fail(NQS_EINVAL, "electron counts (%d,%d) outside [0,K]", n_alpha, n_beta);
  const size_t K2 = size_t(K) * K, K4 = K2 * K2;
  // non-finite values would pass the symmetry checks below (every comparison
  // with NaN is false) and then screen as garbage
  if (!std::isfinite(e_core)) return fail(NQS_EINVAL, "e_core is not finite");
  for (size_t t = 0; t < K2; ++t)
    if (!std::isfinite(h1[t])) return fail(NQS_EINVAL, "h has a non-finite entry at %zu", t);
  for (size_t t = 0; t < K4; ++t)
    if (!std::isfinite(eri[t])) return fail(NQS_EINVAL, "eri has a non-finite entry at %zu", t);
  for (int p = 0; p < K; ++p)
    for (int q = 0; q < K; ++q)
      if (std::fabs(h1[p * K + q] - h1[q * K + p]) > 1e-10 * (1.0 + std::fabs(h1[p * K + q])))
        return fail(NQS_EINVAL, "h is not symmetric at (%d,%d)", p, q);
  double emax = 0.0;
  for (size_t t = 0; t < K4; ++t) emax = std::max(emax, std::fabs(eri[t]));
  const double tol = 1e-10 * std::max(emax, 1e-300);
  std::vector<double> canon(K4);
  auto at = [&](size_t p, size_t q, size_t r, size_t s) { return ((p * K + q) * K + r) * K + s; };
  for (size_t p = 0; p < size_t(K); ++p)
    for (size_t q = 0; q < size_t(K); ++q)
      for (size_t r = 0; r < size_t(K); ++r)
        for (size_t s = 0; s < size_t(K); ++s) {
          size_t a = std::max(p, q), b = std::min(p, q), c = std::max(r, s), d = std::min(r, s);
          size_t ab = a * (a + 1) / 2 + b, cd = c * (c + 1) / 2 + d;
          if (ab < cd) { std::swap(a, c); std::swap(b, d); }
          const double ref = eri[at(a, b, c, d)];
          const double v = eri[at(p, q, r, s)];
          if (std::fabs(v - ref) > tol)
            return fail(NQS_EINVAL, "eri not 8-fold symmetric at (%zu,%zu,%zu,%zu)", p, q, r, s);
          canon[at(p, q, r, s)] = ref;
        }
  std::vector<double> hs(h1, h1 + K2);
  for (int p = 0; p < K; ++p)
    for (int q = 0; q < p; ++q) hs[q * K + p] = hs[p * K + q];
  DeviceGuard g(ctx->device);
  std::unique_ptr<nqs_instance> inst(new nqs_instance());
  inst->ctx = ctx;
  inst->device = ctx->device;
  inst->K = K; inst->na = n_alpha; inst->nb = n_beta; inst->ecore = e_core;
  nqs_status st;
  if ((st = upload(&inst->d_h, hs)) != NQS_OK) return st;
  if ((st = upload(&inst->d_eri, canon)) != NQS_OK) return st;
  std::vector<double> jk(size_t(2) * K * K);
  for (int p = 0; p < K; ++p)
    for (int q = 0; q < K; ++q) {
      jk[size_t(p) * K + q] = canon[((size_t(p) * K + p) * K + q) * K + q];
      jk[size_t(K) * K + size_t(p) * K + q] = canon[((size_t(p) * K + q) * K + q) * K + p];
    }
  if ((st = upload(&inst->d_jk, jk)) != NQS_OK) return st;
  std::vector<double> s3(size_t(2) * K * K * K);
  for (int a = 0; a < K; ++a)
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j) {
        const size_t o = ((size_t(a) * K + i) * K + j) * 2;
        s3[o] = canon[((size_t(a) * K + i) * K + j) * K + j];
        s3[o + 1] = canon[((size_t(a) * K + j) * K + j) * K + i];
      }
  if ((st = upload(&inst->d_s3, s3)) != NQS_OK) return st;
  HamDev& H = inst->H;
  H.h = inst->d_h; H.eri = inst->d_eri; H.jk = inst->d_jk; H.s3 = inst->d_s3; H.ecore = e_core;
  H.K = K; H.na = n_alpha; H.nb = n_beta; H.va = K - n_alpha; H.vb = K - n_beta;
  const int64_t nsa = int64_t(n_alpha) * H.va, nsb = int64_t(n_beta) * H.vb;
  const int64_t daa = choose2(n_alpha) * choose2(H.va), dbb = choose2(n_beta) * choose2(H.vb);
  const int64_t dab = nsa * nsb;
  const int64_t total = nsa + nsb + daa + dbb + dab;
  if (total >= (int64_t(1) << 31)) return fail(NQS_EUNSUPPORTED, "too many connected determinants");
  H.off_sb = uint32_t(nsa);
  H.off_daa = uint32_t(nsa + nsb);
  H.off_dbb = uint32_t(nsa + nsb + daa);
  H.off_dab = uint32_t(nsa + nsb + daa + dbb);
  H.n_conn = uint32_t(total);
  H.npa_v = uint32_t(choose2(H.va));
  H.npb_v = uint32_t(choose2(H.vb));
  H.nsb = uint32_t(nsb);
  H.mg_va = magic(H.va); H.mg_vb = magic(H.vb);
  H.mg_npa_v = magic(H.npa_v); H.mg_npb_v = magic(H.npb_v); H.mg_nsb = magic(H.nsb);
  // exactness of (x * ceil(2^32/d)) >> 32 needs x * d < 2^32 for every use
  const uint64_t lim = uint64_t(1) << 32;
  const uint64_t checks[][2] = {{uint64_t(nsa), uint64_t(H.va)}, {uint64_t(nsb), uint64_t(H.vb)},
                                {uint64_t(daa), uint64_t(H.npa_v)}, {uint64_t(dbb), uint64_t(H.npb_v)},
                                {uint64_t(dab), uint64_t(nsb)}};
  for (auto& c : checks)
    if (c[0] * c[1] >= lim) return fail(NQS_EUNSUPPORTED, "rank arithmetic would overflow");
  *out = inst.release();
  return NQS_OK;
}

nqs_status nqs_instance_destroy(nqs_instance* inst) {
  if (!inst) return NQS_OK;
  DeviceGuard g(inst->device);
  delete inst;
  return NQS_OK;
}

int64_t nqs_instance_n_conn(const nqs_instance* inst) { return inst ? int64_t(inst->H.n_conn) : -1; }

nqs_status nqs_ansatz_create(nqs_ctx* ctx, int K, int n_alpha, int n_beta, int chi,
                             const int32_t* parent_ptr, const int32_t* parent_idx, int n_hidden,
                             int32_t variant, nqs_ansatz** out) {
  if (!ctx || !parent_ptr || !out) return fail(NQS_EINVAL, "NULL argument");
  const int32_t correlator = variant & 0xF;
  if ((correlator != NQS_CORR_COS_RBM && correlator != NQS_CORR_ISING_RBM) ||
      (variant & ~(0xF | NQS_ANSATZ_TENSOR | NQS_ANSATZ_COMPLEX)))
    return fail(NQS_EINVAL, "unknown ansatz variant %d", variant);
  const bool cplx = (variant & NQS_ANSATZ_COMPLEX) != 0;
  if (cplx && (variant & NQS_ANSATZ_TENSOR))
    return fail(NQS_EINVAL, "complex parameters are not combined with the tensor-RNN term");
  if (K < 1 || K > 64) return fail(NQS_EINVAL, "K=%d outside [1,64]", K);
  if (chi < 1 || chi > 64) return fail(NQS_EUNSUPPORTED, "chi=%d outside [1,64]", chi);
  if (cplx && chi > 32) return fail(NQS_EUNSUPPORTED, "complex chi=%d above 32", chi);
  const int chi_c = chi;
  if (cplx) chi = 2 * chi;   // the realified state
  if (n_alpha < 0 || n_alpha > K || n_beta < 0 || n_beta > K) return fail(NQS_EINVAL, "bad electron counts");
  if (n_hidden < 0) return fail(NQS_EINVAL, "n_hidden < 0");
  if (parent_ptr[0] != 0) return fail(NQS_EINVAL, "parent_ptr[0] != 0");
  std::unique_ptr<nqs_ansatz> a(new nqs_ansatz());
  a->ctx = ctx;
  a->device = ctx->device;
  a->K = K; a->na = n_alpha; a->nb = n_beta; a->chi = chi; a->nh = n_hidden;
  a->ising = n_hidden > 0 && correlator == NQS_CORR_ISING_RBM;
  a->tensor = (variant & NQS_ANSATZ_TENSOR) != 0;
  a->cplx = cplx;
  a->chi_c = chi_c;
  a->chip = ((chi + 15) / 16) * 16;
  a->pptr.assign(parent_ptr, parent_ptr + K + 1);
  int maxoff = 0;
  for (int i = 0; i < K; ++i) {
    if (a->pptr[i + 1] < a->pptr[i]) return fail(NQS_EINVAL, "parent_ptr not monotone at %d", i);
    if (a->pptr[i + 1] - a->pptr[i] > 16) return fail(NQS_EUNSUPPORTED, "in-degree above 16 at %d", i);
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) {
      if (!parent_idx) return fail(NQS_EINVAL, "parent_idx is NULL");
      const int j = parent_idx[e];
      if (j < 0 || j >= i) return fail(NQS_EINVAL, "parent %d of site %d does not precede it", j, i);
      if (e > a->pptr[i] && parent_idx[e - 1] >= j) return fail(NQS_EINVAL, "parents of %d not ascending", i);
      maxoff = std::max(maxoff, i - j);
    }
  }
  a->pidx.assign(parent_idx ? parent_idx : parent_ptr, parent_idx ? parent_idx + a->pptr[K] : parent_ptr);
  a->W = maxoff + 1;
  int64_t o = 0;
  a->offM.resize(a->pptr[K]);
  a->offV.resize(K); a->offEta.resize(K); a->offW.resize(K); a->offC.resize(K);
  for (int i = 0; i < K; ++i) {
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) { a->offM[e] = o; o += int64_t(4) * chi * chi; }
    a->offV[i] = o; o += 4 * chi;
    a->offEta[i] = o; o += chi;
    a->offW[i] = o; o += chi;
    a->offC[i] = o; o += 1;
  }
  a->offB = o; o += n_hidden;
  a->offWc = o; o += int64_t(n_hidden) * 2 * K;
  a->offW2 = o;
  if (a->ising) o += int64_t(n_hidden) * 4 * K * K;
  if (cplx) {
    // the realified vector's w2 and c2 (Im z = w2^T x + c2), then the
    // caller's complex layout
    a->offW2x.resize(K);
    a->offC2x.resize(K);
    for (int i = 0; i < K; ++i) {
      a->offW2x[i] = o; o += chi;
      a->offC2x[i] = o; o += 1;
    }
    a->nr_params = o;
    int64_t q = 0;
    a->cx_offM.resize(a->pptr[K]);
    a->cx_offV.resize(K); a->cx_offEta.resize(K); a->cx_offW.resize(K); a->cx_offC.resize(K);
    for (int i = 0; i < K; ++i) {
      for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) { a->cx_offM[e] = q; q += int64_t(8) * chi_c * chi_c; }
      a->cx_offV[i] = q; q += 8 * chi_c;
      a->cx_offEta[i] = q; q += chi_c;
      a->cx_offW[i] = q; q += 2 * chi_c;
      a->cx_offC[i] = q; q += 2;
    }
    a->cx_offB = q;
    q += int64_t(n_hidden) * (2 * K + 1) + (a->ising ? int64_t(n_hidden) * 4 * K * K : 0);
    o = q;   // n_params below: the caller's (complex) layout
  }
  // BDG-TensorRNN block, last: per site with d >= 2 parents the factor
  // matrices K^(0..d) (chi x chi' each) and the cores U^s (chi'^(d+1) each)
  a->tq.assign(K, 0);
  a->offTK.assign(K, 0);
  a->offTU.assign(K, 0);
  for (int i = 0; i < K && a->tensor; ++i) {
    const int d = a->pptr[i + 1] - a->pptr[i];
    if (d < 2) continue;
    if (d > 3) return fail(NQS_EUNSUPPORTED, "tensor term at site %d with %d parents (at most 3)", i, d);
    int q = 1;
    while (true) {
      int64_t pw = 1;
      for (int k = 0; k <= d; ++k) pw *= q;
      if (pw >= int64_t(chi) * chi) break;
      ++q;
    }
    int64_t qd = 1;
    for (int k = 0; k <= d; ++k) qd *= q;
    a->tq[i] = q;
    a->offTK[i] = o; o += int64_t(d + 1) * chi * q;
    a->offTU[i] = o; o += 4 * qd;
  }
  a->n_params = o;
  if (!cplx) a->nr_params = o;
  DeviceGuard g(ctx->device);
  nqs_status st;
  std::vector<int> pp(a->pptr.begin(), a->pptr.end()), pi(a->pidx.begin(), a->pidx.end());
  if ((st = upload(&a->d_pptr, pp)) != NQS_OK) return st;
  if ((st = upload(&a->d_pidx, pi)) != NQS_OK) return st;
  std::vector<int> slot(pi.size());
  for (size_t e = 0; e < pi.size(); ++e) slot[e] = pi[e] % a->W;
  if ((st = upload(&a->d_slot, slot)) != NQS_OK) return st;
  // LDS ring of the forward kernels: site i's carried state goes to slot
  // wsl[i], one whose previous state no site after i reads (its last reader
  // may be site i itself: a site reads its parents before it writes); the
  // ring needs as many slots as states are live at once, which can be fewer
  // than the largest parent offset.  live[i], i = 0..K: bit s set for each
  // state s < i that a site >= i reads (a row resumed at i loads exactly
  // these).  Rows resume at K too (a sample's own row, and a row with fewer
  // changed sites than its resume level): live[K] = 0.
  std::vector<int> lastu(K), wsl(K), holder;
  std::vector<uint64_t> live(K + 1, 0);
  for (int s = 0; s < K; ++s) lastu[s] = s;
  for (int i = 0; i < K; ++i)
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) lastu[pi[e]] = std::max(lastu[pi[e]], i);
  for (int i = 0; i < K; ++i) {
    size_t k = 0;
    while (k < holder.size() && lastu[holder[k]] > i) ++k;
    if (k == holder.size()) holder.push_back(i); else holder[k] = i;
    wsl[i] = int(k);
  }
  a->ring = int(holder.size());
  for (int i = 0; i < K; ++i)
    for (int s2 = 0; s2 < i; ++s2)
      if (lastu[s2] >= i) live[i] |= 1ull << s2;
  if ((st = upload(&a->d_wsl, wsl)) != NQS_OK) return st;
  if ((st = upload(&a->d_live, live)) != NQS_OK) return st;
  // forward edges: a parentless site gets one zero edge, marked by the slot
  // index a->ring (no such slot: the kernels take a zero operand)
  std::vector<int> fptr(1, 0), fslot;
  for (int i = 0; i < K; ++i) {
    if (a->pptr[i + 1] == a->pptr[i]) fslot.push_back(a->ring);
    for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) fslot.push_back(wsl[pi[e]]);
    fptr.push_back(int(fslot.size()));
  }
  a->d1 = true;
  for (int i = 0; i < K; ++i) a->d1 = a->d1 && fptr[i + 1] - fptr[i] == 1;
  if ((st = upload(&a->d_fptr, fptr)) != NQS_OK) return st;
  if ((st = upload(&a->d_fslot, fslot)) != NQS_OK) return st;
  if ((st = upload(&a->d_offM, a->offM)) != NQS_OK) return st;
  if ((st = upload(&a->d_offV, a->offV)) != NQS_OK) return st;
  if ((st = upload(&a->d_offEta, a->offEta)) != NQS_OK) return st;
  if (cplx) {
    std::vector<int64_t> tab;
    for (auto* v : {&a->offW, &a->offC, &a->offW2x, &a->offC2x, &a->cx_offV, &a->cx_offEta, &a->cx_offW,
                    &a->cx_offC, &a->cx_offM})
      tab.insert(tab.end(), v->begin(), v->end());
    if ((st = upload(&a->d_cx, tab)) != NQS_OK) return st;
  }
  if (a->tensor) {
    // kernel layout offsets (elements; every block starts on a multiple of 16)
    const int cp = a->chip;
    auto r16 = [](int64_t x) { return (x + 15) / 16 * 16; };
    int qmax = 0;
    for (int i = 0; i < K; ++i) qmax = std::max(qmax, a->tq[i]);
    const int qp = qmax <= 8 ? 8 : 16;
    a->tn_qp = qp;
    std::vector<int> edge(size_t(a->pptr[K]) * 2), site(size_t(K) * 8, 0);
    int64_t q = 0;
    for (int i = 0; i < K; ++i) {
      for (int e = a->pptr[i]; e < a->pptr[i + 1]; ++e) {
        edge[2 * e] = int(q);
        edge[2 * e + 1] = a->pidx[e] % a->W;
        q += int64_t(4) * cp * cp;
      }
      int* st8 = site.data() + 8 * i;
      st8[0] = int(q); q += 4 * cp;
      st8[1] = int(q); q += cp;
      st8[2] = int(q); q += cp;
      st8[3] = int(q); q += 16;
      const int tq = a->tq[i], d = a->pptr[i + 1] - a->pptr[i];
      st8[4] = tq;
      if (tq) {
        int64_t qd = 1;
        for (int k = 0; k <= d; ++k) qd *= tq;
        st8[5] = int(q); q += r16(int64_t(tq) * cp);
        st8[6] = int(q); q += r16(int64_t(d) * cp * qp);
        st8[7] = int(q); q += r16(4 * (qd / tq) * qp);   // U^s rows padded to qp in the last index
      }
    }
    if (q >= (int64_t(1) << 31)) return fail(NQS_EUNSUPPORTED, "tensor-RNN parameter layout too large");
    a->tn_size = q;
    const int rw = (chi + 3) / 4 * 4;
    a->tn_f64_ok = tn_lds_bytes(a->W, rw, 0) <= 64 * 1024;
    if (tn_lds_bytes(a->W, rw, 1) > 64 * 1024)
      return fail(NQS_EUNSUPPORTED, "tensor-RNN ring of %d x %d states does not fit the LDS", a->W, rw);
    if ((st = upload(&a->d_tn_edge, edge)) != NQS_OK) return st;
    if ((st = upload(&a->d_tn_site, site)) != NQS_OK) return st;
    a->tn_edge_host = edge;
    a->tn_site_host = site;
    // the MFMA forward carries the tensor term when chip <= 32 and chi' <= 8
    a->tn_mfma = a->chip <= 32 && qmax <= 8;
    if (a->tn_mfma) {
      const int KSq = a->chip / 4, TPCq = a->chip / 16;
      std::vector<int> ts(size_t(K) * 4, 0);
      int64_t cur = 0;
      for (int i = 0; i < K; ++i) {
        const int tq = a->tq[i], d = a->pptr[i + 1] - a->pptr[i];
        if (!tq) continue;
        int nlead = 1;
        for (int k = 0; k < d - 1; ++k) nlead *= tq;
        ts[4 * i] = tq;
        ts[4 * i + 1] = int(cur); cur += int64_t(d) * KSq * 64;
        ts[4 * i + 2] = int(cur); cur += int64_t(nlead) * 2 * 2 * 64;
        ts[4 * i + 3] = int(cur); cur += int64_t(4) * TPCq * 4 * 64;
      }
      if (cur >= (int64_t(1) << 31)) return fail(NQS_EUNSUPPORTED, "tensor-RNN operand stream too large");
      a->ta_size = cur;
      a->tsite_host = ts;
      if ((st = upload(&a->d_tsite, ts)) != NQS_OK) return st;
    }
  }
  *out = a.release();
  return NQS_OK;
}

nqs_status nqs_ansatz_destroy(nqs_ansatz* ans) {
  if (!ans) return NQS_OK;
  DeviceGuard g(ans->device);
  delete ans;
  return NQS_OK;
}

int64_t nqs_ansatz_n_params(const nqs_ansatz* ans) { return ans ? ans->n_params : -1; }

nqs_status nqs_ansatz_bind_params(nqs_ansatz* ans, const double* params, hipStream_t stream) {
  if (!ans || !params) return fail(NQS_EINVAL, "NULL argument");
  DeviceGuard g(ans->ctx->device);
  std::vector<double> prm(ans->n_params);
  HIPCHK(hipMemcpyAsync(prm.data(), params, prm.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (ans->cplx) {
    // the realified vector: per edge and state M_r = [[Re M, -Im M], [Im M, Re M]],
    // v_r = [Re v; Im v], eta_r = [eta; eta], w_r = [Re w; -Im w], c_r = Re c,
    // w2 = [Im w; Re w], c2 = Im c; the correlator block as it is
    const int n = ans->chi_c, n2 = 2 * n;
    for (int i = 0; i < ans->K; ++i)
      for (int u = 0; u < n; ++u)
        if (!(prm[ans->cx_offEta[i] + u] >= 0.0))
          return fail(NQS_EINVAL, "eta[%d][%d] = %g is negative or NaN", i, u, prm[ans->cx_offEta[i] + u]);
    std::vector<double> r(ans->nr_params, 0.0);
    for (int i = 0; i < ans->K; ++i) {
      for (int e = ans->pptr[i]; e < ans->pptr[i + 1]; ++e)
        for (int s = 0; s < 4; ++s)
          for (int u = 0; u < n; ++u)
            for (int k = 0; k < n; ++k) {
              const double* z = prm.data() + ans->cx_offM[e] + 2 * ((int64_t(s) * n + u) * n + k);
              double* B = r.data() + ans->offM[e] + int64_t(s) * n2 * n2;
              B[int64_t(u) * n2 + k] = z[0];
              B[int64_t(u) * n2 + k + n] = -z[1];
              B[int64_t(u + n) * n2 + k] = z[1];
              B[int64_t(u + n) * n2 + k + n] = z[0];
            }
      for (int s = 0; s < 4; ++s)
        for (int u = 0; u < n; ++u) {
          r[ans->offV[i] + s * n2 + u] = prm[ans->cx_offV[i] + 2 * (s * n + u)];
          r[ans->offV[i] + s * n2 + n + u] = prm[ans->cx_offV[i] + 2 * (s * n + u) + 1];
        }
      for (int u = 0; u < n; ++u) {
        const double et = prm[ans->cx_offEta[i] + u];
        const double wr = prm[ans->cx_offW[i] + 2 * u], wi = prm[ans->cx_offW[i] + 2 * u + 1];
        r[ans->offEta[i] + u] = et;
        r[ans->offEta[i] + n + u] = et;
        r[ans->offW[i] + u] = wr;
        r[ans->offW[i] + n + u] = -wi;
        r[ans->offW2x[i] + u] = wi;
        r[ans->offW2x[i] + n + u] = wr;
      }
      r[ans->offC[i]] = prm[ans->cx_offC[i]];
      r[ans->offC2x[i]] = prm[ans->cx_offC[i] + 1];
    }
    std::copy(prm.begin() + ans->cx_offB, prm.end(), r.begin() + ans->offB);
    prm.swap(r);
  }
  for (int i = 0; i < ans->K; ++i)
    for (int u = 0; u < ans->chi; ++u)
      if (!(prm[ans->offEta[i] + u] >= 0.0))
        return fail(NQS_EINVAL, "eta[%d][%d] = %g is negative or NaN", i, u, prm[ans->offEta[i] + u]);
  // the old layouts are replaced from here on: until every one is rebuilt the
  // ansatz counts as unbound, so a failure below leaves calls refusing it
  // instead of launching on half-built layouts
  ans->bound = false;
  nqs_status st;
  if ((st = build_layout<double>(ans, prm, ans->L64, false)) != NQS_OK) return st;
  if ((st = build_layout<float>(ans, prm, ans->L32, false)) != NQS_OK) return st;
  bool all_pos = true;
  for (int i = 0; i < ans->K; ++i)
    for (int u = 0; u < ans->chi; ++u) all_pos = all_pos && prm[ans->offEta[i] + u] > 0.0;
  ans->has_fold = false;
  ans->F64.free_all();
  ans->F32.free_all();
  if (all_pos) {
    if ((st = build_layout<double>(ans, prm, ans->F64, true)) != NQS_OK) return st;
    if ((st = build_layout<float>(ans, prm, ans->F32, true)) != NQS_OK) return st;
    ans->has_fold = true;
  }
  if (!ans->cplx && (st = build_bf16(ans, prm, ans->has_fold)) != NQS_OK) return st;
  if (ans->tensor && (st = build_tn(ans, prm)) != NQS_OK) return st;
  if (ans->d_cb) { (void)hipFree(ans->d_cb); ans->d_cb = nullptr; }
  if (ans->d_cW) { (void)hipFree(ans->d_cW); ans->d_cW = nullptr; }
  if (ans->d_cW1t) { (void)hipFree(ans->d_cW1t); ans->d_cW1t = nullptr; }
  if (ans->d_cS) { (void)hipFree(ans->d_cS); ans->d_cS = nullptr; }
  if (ans->d_cS32) { (void)hipFree(ans->d_cS32); ans->d_cS32 = nullptr; }
  if (ans->nh) {
    const int nh = ans->nh, nv = 2 * ans->K;
    std::vector<double> b(prm.begin() + ans->offB, prm.begin() + ans->offB + nh);
    std::vector<double> W(prm.begin() + ans->offWc, prm.begin() + ans->offWc + int64_t(nh) * nv);
    if ((st = upload(&ans->d_cb, b)) != NQS_OK) return st;
    if ((st = upload(&ans->d_cW, W)) != NQS_OK) return st;
    // hidden unit fastest: W^T [P][k] (both correlators' row kernels read it)
    std::vector<double> Wt(size_t(nv) * nh);
    for (int k = 0; k < nh; ++k)
      for (int P = 0; P < nv; ++P) Wt[size_t(P) * nh + k] = W[size_t(k) * nv + P];
    if ((st = upload(&ans->d_cW1t, Wt)) != NQS_OK) return st;
    if (ans->ising) {
      // S [P][Q][k] = (W2[k][P][Q] + W2[k][Q][P]) / 2
      std::vector<double> Sy(size_t(nv) * nv * nh);
      const double* W2 = prm.data() + ans->offW2;
      for (int k = 0; k < nh; ++k)
        for (int P = 0; P < nv; ++P)
          for (int Q = 0; Q < nv; ++Q)
            Sy[(size_t(P) * nv + Q) * nh + k] =
                0.5 * (W2[(size_t(k) * nv + P) * nv + Q] + W2[(size_t(k) * nv + Q) * nv + P]);
      if ((st = upload(&ans->d_cS, Sy)) != NQS_OK) return st;
      std::vector<float> Sy32(Sy.begin(), Sy.end());
      if ((st = upload(&ans->d_cS32, Sy32)) != NQS_OK) return st;
    }
  }
  ans->bound = true;
  return NQS_OK;
}

}  // extern "C"

namespace {

nqs_status check_samples(nqs_ctx* ctx, const uint64_t* samples, int64_t N, int K, int na, int nb,
                         hipStream_t st, Arena* arena = nullptr) {
  if (N == 0) return NQS_OK;
  Scratch S(ctx, st, arena);
  int* bad = S.get<int>(1);
  if (!bad) return fail(NQS_ENOMEM, "workspace allocation failed");
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
  HIPCHK(launch_validate(samples, N, K, na, nb, bad, st));
  int hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hb) return fail(NQS_EINVAL, "a sample lies outside the (%d,%d) sector of K=%d", na, nb, K);
  return NQS_OK;
}

// Device state of resumed amplitude rows (FP64/FP32): the samples' carried
// states and log-product states, and the order of the current pass's rows.
struct Resume {
  void* hs = nullptr;       // [K][N][chip] T (BF16: uint16)
  uint16_t* hs_lo = nullptr;  // split BF16: the lo parts of hs
  int32_t* he = nullptr;    // BF16: [K][N] state exponents
  void* pm = nullptr;       // [K+1][N] T (BF16: float)
  int32_t* pe = nullptr;    // [K+1][N]
  int8_t* pg = nullptr;     // [K+1][N]
  void* pz = nullptr;       // complex parameters: [K+1][N][2] T
  int64_t ns = 0;
  int32_t* perm = nullptr;  // [rows of a pass] row of each sorted position
  uint8_t* t0 = nullptr;    // [rows of a pass] sorted first changed sites
  int32_t* cnt = nullptr;   // [order blocks][K+1]
  int64_t* tot = nullptr;   // [K+1]
  const int32_t* owner = nullptr;
  // one node level (FP64/FP32): node storage and the rows' nodes
  void* nhs = nullptr;      // [entries][chip] T
  void* nlp = nullptr;      // [entries] LogProd<T> (16 bytes)
  void* npz = nullptr;      // complex parameters: [entries][2] T
  const NodeRec* nrec = nullptr;     // [nodes]
  const int32_t* unode = nullptr;
};

template <typename T>
PsiStates<T> states(const Resume& r) {
  PsiStates<T> X;
  X.hs = static_cast<T*>(r.hs);
  X.pm = static_cast<T*>(r.pm);
  X.pe = r.pe;
  X.pg = r.pg;
  X.pz = static_cast<T*>(r.pz);
  X.ns = r.ns;
  X.perm = r.perm;
  X.t0 = r.t0;
  X.owner = r.owner;
  X.nhs = static_cast<T*>(r.nhs);
  X.nlp = static_cast<LogProd<T>*>(r.nlp);
  X.npz = static_cast<T*>(r.npz);
  X.nrec = r.nrec;
  X.unode = r.unode;
  return X;
}

B16States states_b16(const Resume& r) {
  B16States X;
  X.hs = static_cast<uint16_t*>(r.hs);
  X.hs_lo = r.hs_lo;
  X.he = r.he;
  X.pm = static_cast<float*>(r.pm);
  X.pe = r.pe;
  X.pg = r.pg;
  X.ns = r.ns;
  X.perm = r.perm;
  X.t0 = r.t0;
  X.owner = r.owner;
  return X;
}

// BF16 operands on MFMA, plain or split (hi + lo parts)
bool is_bf16(int precision) { return precision == NQS_BF16 || precision == NQS_BF16X3; }

// bytes per element of the resume state arrays: carried state (BF16 forms: the
// hi part), log-product mantissa
size_t state_bytes(int precision) { return precision == NQS_F64 ? 8 : (precision == NQS_F32 ? 4 : 2); }
size_t mantissa_bytes(int precision) { return precision == NQS_F64 ? 8 : 4; }

// amplitudes of R rows into (lphi, sphi).  mode PSI_STORE (samples, with rs)
// or PSI_SEED (rows of a pass, with rs and its order).
// phs: complex parameters, the phase of each row
nqs_status run_amplitudes(const nqs_ansatz* a, int precision, const uint64_t* m, int64_t R, double* lphi,
                          int8_t* sphi, hipStream_t st, const Resume* rs = nullptr, int mode = PSI_PLAIN,
                          double* phs = nullptr) {
  if (mode != PSI_PLAIN && !rs) return fail(NQS_EINVAL, "resume state missing");
  if (a->cplx) {
    if (!phs) return fail(NQS_EINVAL, "complex amplitudes need their phases");
    if (precision == NQS_F64) {
      HIPCHK(launch_psi_f64(a->params(a->fwd64()), m, R, lphi, sphi, st,
                            rs ? states<double>(*rs) : PsiStates<double>(), mode, phs));
    } else if (precision == NQS_F32) {
      HIPCHK(launch_psi_f32(a->params(a->fwd32()), m, R, lphi, sphi, st,
                            rs ? states<float>(*rs) : PsiStates<float>(), mode, phs));
    } else {
      return fail(NQS_EUNSUPPORTED, "complex amplitudes run in FP64 or FP32");
    }
    return NQS_OK;
  }
  if (a->tensor && is_bf16(precision)) return fail(NQS_EUNSUPPORTED, "the tensor-RNN runs in FP64 or FP32");
  if (a->tensor && !a->tn_mfma) {
    // the thread-per-row kernel (chi' > 8 or chi > 32)
    if (mode != PSI_PLAIN) return fail(NQS_EINVAL, "tensor-RNN rows are evaluated from site 0");
    if (precision == NQS_F64) {
      if (!a->tn_f64_ok) return fail(NQS_EUNSUPPORTED, "FP64 tensor-RNN ring does not fit the LDS");
      HIPCHK(launch_psi_tn_f64(a->tn<double>(a->tn64), m, R, lphi, sphi, st));
    } else if (precision == NQS_F32) {
      HIPCHK(launch_psi_tn_f32(a->tn<float>(a->tn32), m, R, lphi, sphi, st));
    } else {
      return fail(NQS_EUNSUPPORTED, "the tensor-RNN runs in FP64 or FP32");
    }
    return NQS_OK;
  }
  if (precision == NQS_F64) {
    HIPCHK(launch_psi_f64(a->params(a->fwd64()), m, R, lphi, sphi, st,
                          rs ? states<double>(*rs) : PsiStates<double>(), mode));
  } else if (precision == NQS_F32) {
    HIPCHK(launch_psi_f32(a->params(a->fwd32()), m, R, lphi, sphi, st,
                          rs ? states<float>(*rs) : PsiStates<float>(), mode));
  } else if (is_bf16(precision)) {
    const PsiLayout<float>& L = a->fwd32();
    B16Params P{};
    P.K = a->K; P.chi = a->chi; P.chip = a->chip; P.na = a->na; P.nb = a->nb; P.W = a->ring;
    P.pptr = a->d_fptr; P.slot = a->d_fslot; P.wsl = a->d_wsl; P.live = a->d_live;
    P.A = a->bfA; P.Alo = a->bfAlo;
    P.v = L.v; P.eta = L.eta; P.w = L.w; P.c = L.c; P.folded = L.folded; P.d1 = a->d1;
    hipError_t e = launch_psi_bf16(P, m, R, lphi, sphi, st, rs ? states_b16(*rs) : B16States(), mode,
                                   precision == NQS_BF16X3);
    if (e == hipErrorNotSupported) return fail(NQS_EUNSUPPORTED, "BF16 amplitude path not available");
    HIPCHK(e);
  } else {
    return fail(NQS_EINVAL, "unknown precision %d", precision);
  }
  return NQS_OK;
}

struct Pipeline {
  // per sample
  uint64_t *masks, *qpref, *segq, *Qn, *um;
  uint32_t* segd;
  int64_t *Dn, *Un, *rowptr;
  int32_t* urank;
  double *ucoef, *hdiag;
  EnumGeom G;
  int qshift;
  int64_t R;                        // total rows
  std::vector<int64_t> rowptr_host; // [N+1]
  // rows of the current pass
  Rows rows;
  int64_t rows_cap;
};

EnumGeom make_geom(int64_t n_conn, int64_t N) {
  EnumGeom G;
  G.nchunks = int((n_conn + 63) / 64);
  int64_t S = (32768 + N - 1) / std::max<int64_t>(N, 1);
  S = std::max<int64_t>(1, std::min<int64_t>(S, std::min<int64_t>(64, std::max(G.nchunks, 1))));
  G.S = int(S);
  G.cps = (std::max(G.nchunks, 1) + G.S - 1) / G.S;
  return G;
}

// node storage of a pass.  Measured per row on samples drawn from Phi^2 (chain
// K = 20, dense K = 20, lattice K = 18, NN+NNN chain K = 50), nodes keyed by
// the first two changes: 0.07-0.22 nodes, 0.95-3.3 log-product entries
// (about K / 15) and 0.37-0.87 carried-state slots read at the rows' own
// resume sites (about (W - 1) K / 100 with W - 1 parent offsets); keyed by
// the first change alone, 0.05-0.16 entries.  The capacities leave a quarter
// or more over these; samples beyond a capacity resume at c1.  The
// tensor-term kernels store every carried state (a slot per entry).
NodeCaps node_caps(int64_t pass_rows, int K, int W, bool pair, bool tn, double scale = 1.0) {
  const int64_t floor = int64_t(16) * K * (K + 1);
  NodeCaps c;
  if (tn) {
    c.entries = pair ? std::max<int64_t>(pass_rows / 2 * 3, floor) : std::max<int64_t>(pass_rows / 8, floor / 4);
    c.nodes = c.entries;
    c.own_slots = c.entries;
  } else {
    c.nodes = std::max<int64_t>(pass_rows / 3, floor);
    c.entries = std::max<int64_t>(pass_rows / 16 * (16 + K), floor);
    c.own_slots = std::min(c.entries, std::max<int64_t>(pass_rows / 100 * (35 + int64_t(W - 1) * K), floor));
  }
  if (scale < 1.0) {
    c.nodes = std::max<int64_t>(1, int64_t(double(c.nodes) * scale));
    c.entries = std::max<int64_t>(1, int64_t(double(c.entries) * scale));
    c.own_slots = std::max<int64_t>(1, int64_t(double(c.own_slots) * scale));
  }
  return c;
}

// carried-state slots to allocate: the rows' own reads plus the reserve for
// the wavefront starts (tensor-term kernels: one per entry)
int64_t node_slots(const NodeCaps& c, int K, bool tn) { return tn ? c.entries : c.own_slots + slot_reserve(K); }

// nodes keyed by the first two changes where the pair table fits the LDS
// (tensor-term kernels: up to K = 30, as they store every carried state)
bool pair_nodes(int K, bool tn) { return node_pairs(K) && (!tn || K <= 30); }

int64_t max_samples_per_pass(const std::vector<std::pair<int64_t, int64_t>>& passes) {
  int64_t m = 1;
  for (auto& p : passes) m = std::max(m, p.second - p.first);
  return m;
}

// largest number of rows any pass can hold: a pass takes whole samples, so it
// holds at most max(max_rows_per_pass, rows of the largest sample)
int64_t pass_rows_bound(const HamDev& H, const nqs_eloc_opts& o, int64_t total_rows) {
  if (o.max_rows_per_pass <= 0) return total_rows;
  const int64_t one = 1 + int64_t(H.n_conn) + std::max(o.n_eps, 0);
  return std::max<int64_t>(o.max_rows_per_pass, one);
}

// enumerate + screen + draw + row pointer (host copy); no rows yet
nqs_status count_and_draw(Scratch& S, const nqs_instance* inst, const uint64_t* samples, int64_t N,
                          const nqs_eloc_opts& o, Pipeline& P, hipStream_t st, hipEvent_t* ev) {
  const HamDev& H = inst->H;
  P.G = make_geom(H.n_conn, N);
  int e2 = 0;
  if (o.eps > 0) std::frexp(o.eps, &e2);
  P.qshift = 40 - e2;
  const int ne = std::max(o.n_eps, 0);
  const size_t NC = size_t(N) * P.G.nchunks;
  P.masks = S.get<uint64_t>(NC);
  P.qpref = S.get<uint64_t>(NC);
  P.segq = S.get<uint64_t>(size_t(N) * P.G.S);
  P.segd = S.get<uint32_t>(size_t(N) * P.G.S);
  P.Qn = S.get<uint64_t>(N);
  P.Dn = S.get<int64_t>(N);
  P.Un = S.get<int64_t>(N);
  P.rowptr = S.get<int64_t>(N + 1);
  P.urank = S.get<int32_t>(size_t(N) * std::max(ne, 1));
  P.ucoef = S.get<double>(size_t(N) * std::max(ne, 1));
  P.um = S.get<uint64_t>(size_t(N) * std::max(ne, 1) * 2);
  P.hdiag = S.get<double>(N);
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  if (ev) HIPCHK(hipEventRecord(ev[0], st));
  HIPCHK(launch_enum_count(H, P.G, samples, N, o.eps, P.qshift, P.masks, P.qpref, P.segq, P.segd, st));
  HIPCHK(launch_sample_scan(P.G, N, P.segq, P.segd, P.Qn, P.Dn, st));
  if (ev) HIPCHK(hipEventRecord(ev[1], st));
  if (ne > 0) {
    DrawKeys k;
    k.key0 = uint32_t(o.seed); k.key1 = uint32_t(o.seed >> 32);
    k.ctr2 = uint32_t(o.stream_id); k.ctr3 = uint32_t(o.stream_id >> 32);
    k.sample_base = uint32_t(o.sample_base);
    HIPCHK(launch_draw(H, P.G, samples, N, o.eps, P.qshift, ne, k, P.qpref, P.segq, P.Qn, P.urank, P.ucoef,
                       P.um, P.Un, st));
  } else {
    HIPCHK(hipMemsetAsync(P.Un, 0, sizeof(int64_t) * N, st));
  }
  HIPCHK(launch_row_counts(N, P.Dn, P.Un, P.rowptr, st));
  HIPCHK(launch_diag(H, samples, N, P.hdiag, st));
  if (ev) HIPCHK(hipEventRecord(ev[2], st));
  P.rowptr_host.resize(N + 1);
  HIPCHK(hipMemcpyAsync(P.rowptr_host.data(), P.rowptr, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  P.R = P.rowptr_host[N];
  return NQS_OK;
}

// rank: only for inspection (nqs_rows); the local energy does not need it
nqs_status alloc_rows(Scratch& S, Pipeline& P, int64_t cap, bool with_rank) {
  P.rows_cap = cap;
  P.rows.m = S.get<uint64_t>(size_t(cap) * 2);
  P.rows.coef = S.get<double>(cap);
  P.rows.owner = S.get<int32_t>(cap);
  P.rows.rank = with_rank ? S.get<int64_t>(cap) : nullptr;
  if (S.oom) return fail(NQS_ENOMEM, "row workspace allocation failed (%lld rows)", (long long)cap);
  return NQS_OK;
}

nqs_status fill_range(const nqs_instance* inst, const uint64_t* samples, int64_t n0, int64_t n1,
                      const nqs_eloc_opts& o, Pipeline& P, hipStream_t st) {
  HIPCHK(launch_fill(inst->H, P.G, samples, n0, n1, P.masks, P.segd, P.rowptr, P.rowptr_host[n0], P.Dn, P.Un,
                     P.urank, P.ucoef, P.um, std::max(o.n_eps, 1), P.rows, st));
  return NQS_OK;
}

// greedy split of [0, N) into sample ranges whose rows fit `cap`
std::vector<std::pair<int64_t, int64_t>> plan_passes(const std::vector<int64_t>& rp, int64_t cap) {
  std::vector<std::pair<int64_t, int64_t>> out;
  const int64_t N = int64_t(rp.size()) - 1;
  int64_t n0 = 0;
  while (n0 < N) {
    int64_t n1 = n0 + 1;
    while (n1 < N && rp[n1 + 1] - rp[n0] <= cap) ++n1;
    out.emplace_back(n0, n1);
    n0 = n1;
  }
  return out;
}

nqs_status check_opts(const nqs_eloc_opts* o) {
  if (!o) return fail(NQS_EINVAL, "opts is NULL");
  if (!(o->eps >= 0.0) || std::isinf(o->eps)) return fail(NQS_EINVAL, "eps must be finite and >= 0");
  if (o->n_eps < 0) return fail(NQS_EINVAL, "n_eps < 0");
  if (o->n_eps > 1024) return fail(NQS_EUNSUPPORTED, "n_eps > 1024 per sample");
  if (o->precision < 0 || o->precision > 3) return fail(NQS_EINVAL, "unknown precision");
  if (o->max_rows_per_pass < 0) return fail(NQS_EINVAL, "max_rows_per_pass < 0");
  if (o->flags & ~NQS_ELOC_FULL_RECOMPUTE) return fail(NQS_EINVAL, "unknown flags 0x%x", unsigned(o->flags));
  return NQS_OK;
}

// rows resume from their samples' states
bool resumes(const nqs_eloc_opts& o) { return !(o.flags & NQS_ELOC_FULL_RECOMPUTE); }

// precision / ansatz combinations the amplitude kernels do not run: refused
// before a call queues any work
nqs_status check_supported(const nqs_ansatz* a, int precision) {
  if (is_bf16(precision) && a->cplx) return fail(NQS_EUNSUPPORTED, "complex amplitudes run in FP64 or FP32");
  if (is_bf16(precision) && a->tensor) return fail(NQS_EUNSUPPORTED, "the tensor-RNN runs in FP64 or FP32");
  if (a->tensor && !a->tn_mfma && precision == NQS_F64 && !a->tn_f64_ok)
    return fail(NQS_EUNSUPPORTED, "FP64 tensor-RNN ring does not fit the LDS");
  return NQS_OK;
}

}  // namespace

extern "C" {

nqs_status nqs_connected(nqs_ctx* ctx, const nqs_instance* inst, const uint64_t* samples, int64_t N,
                         uint64_t* m_out, double* h_out, double* hdiag_out, hipStream_t stream) {
  if (!ctx || !inst || (!samples && N > 0) || N < 0) return fail(NQS_EINVAL, "bad arguments");
  DeviceGuard g(ctx->device);
  nqs_status s = check_samples(ctx, samples, N, inst->K, inst->na, inst->nb, stream);
  if (s != NQS_OK) return s;
  if (m_out || h_out) HIPCHK(launch_connected(inst->H, samples, N, m_out, h_out, stream));
  if (hdiag_out) HIPCHK(launch_diag(inst->H, samples, N, hdiag_out, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return NQS_OK;
}

nqs_status nqs_logpsi_phase(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                            int32_t precision, double* logabs, double* phase, hipStream_t stream) {
  if (!ctx || !ans || (!samples && N > 0) || N < 0) return fail(NQS_EINVAL, "bad arguments");
  if (!ans->bound) return fail(NQS_EINVAL, "parameters not bound");
  DeviceGuard g(ctx->device);
  nqs_status s = check_samples(ctx, samples, N, ans->K, ans->na, ans->nb, stream);
  if (s != NQS_OK) return s;
  if (N == 0) return NQS_OK;
  Scratch S(ctx, stream);
  double* lphi = S.get<double>(N);
  int8_t* sphi = S.get<int8_t>(N);
  double* phs = ans->cplx ? S.get<double>(N) : nullptr;
  double* lf = ans->nh ? S.get<double>(N) : nullptr;
  int8_t* sf = ans->nh ? S.get<int8_t>(N) : nullptr;
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  if ((s = run_amplitudes(ans, precision, samples, N, lphi, sphi, stream, nullptr, PSI_PLAIN, phs)) != NQS_OK)
    return s;
  if (ans->nh) HIPCHK(launch_corr_direct(ans->corr(), samples, N, lf, sf, stream));
  HIPCHK(launch_gather_logpsi_phase(N, lphi, sphi, phs, lf, sf, logabs, phase, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return NQS_OK;
}

nqs_status nqs_logpsi(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                      int32_t precision, double* logabs, int8_t* sign, hipStream_t stream) {
  if (!ctx || !ans || (!samples && N > 0) || N < 0) return fail(NQS_EINVAL, "bad arguments");
  if (!ans->bound) return fail(NQS_EINVAL, "parameters not bound");
  if (ans->cplx) return fail(NQS_EINVAL, "complex parameters have a phase, not a sign: use nqs_logpsi_phase");
  DeviceGuard g(ctx->device);
  nqs_status s = check_samples(ctx, samples, N, ans->K, ans->na, ans->nb, stream);
  if (s != NQS_OK) return s;
  if (N == 0) return NQS_OK;
  Scratch S(ctx, stream);
  double* lphi = S.get<double>(N);
  int8_t* sphi = S.get<int8_t>(N);
  double* lf = ans->nh ? S.get<double>(N) : nullptr;
  int8_t* sf = ans->nh ? S.get<int8_t>(N) : nullptr;
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  if ((s = run_amplitudes(ans, precision, samples, N, lphi, sphi, stream)) != NQS_OK) return s;
  if (ans->nh) HIPCHK(launch_corr_direct(ans->corr(), samples, N, lf, sf, stream));
  HIPCHK(launch_gather_logpsi(N, lphi, sphi, lf, sf, logabs, sign, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return NQS_OK;
}

nqs_status nqs_logpsi_vjp(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                          const double* cot, int32_t precision, double* grad, hipStream_t stream) {
  return nqs_logpsi_vjp_phase(ctx, ans, samples, N, cot, nullptr, precision, grad, stream);
}

nqs_status nqs_logpsi_vjp_phase(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                                const double* cot, const double* cot_phase, int32_t precision, double* grad,
                                hipStream_t stream) {
  if (!ctx || !ans || (!samples && N > 0) || N < 0 || (!cot && N > 0) || !grad)
    return fail(NQS_EINVAL, "bad arguments");
  if (!ans->bound) return fail(NQS_EINVAL, "parameters not bound");
  if (precision != NQS_F64 && precision != NQS_F32)
    return fail(NQS_EUNSUPPORTED, "the adjoint runs in FP64 or FP32");
  if (ans->tensor && precision == NQS_F64 && !ans->tn_f64_ok)
    return fail(NQS_EUNSUPPORTED, "FP64 tensor-RNN ring does not fit the LDS");
  DeviceGuard g(ctx->device);
  nqs_status s = check_samples(ctx, samples, N, ans->K, ans->na, ans->nb, stream);
  if (s != NQS_OK) return s;
  if (N == 0) return NQS_OK;
  const int64_t Rpad = (N + 15) / 16 * 16;
  const int64_t per = std::max<int64_t>(64, (Rpad / 32 + 15) / 16 * 16);
  const int rows_per_split = int(per);
  const int nsplit = int((Rpad + per - 1) / per);
  // the adjoint accumulates over the kernels' (for complex parameters the
  // realified) packed vector
  const int64_t np = ans->nr_params;
  const bool phase = ans->cplx && cot_phase != nullptr;
  const size_t hsz = size_t(ans->K) * Rpad * ans->chip;
  const size_t esz = precision == NQS_F64 ? 8 : 4;
  Scratch S(ctx, stream);
  void* Hbuf = S.get<unsigned char>(hsz * esz);
  void* dcarry = S.get<unsigned char>(hsz * esz);
  void* Dc = S.get<unsigned char>(size_t(Rpad) * 4 * ans->chip * esz);
  void* Eeta = S.get<unsigned char>(size_t(Rpad) * ans->chip * esz);
  double* lphi = S.get<double>(N);
  int8_t* sphi = S.get<int8_t>(N);
  double* gpart = S.get<double>(size_t(nsplit) * np);
  double* cotp = S.get<double>(Rpad);
  double* cotq = phase ? S.get<double>(Rpad) : nullptr;
  void* ab = phase ? S.get<unsigned char>(size_t(Rpad) * 2 * esz) : nullptr;
  double* gr = ans->cplx ? S.get<double>(np) : nullptr;
  double* dth = ans->nh ? S.get<double>(size_t(N) * ans->nh) : nullptr;
  // tensor term: row scratch of the current site (t^s, projections, core, their cotangents)
  void* tnb = ans->tensor ? S.get<unsigned char>(size_t(Rpad) * (4 * ans->chip + 14 * 16) * esz) : nullptr;
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  std::vector<int> tdeg(ans->K);
  for (int i = 0; i < ans->K; ++i) tdeg[i] = ans->pptr[i + 1] - ans->pptr[i];
  auto tn_adj = [&](auto* base, const auto& P) {
    typedef typename std::remove_pointer<decltype(base)>::type T;
    TnAdj<T> A;
    A.P = P;
    A.tq_host = ans->tq.data();
    A.d_host = tdeg.data();
    A.offTK_host = ans->offTK.data();
    A.offTU_host = ans->offTU.data();
    A.TT = base;
    A.PJ = A.TT + size_t(Rpad) * 4 * ans->chip;
    A.QS = A.PJ + size_t(Rpad) * 3 * 16;
    A.DQ = A.QS + size_t(Rpad) * 4 * 16;
    A.DP = A.DQ + size_t(Rpad) * 4 * 16;
    return A;
  };
  HIPCHK(hipMemsetAsync(dcarry, 0, hsz * esz, stream));
  HIPCHK(hipMemsetAsync(gpart, 0, sizeof(double) * nsplit * np, stream));
  HIPCHK(hipMemsetAsync(cotp, 0, sizeof(double) * Rpad, stream));
  HIPCHK(hipMemcpyAsync(cotp, cot, sizeof(double) * N, hipMemcpyDeviceToDevice, stream));
  if (phase) {
    HIPCHK(hipMemsetAsync(cotq, 0, sizeof(double) * Rpad, stream));
    HIPCHK(hipMemcpyAsync(cotq, cot_phase, sizeof(double) * N, hipMemcpyDeviceToDevice, stream));
  }
  if (gr) HIPCHK(hipMemsetAsync(gr, 0, sizeof(double) * np, stream));
  auto with_phase = [&](auto P, const auto& L) {
    typedef typename std::remove_const<typename std::remove_pointer<decltype(L.w)>::type>::type T;
    if (phase) {
      P.w = L.w; P.c = L.c; P.w2 = L.w2; P.c2 = L.c2;
      P.cotp = cotq;
      P.ab = (T*)ab;
      P.offW = ans->d_cx; P.offC = ans->d_cx + ans->K; P.offW2 = ans->d_cx + 2 * ans->K;
      P.offC2 = ans->d_cx + 3 * ans->K;
    }
    return P;
  };
  if (ans->tensor) HIPCHK(hipMemsetAsync(Hbuf, 0, hsz * esz, stream));   // units past ceil4(chi) stay zero
  if (precision == NQS_F64) {
    TnAdj<double> A{};
    if (ans->tensor) {
      A = tn_adj((double*)tnb, ans->tn<double>(ans->tn64));
      HIPCHK(launch_psi_tn_f64(A.P, samples, N, lphi, sphi, stream, (double*)Hbuf, Rpad));
    } else {
      PsiStates<double> X;
      X.hs = (double*)Hbuf;
      X.ns = Rpad;
      HIPCHK(launch_psi_f64(ans->params(ans->L64), samples, N, lphi, sphi, stream, X, PSI_STORE));
    }
    HIPCHK(launch_bwd_sweep_f64(with_phase(ans->adj(ans->L64), ans->L64), samples, N, Rpad, cotp,
                                (const double*)Hbuf, (double*)dcarry, (double*)Dc, (double*)Eeta, rows_per_split,
                                nsplit, gpart, np, stream, ans->tensor ? &A : nullptr));
  } else {
    TnAdj<float> A{};
    if (ans->tensor) {
      A = tn_adj((float*)tnb, ans->tn<float>(ans->tn32));
      HIPCHK(launch_psi_tn_f32(A.P, samples, N, lphi, sphi, stream, (float*)Hbuf, Rpad));
    } else {
      PsiStates<float> X;
      X.hs = (float*)Hbuf;
      X.ns = Rpad;
      HIPCHK(launch_psi_f32(ans->params(ans->L32), samples, N, lphi, sphi, stream, X, PSI_STORE));
    }
    HIPCHK(launch_bwd_sweep_f32(with_phase(ans->adj(ans->L32), ans->L32), samples, N, Rpad, cotp,
                                (const float*)Hbuf, (float*)dcarry, (float*)Dc, (float*)Eeta, rows_per_split,
                                nsplit, gpart, np, stream, ans->tensor ? &A : nullptr));
  }
  if (ans->nh)
    HIPCHK(launch_corr_backward(ans->corr(), samples, N, cotp, dth, rows_per_split, nsplit, ans->offB,
                                ans->offWc, ans->offW2, gpart, np, stream));
  if (ans->cplx) {
    HIPCHK(launch_sum_parts(np, nsplit, gpart, gr, stream));
    HIPCHK(launch_cx_grad_map(ans->cxmap(), gr, grad, stream));
  } else {
    HIPCHK(launch_sum_parts(np, nsplit, gpart, grad, stream));
  }
  HIPCHK(hipStreamSynchronize(stream));
  return NQS_OK;
}

}  // extern "C"

namespace {

// The local-energy pipeline.  cx: complex outputs (eloc_im, etnum_im, phase in
// place of sign); required for an ansatz with complex parameters.
nqs_status eloc_run(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans, const uint64_t* samples,
                    const double* counts, int64_t N, const nqs_eloc_opts* opts, double* eloc, double* eloc_im,
                    double* etnum, double* etnum_im, double* logabs, int8_t* sign, double* phase, double* fsq,
                    nqs_eloc_stats* stats, hipStream_t stream, bool cx, Arena* arena = nullptr) {
  if (!ctx || !inst || !ans || (!samples && N > 0) || N < 0) return fail(NQS_EINVAL, "bad arguments");
  nqs_status s = check_opts(opts);
  if (s != NQS_OK) return s;
  if (!ans->bound) return fail(NQS_EINVAL, "parameters not bound");
  if (ans->K != inst->K || ans->na != inst->na || ans->nb != inst->nb)
    return fail(NQS_EINVAL, "ansatz and instance describe different sectors");
  if (N > (int64_t(1) << 31) - 1) return fail(NQS_EUNSUPPORTED, "N too large");
  if ((s = check_supported(ans, opts->precision)) != NQS_OK) return s;
  DeviceGuard g(ctx->device);
  if ((s = check_samples(ctx, samples, N, inst->K, inst->na, inst->nb, stream, arena)) != NQS_OK) return s;
  if (N == 0) {
    if (stats) { std::memset(stats, 0, sizeof *stats); stats->n_conn = inst->H.n_conn; }
    return NQS_OK;
  }
  Scratch S(ctx, stream, arena);
  hipEvent_t ev[3] = {}, pe[3] = {};
  const bool timing = stats != nullptr;
  if (timing) {
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    for (auto& e : pe) HIPCHK(hipEventCreate(&e));
  }
  struct EvGuard {
    hipEvent_t* a; hipEvent_t* b; bool on;
    ~EvGuard() { if (on) for (int k = 0; k < 3; ++k) { (void)hipEventDestroy(a[k]); (void)hipEventDestroy(b[k]); } }
  } evg{ev, pe, timing};
  Pipeline P{};
  if ((s = count_and_draw(S, inst, samples, N, *opts, P, stream, timing ? ev : nullptr)) != NQS_OK) return s;
  const int64_t R = P.R;
  const int64_t cap = std::min<int64_t>(R, pass_rows_bound(inst->H, *opts, R));
  auto passes = plan_passes(P.rowptr_host, cap);
  int64_t cap_used = 0;
  for (auto& pr : passes) cap_used = std::max(cap_used, P.rowptr_host[pr.second] - P.rowptr_host[pr.first]);
  if ((s = alloc_rows(S, P, cap_used, false)) != NQS_OK) return s;
  double* lphi = S.get<double>(cap_used);
  int8_t* sphi = S.get<int8_t>(cap_used);
  double* lf = ans->nh ? S.get<double>(cap_used) : nullptr;
  int8_t* sf = ans->nh ? S.get<int8_t>(cap_used) : nullptr;
  double* theta = ans->nh ? S.get<double>(size_t(N) * ans->nh) : nullptr;
  // Ising-RBM: per-sample row-update table [N][2K][nh]
  double* Etab = ans->ising ? S.get<double>(size_t(N) * 2 * ans->K * ans->nh) : nullptr;
  double* el = eloc ? eloc : S.get<double>(N);
  double* et = etnum ? etnum : S.get<double>(N);
  double* el_i = cx ? (eloc_im ? eloc_im : S.get<double>(N)) : nullptr;
  double* et_i = cx ? (etnum_im ? etnum_im : S.get<double>(N)) : nullptr;
  double* phs = ans->cplx ? S.get<double>(cap_used) : nullptr;
  double* f2 = fsq ? fsq : S.get<double>(N);
  double* sums = S.get<double>(8);
  const int K = ans->K;
  const bool resume = resumes(*opts) && (!ans->tensor || ans->tn_mfma) && cap_used < (int64_t(1) << 31);
  Resume rs;
  double* lphi_s = nullptr;
  int8_t* sphi_s = nullptr;
  double* phs_s = nullptr;   // complex parameters: phases of the samples' pass and of the node pass
  double* phs_n = nullptr;
  if (resume) {
    rs.hs = S.get<unsigned char>(size_t(K) * N * ans->chip * state_bytes(opts->precision));
    if (is_bf16(opts->precision)) rs.he = S.get<int32_t>(size_t(K) * N);
    if (opts->precision == NQS_BF16X3) rs.hs_lo = S.get<uint16_t>(size_t(K) * N * ans->chip);
    rs.pm = S.get<unsigned char>(size_t(K + 1) * N * mantissa_bytes(opts->precision));
    rs.pe = S.get<int32_t>(size_t(K + 1) * N);
    rs.pg = S.get<int8_t>(size_t(K + 1) * N);
    if (ans->cplx) rs.pz = S.get<unsigned char>(size_t(K + 1) * N * 2 * mantissa_bytes(opts->precision));
    rs.ns = N;
    rs.perm = S.get<int32_t>(cap_used);
    rs.t0 = S.get<uint8_t>(cap_used);
    P.rows.t0 = S.get<uint8_t>(cap_used);
    rs.cnt = S.get<int32_t>(size_t(order_blocks(cap_used)) * (K + 1));
    rs.tot = S.get<int64_t>(K + 1);
    rs.owner = P.rows.owner;
    lphi_s = S.get<double>(N);
    sphi_s = S.get<int8_t>(N);
    if (ans->cplx) phs_s = S.get<double>(N);
  }
  // one level of shared prefixes (FP64/FP32; BF16 rows are cheap enough per
  // site that a node pass does not pay): node list, compact storage
  const bool nodes = resume && !is_bf16(opts->precision);
  const int64_t max_pass_samples = max_samples_per_pass(passes);
  const bool tn = ans->tensor;
  const bool pair = pair_nodes(K, tn);
  const NodeCaps caps = node_caps(cap_used, K, ans->W, pair, tn, ctx->node_cap_scale.load());
  const int64_t scap = node_slots(caps, K, tn);
  NodeList nl{};
  int32_t *ncnt = nullptr, *row_node = nullptr, *nperm = nullptr;
  int64_t *nent = nullptr, *nslt = nullptr, *nbase = nullptr, *ebase = nullptr, *ntot = nullptr;
  int64_t* sbsum = nullptr;
  NodeRec* nrec = nullptr;
  int* sover = nullptr;
  uint8_t *row_site = nullptr, *nt0s = nullptr, *ntmp_k = nullptr;
  int32_t* ntmp_p = nullptr;
  int32_t* ncnt_s = nullptr;
  int64_t* ntot_s = nullptr;
  double* lphi_n = nullptr;
  int8_t* sphi_n = nullptr;
  if (nodes) {
    const size_t esz = state_bytes(opts->precision);
    ncnt = S.get<int32_t>(max_pass_samples);
    nent = S.get<int64_t>(max_pass_samples);
    nslt = S.get<int64_t>(max_pass_samples);
    nbase = S.get<int64_t>(max_pass_samples);
    ebase = S.get<int64_t>(max_pass_samples);
    ntot = S.get<int64_t>(3);
    nl.m = S.get<uint64_t>(size_t(caps.nodes) * 2);
    nl.owner = S.get<int32_t>(caps.nodes);
    nl.c1 = S.get<uint8_t>(caps.nodes);
    nl.e1 = S.get<uint8_t>(caps.nodes);
    nl.off = S.get<int64_t>(caps.nodes);
    nperm = S.get<int32_t>(caps.nodes);
    nt0s = S.get<uint8_t>(caps.nodes);
    ntmp_p = S.get<int32_t>(size_t(caps.nodes) * 2);
    ntmp_k = S.get<uint8_t>(size_t(caps.nodes) * 2);
    nl.need = S.get<uint64_t>(caps.nodes);
    nrec = S.get<NodeRec>(caps.nodes);
    if (!tn) {
      sbsum = S.get<int64_t>(slot_blocks(caps.nodes));
      sover = S.get<int>(1);
    }
    ncnt_s = S.get<int32_t>(size_t(order_blocks(cap_used)) * (K + 1));
    ntot_s = S.get<int64_t>(K + 1);
    lphi_n = S.get<double>(caps.nodes);
    sphi_n = S.get<int8_t>(caps.nodes);
    rs.nhs = S.get<unsigned char>(size_t(scap) * ans->chip * esz);
    rs.nlp = S.get<LogProd<double>>(caps.entries);
    if (ans->cplx) {
      rs.npz = S.get<unsigned char>(size_t(caps.entries) * 2 * mantissa_bytes(opts->precision));
      phs_n = S.get<double>(caps.nodes);
    }
    row_node = S.get<int32_t>(cap_used);
    row_site = S.get<uint8_t>(cap_used);
    P.rows.sec = S.get<uint32_t>(cap_used);
  }
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  if (sover) HIPCHK(hipMemsetAsync(sover, 0, sizeof(int), stream));
  if (ans->nh) HIPCHK(launch_corr_theta(ans->corr(), samples, N, theta, Etab, opts->precision, stream));
  float ms_rows = 0, ms_amp = 0, ms_red = 0, ms_psi = 0;
  int64_t site_rows = 0;
  double psi_flops = 0;
  // algorithmic flops of a row evaluated from site k on: 8 chi^2 d_i per site i >= k
  std::vector<double> tail_flops(K + 1, 0.0);
  for (int i = K - 1; i >= 0; --i)
    tail_flops[i] = tail_flops[i + 1] + site_flops(*ans, i);
  hipEvent_t kq[2] = {};
  struct KqGuard {
    hipEvent_t* e;
    ~KqGuard() { for (int k = 0; k < 2; ++k) if (e[k]) (void)hipEventDestroy(e[k]); }
  } kqg{kq};
  if (timing) for (auto& e : kq) HIPCHK(hipEventCreate(&e));
  if (resume) {
    // the samples' own pass: carried and log-product states at every site
    if (timing) HIPCHK(hipEventRecord(pe[0], stream));
    if ((s = run_amplitudes(ans, opts->precision, samples, N, lphi_s, sphi_s, stream, &rs, PSI_STORE, phs_s)) !=
        NQS_OK)
      return s;
    site_rows += int64_t(N) * K;
    if (timing) {
      HIPCHK(hipEventRecord(pe[1], stream));
      HIPCHK(hipEventSynchronize(pe[1]));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, pe[0], pe[1]));
      ms_amp += t;
    }
  }
  for (auto& pr : passes) {
    const int64_t n0 = pr.first, n1 = pr.second;
    const int64_t Rp = P.rowptr_host[n1] - P.rowptr_host[n0];
    if (timing) HIPCHK(hipEventRecord(pe[0], stream));
    if ((s = fill_range(inst, samples, n0, n1, *opts, P, stream)) != NQS_OK) return s;
    if (timing) HIPCHK(hipEventRecord(pe[1], stream));
    if (resume) {
      const uint8_t* key = P.rows.t0;
      rs.unode = nullptr;
      if (nodes) {
        // nodes of this pass: count, place (host learns the totals), assign
        const int64_t ns = n1 - n0, row_base = P.rowptr_host[n0];
        HIPCHK(launch_node_count(P.rows.t0, P.rows.sec, samples, P.rowptr, n0, n1, row_base, K, ans->W, pair, ncnt,
                                 nent, nslt, stream));
        HIPCHK(launch_node_scan(ns, caps, ncnt, nent, nslt, nbase, ebase, ntot, stream));
        int64_t tot2[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(tot2, ntot, sizeof tot2, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        HIPCHK(launch_node_assign(P.rows.t0, P.rows.sec, samples, P.rowptr, n0, n1, row_base, K, ans->W, pair, nbase,
                                  ebase, nl, row_node, row_site, stream));
        const int64_t nn = tot2[0];
        // the rows' order first: it fixes which node states the row pass reads
        HIPCHK(launch_order_t0(row_site, Rp, K, rs.cnt, rs.tot, rs.perm, rs.t0, stream));
        if (nn > 0) {
          HIPCHK(launch_node_need(rs.perm, rs.t0, Rp, ans->W, row_node, nl.c1, nl.need, stream));
          // node records; carried-state slots only for the sites some row
          // reads (the tensor-term kernels store every site, a slot per entry)
          HIPCHK(launch_node_records(nl, nn, !tn, scap, sbsum, ntot + 2, nrec, sover, stream));
          // the node pass: resumed from the samples at the changed site, stores compactly
          // node units by changed site, and from chi = 32 on by (changed
          // site, last site): a wavefront starts at its first unit's changed
          // site and stops after its units' last site.  At smaller chi a site
          // costs little next to a unit's start, and the changed-site order,
          // which keeps a sample's units together, measured faster.
          if (ans->chip >= 32)
            HIPCHK(launch_order_t0_t1(nl.c1, nl.e1, nn, K, ncnt_s, ntot_s, ntmp_p, ntmp_k, nperm, nt0s, stream));
          else
            HIPCHK(launch_order_t0(nl.c1, nn, K, ncnt_s, ntot_s, nperm, nt0s, stream));
          Resume rn = rs;
          rn.perm = nperm;
          rn.t0 = nt0s;
          rn.owner = nl.owner;
          rn.nrec = nrec;
          rn.unode = nullptr;
          if ((s = run_amplitudes(ans, opts->precision, nl.m, nn, lphi_n, sphi_n, stream, &rn, PSI_NODE, phs_n)) !=
              NQS_OK)
            return s;
          // a node is evaluated from its first changed site to the largest
          // resume site of its rows: (entries - 1) sites
          site_rows += tot2[1] - tot2[0];
        }
        rs.nrec = nrec;
        rs.unode = row_node;
      } else {
        HIPCHK(launch_order_t0(key, Rp, K, rs.cnt, rs.tot, rs.perm, rs.t0, stream));
      }
      if (timing) HIPCHK(hipEventRecord(kq[0], stream));
      if ((s = run_amplitudes(ans, opts->precision, P.rows.m, Rp, lphi, sphi, stream, &rs, PSI_SEED, phs)) != NQS_OK)
        return s;
      if (timing) HIPCHK(hipEventRecord(kq[1], stream));
      if (stats) {
        std::vector<int64_t> tot(K + 1);
        HIPCHK(hipMemcpyAsync(tot.data(), rs.tot, sizeof(int64_t) * (K + 1), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        for (int k = 0; k <= K; ++k) {
          site_rows += tot[k] * (K - k);
          psi_flops += double(tot[k]) * tail_flops[k];
        }
      }
    } else {
      if (timing) HIPCHK(hipEventRecord(kq[0], stream));
      if ((s = run_amplitudes(ans, opts->precision, P.rows.m, Rp, lphi, sphi, stream, nullptr, PSI_PLAIN, phs)) !=
          NQS_OK)
        return s;
      if (timing) HIPCHK(hipEventRecord(kq[1], stream));
      site_rows += Rp * K;
      psi_flops += double(Rp) * tail_flops[0];
    }
    if (timing) HIPCHK(hipEventRecord(pe[2], stream));
    if (ans->nh)
      HIPCHK(launch_corr_rows(ans->corr(), P.rows.m, P.rows.owner, samples, theta, Etab, Rp, opts->precision, lf,
                              sf, stream));
    if (cx)
      HIPCHK(launch_reduce_cx(n0, n1, P.rowptr, P.rowptr_host[n0], P.rows.coef, lphi, sphi, phs, lf, sf, P.hdiag,
                              el, el_i, et, et_i, logabs, phase, f2, stream));
    else
      HIPCHK(launch_reduce(n0, n1, P.rowptr, P.rowptr_host[n0], P.rows.coef, lphi, sphi, lf, sf, P.hdiag, el, et,
                           logabs, sign, f2, stream));
    if (timing) {
      hipEvent_t done;
      HIPCHK(hipEventCreate(&done));
      HIPCHK(hipEventRecord(done, stream));
      HIPCHK(hipEventSynchronize(done));
      float t = 0;
      HIPCHK(hipEventElapsedTime(&t, pe[0], pe[1])); ms_rows += t;
      HIPCHK(hipEventElapsedTime(&t, pe[1], pe[2])); ms_amp += t;
      HIPCHK(hipEventElapsedTime(&t, pe[2], done)); ms_red += t;
      HIPCHK(hipEventElapsedTime(&t, kq[0], kq[1])); ms_psi += t;
      (void)hipEventDestroy(done);
    }
  }
  HIPCHK(launch_batch_sums(N, counts, el, et, f2, sums, stream, el_i, et_i));
  double hs[8] = {0};
  int slot_overflow = 0;
  if (stats) HIPCHK(hipMemcpyAsync(hs, sums, sizeof hs, hipMemcpyDeviceToHost, stream));
  if (sover) HIPCHK(hipMemcpyAsync(&slot_overflow, sover, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (slot_overflow) return fail(NQS_EDEVICE, "node state slots exceeded their capacity");
  if (stats) {
    std::vector<int64_t> Dn(N), Un(N);
    HIPCHK(hipMemcpy(Dn.data(), P.Dn, sizeof(int64_t) * N, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(Un.data(), P.Un, sizeof(int64_t) * N, hipMemcpyDeviceToHost));
    std::memset(stats, 0, sizeof *stats);
    stats->n_samples = N;
    stats->n_conn = inst->H.n_conn;
    stats->n_rows = R;
    for (int64_t n = 0; n < N; ++n) { stats->n_det_rows += Dn[n]; stats->n_draw_rows += Un[n]; }
    stats->sum_c = hs[0];
    stats->B = hs[4];
    stats->E = hs[3];
    stats->var = hs[5];
    stats->n_zero_amp = int64_t(hs[6]);
    stats->n_passes = int64_t(passes.size());
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1])); stats->ms_enumerate = t;
    HIPCHK(hipEventElapsedTime(&t, ev[1], ev[2])); stats->ms_draw = t;
    stats->ms_rows = ms_rows;
    stats->ms_amplitude = ms_amp;
    stats->ms_reduce = ms_red;
    stats->n_site_rows = site_rows;
    stats->ms_psi = ms_psi;
    stats->psi_flops = psi_flops;
    stats->E_im = hs[7];
  }
  return NQS_OK;
}

}  // namespace

extern "C" {

nqs_status nqs_eloc(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans,
                    const uint64_t* samples, const double* counts, int64_t N,
                    const nqs_eloc_opts* opts, double* eloc, double* etnum, double* logabs,
                    int8_t* sign, double* fsq, nqs_eloc_stats* stats, hipStream_t stream) {
  if (ans && ans->cplx)
    return fail(NQS_EINVAL, "complex parameters give complex local energies: use nqs_eloc_complex");
  return eloc_run(ctx, inst, ans, samples, counts, N, opts, eloc, nullptr, etnum, nullptr, logabs, sign, nullptr, fsq,
                  stats, stream, false);
}

nqs_status nqs_eloc_noalloc(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans,
                            const uint64_t* samples, const double* counts, int64_t N,
                            const nqs_eloc_opts* opts, double* eloc, double* etnum, double* logabs,
                            int8_t* sign, double* fsq, hipStream_t stream) {
  if (!ctx) return fail(NQS_EINVAL, "ctx is NULL");
  if (ans && ans->cplx)
    return fail(NQS_EINVAL, "complex parameters give complex local energies: use nqs_eloc_complex");
  if (!ctx->arena)
    return fail(NQS_EDEVICE, "static workspace of device %d unavailable: %s", ctx->device,
                hipGetErrorString(ctx->arena_err));
  Arena A;
  A.base = static_cast<unsigned char*>(ctx->arena);
  A.size = kStaticWorkspaceBytes;
  nqs_status s = eloc_run(ctx, inst, ans, samples, counts, N, opts, eloc, nullptr, etnum, nullptr, logabs, sign,
                          nullptr, fsq, nullptr, stream, false, &A);
  if (s != NQS_OK) {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(stream);   // queued work may still use the array
    (void)hipGetLastError();
    if (A.overflow)
      return fail(NQS_ENOMEM, "the call needs more than the %zu-byte static workspace (bound it with "
                  "max_rows_per_pass; see nqs_eloc_workspace_bytes)", kStaticWorkspaceBytes);
  }
  return s;
}

nqs_status nqs_eloc_complex(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans,
                            const uint64_t* samples, const double* counts, int64_t N,
                            const nqs_eloc_opts* opts, double* eloc_re, double* eloc_im, double* etnum_re,
                            double* etnum_im, double* logabs, double* phase, double* fsq,
                            nqs_eloc_stats* stats, hipStream_t stream) {
  return eloc_run(ctx, inst, ans, samples, counts, N, opts, eloc_re, eloc_im, etnum_re, etnum_im, logabs, nullptr,
                  phase, fsq, stats, stream, true);
}

namespace {
// a pool block released when the holder goes out of scope
// (behind the work queued on its stream, as for Scratch)
struct PoolBlock {
  nqs_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  void* p = nullptr;
  PoolBlock() = default;
  PoolBlock(const PoolBlock&) = delete;
  PoolBlock& operator=(const PoolBlock&) = delete;
  bool get(nqs_ctx* c, size_t bytes, hipStream_t s) {
    reset();
    ctx = c;
    st = s;
    p = c->acquire(std::max<size_t>(bytes, 1));
    return p != nullptr;
  }
  void reset() {
    if (p) {
      std::vector<void*> v{p};
      ctx->release_after(v, st);
    }
    p = nullptr;
  }
  void swap(PoolBlock& o) {
    std::swap(ctx, o.ctx);
    std::swap(st, o.st);
    std::swap(p, o.p);
  }
  ~PoolBlock() { reset(); }
};

// unique ONVs with counts and amplitudes, in one pool block
struct UniqueSet {
  PoolBlock blk;
  uint64_t* m = nullptr;
  int64_t* c = nullptr;
  double* l = nullptr;
  int8_t* s = nullptr;
  bool alloc(nqs_ctx* ctx, int64_t n, hipStream_t st) {
    const size_t n8 = size_t(std::max<int64_t>(n, 1));
    const size_t bm = n8 * 16, bc = n8 * 8, bl = n8 * 8, bs = (n8 + 255) / 256 * 256;
    if (!blk.get(ctx, bm + bc + bl + bs, st)) return false;
    char* q = static_cast<char*>(blk.p);
    m = reinterpret_cast<uint64_t*>(q);
    c = reinterpret_cast<int64_t*>(q + bm);
    l = reinterpret_cast<double*>(q + bm + bc);
    s = reinterpret_cast<int8_t*>(q + bm + bc + bl);
    return true;
  }
};
}  // namespace

nqs_status nqs_sample(nqs_ctx* ctx, const nqs_ansatz* ans, int64_t n_draws, uint64_t seed, int64_t draw_base,
                      int32_t precision, int64_t max_draws_per_pass, int64_t cap, uint64_t* samples, int64_t* counts,
                      double* logabs, int8_t* sign, int64_t* n_unique, hipStream_t stream) {
  if (!ctx || !ans || n_draws < 0 || draw_base < 0 || max_draws_per_pass < 0 || cap < 0 || !n_unique ||
      (cap > 0 && (!samples || !counts)))
    return fail(NQS_EINVAL, "bad arguments");
  if (n_draws > std::numeric_limits<int64_t>::max() - draw_base) return fail(NQS_EINVAL, "draw index overflow");
  if (!ans->bound) return fail(NQS_EINVAL, "parameters not bound");
  if (precision != NQS_F64 && precision != NQS_F32)
    return fail(NQS_EUNSUPPORTED, "sampling runs in FP64 or FP32");
  if (ans->cplx && sign)
    return fail(NQS_EINVAL, "complex parameters have a phase, not a sign: pass sign = NULL (nqs_logpsi_phase)");
  const int64_t chunk = max_draws_per_pass > 0 && max_draws_per_pass < n_draws ? max_draws_per_pass : n_draws;
  constexpr int64_t kMaxSort = (int64_t(1) << 31) - 1;   // hipCUB item count
  if (chunk > kMaxSort) return fail(NQS_EUNSUPPORTED, "more than 2^31 - 1 draws in one pass");
  DeviceGuard g(ctx->device);
  *n_unique = 0;
  if (n_draws == 0) return NQS_OK;
  const bool two = 2 * ans->K > 64;
  Scratch S(ctx, stream);
  uint64_t* m = S.get<uint64_t>(size_t(chunk) * 2);
  double* lphi = S.get<double>(chunk);
  int8_t* sphi = S.get<int8_t>(chunk);
  int64_t* nu = S.get<int64_t>(1);
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  // draws run in passes of at most `chunk`; each pass is merged with the unique
  // set of the passes before it (their counts as weights), so the workspace is
  // bounded by the pass size plus the number of unique draws
  UniqueSet set;
  int64_t u = 0;
  for (int64_t d0 = 0; d0 < n_draws; d0 += chunk) {
    const int64_t ch = std::min(chunk, n_draws - d0);
    const bool last = d0 + ch >= n_draws;
    SampleArgs SA;
    SA.k0 = uint32_t(seed);
    SA.k1 = uint32_t(seed >> 32);
    SA.p0 = draw_base + d0;
    SA.out = m;
    if (ans->tensor && !ans->tn_mfma && precision == NQS_F64) {
      if (!ans->tn_f64_ok) return fail(NQS_EUNSUPPORTED, "FP64 tensor-RNN ring does not fit the LDS");
      HIPCHK(launch_sample_tn_f64(ans->tn<double>(ans->tn64), ch, lphi, sphi, stream, SA));
    } else if (ans->tensor && !ans->tn_mfma) {
      HIPCHK(launch_sample_tn_f32(ans->tn<float>(ans->tn32), ch, lphi, sphi, stream, SA));
    } else if (precision == NQS_F64) {
      HIPCHK(launch_sample_f64(ans->params(ans->fwd64()), ch, lphi, sphi, stream, SA));
    } else {
      HIPCHK(launch_sample_f32(ans->params(ans->fwd32()), ch, lphi, sphi, stream, SA));
    }
    const int64_t n = u + ch;
    if (n > kMaxSort) return fail(NQS_EUNSUPPORTED, "more than 2^31 - 1 unique draws plus one pass");
    Scratch T(ctx, stream);
    const uint64_t* im = m;
    const double* il = lphi;
    const int8_t* is = sphi;
    int64_t* iw = nullptr;
    if (u > 0) {
      uint64_t* cm = T.get<uint64_t>(size_t(n) * 2);
      double* cl = T.get<double>(n);
      int8_t* cs = T.get<int8_t>(n);
      iw = T.get<int64_t>(n);
      if (T.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
      HIPCHK(hipMemcpyAsync(cm, set.m, size_t(u) * 16, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpyAsync(cm + 2 * u, m, size_t(ch) * 16, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpyAsync(cl, set.l, size_t(u) * 8, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpyAsync(cl + u, lphi, size_t(ch) * 8, hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpyAsync(cs, set.s, size_t(u), hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpyAsync(cs + u, sphi, size_t(ch), hipMemcpyDeviceToDevice, stream));
      HIPCHK(hipMemcpyAsync(iw, set.c, size_t(u) * 8, hipMemcpyDeviceToDevice, stream));
      HIPCHK(launch_fill_i64(iw + u, ch, 1, stream));
      im = cm;
      il = cl;
      is = cs;
    }
    UniqueScratch w{};
    HIPCHK(unique_temp_bytes(n, &w.temp_bytes));
    w.temp = T.get<unsigned char>(w.temp_bytes);
    w.key_a = T.get<uint64_t>(n);
    w.key_b = T.get<uint64_t>(n);
    w.ord_a = T.get<uint32_t>(n);
    w.ord_b = T.get<uint32_t>(n);
    w.flag = T.get<int32_t>(n);
    w.pos = T.get<int32_t>(n);
    w.start = T.get<int64_t>(n);
    w.wsum = iw ? T.get<int64_t>(n) : nullptr;
    if (T.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
    if (last) {
      HIPCHK(launch_unique(im, il, is, iw, n, two, w, cap, samples, counts, logabs, sign, nu, stream));
      int64_t h = 0;
      HIPCHK(hipMemcpyAsync(&h, nu, sizeof h, hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));   // before this pass's buffers go back to the pool
      *n_unique = h;
    } else {
      UniqueSet next;
      if (!next.alloc(ctx, n, stream)) return fail(NQS_ENOMEM, "workspace allocation failed");
      HIPCHK(launch_unique(im, il, is, iw, n, two, w, n, next.m, next.c, next.l, next.s, nu, stream));
      HIPCHK(hipMemcpyAsync(&u, nu, sizeof u, hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));   // the old set and this pass's buffers are free after this
      set.blk.swap(next.blk);
      set.m = next.m;
      set.c = next.c;
      set.l = next.l;
      set.s = next.s;
    }
  }
  return NQS_OK;
}

nqs_status nqs_rows(nqs_ctx* ctx, const nqs_instance* inst, const uint64_t* samples, int64_t N,
                    const nqs_eloc_opts* opts, int64_t cap, int64_t* row_ptr, int64_t* n_det,
                    uint64_t* Q, int64_t* rank, double* coef, uint64_t* m, int64_t* n_rows,
                    hipStream_t stream) {
  if (!ctx || !inst || (!samples && N > 0) || N < 0 || cap < 0) return fail(NQS_EINVAL, "bad arguments");
  nqs_status s = check_opts(opts);
  if (s != NQS_OK) return s;
  DeviceGuard g(ctx->device);
  if ((s = check_samples(ctx, samples, N, inst->K, inst->na, inst->nb, stream)) != NQS_OK) return s;
  if (N == 0) { if (n_rows) *n_rows = 0; return NQS_OK; }
  Scratch S(ctx, stream);
  Pipeline P{};
  if ((s = count_and_draw(S, inst, samples, N, *opts, P, stream, nullptr)) != NQS_OK) return s;
  const int64_t R = P.R, w = std::min(R, cap);
  if (w > 0) {
    if ((s = alloc_rows(S, P, R, true)) != NQS_OK) return s;
    if ((s = fill_range(inst, samples, 0, N, *opts, P, stream)) != NQS_OK) return s;
  }
  if (row_ptr) HIPCHK(hipMemcpyAsync(row_ptr, P.rowptr, sizeof(int64_t) * (N + 1), hipMemcpyDeviceToDevice, stream));
  if (n_det) HIPCHK(hipMemcpyAsync(n_det, P.Dn, sizeof(int64_t) * N, hipMemcpyDeviceToDevice, stream));
  if (Q) HIPCHK(hipMemcpyAsync(Q, P.Qn, sizeof(uint64_t) * N, hipMemcpyDeviceToDevice, stream));
  if (w > 0) {
    if (rank) HIPCHK(hipMemcpyAsync(rank, P.rows.rank, sizeof(int64_t) * w, hipMemcpyDeviceToDevice, stream));
    if (coef) HIPCHK(hipMemcpyAsync(coef, P.rows.coef, sizeof(double) * w, hipMemcpyDeviceToDevice, stream));
    if (m) HIPCHK(hipMemcpyAsync(m, P.rows.m, sizeof(uint64_t) * 2 * w, hipMemcpyDeviceToDevice, stream));
  }
  HIPCHK(hipStreamSynchronize(stream));
  if (n_rows) *n_rows = R;
  return NQS_OK;
}

nqs_status nqs_eloc_workspace_bytes(const nqs_instance* inst, const nqs_ansatz* ans, int64_t N,
                                    const nqs_eloc_opts* opts, int64_t n_rows, size_t* bytes) {
  if (!inst || !ans || !opts || !bytes || N < 0 || n_rows < 0) return fail(NQS_EINVAL, "bad arguments");
  if (N == 0) { *bytes = 0; return NQS_OK; }
  const EnumGeom G = make_geom(inst->H.n_conn, N);
  const int64_t ne = std::max(opts->n_eps, 1);
  auto al = [](size_t b) { return size_class(b); };
  size_t b = 0;
  // count_and_draw
  b += 2 * al(size_t(N) * G.nchunks * 8);
  b += al(size_t(N) * G.S * 8) + al(size_t(N) * G.S * 4);
  b += 3 * al(size_t(N) * 8) + al(size_t(N + 1) * 8);
  b += al(size_t(N) * ne * 4) + al(size_t(N) * ne * 8) + al(size_t(N) * ne * 16);
  b += al(size_t(N) * 8);
  // rows of the largest pass: m(16) coef(8) owner(4) lphi(8) sphi(1), with a correlator lf(8) sf(1)
  const int64_t rows = opts->max_rows_per_pass > 0 ? pass_rows_bound(inst->H, *opts, 0) : n_rows;
  b += al(size_t(rows) * 16) + al(size_t(rows) * 8) + al(size_t(rows) * 4);
  b += al(size_t(rows) * 8) + al(size_t(rows));
  if (ans->nh) b += al(size_t(rows) * 8) + al(size_t(rows));
  if (ans->nh) b += al(size_t(N) * ans->nh * 8);
  if (ans->ising) b += al(size_t(N) * 2 * ans->K * ans->nh * 8);
  if (resumes(*opts)) {
    // samples' carried and log-product states, the pass's row order
    const int K = ans->K;
    b += al(size_t(K) * N * ans->chip * state_bytes(opts->precision));
    if (is_bf16(opts->precision)) b += al(size_t(K) * N * 4);
    if (opts->precision == NQS_BF16X3) b += al(size_t(K) * N * ans->chip * 2);
    b += al(size_t(K + 1) * N * mantissa_bytes(opts->precision)) + al(size_t(K + 1) * N * 4);
    b += al(size_t(K + 1) * N) + al(size_t(rows) * 4) + 2 * al(size_t(rows));
    b += al(size_t(order_blocks(rows)) * (K + 1) * 4) + al(size_t(K + 1) * 8);
    b += al(size_t(N) * 8) + al(size_t(N));
    if (!is_bf16(opts->precision)) {
      // node level: per-sample counts, node list, node order, storage, rows' nodes
      const bool tn = ans->tensor;
      const NodeCaps c = node_caps(rows, K, ans->W, pair_nodes(K, tn), tn);
      const int64_t nslots = node_slots(c, K, tn);
      const size_t esz = state_bytes(opts->precision);
      b += al(size_t(N) * 4) + 4 * al(size_t(N) * 8) + al(24);
      b += al(size_t(c.nodes) * 16) + al(size_t(c.nodes) * 4) + 2 * al(size_t(c.nodes)) + al(size_t(c.nodes) * 8);
      b += al(size_t(c.nodes) * 4) + al(size_t(c.nodes)) + al(size_t(c.nodes) * 8);
      b += al(size_t(c.nodes) * 8) + al(size_t(c.nodes) * 2);
      b += al(size_t(c.nodes) * sizeof(NodeRec));
      if (!tn) b += al(size_t(slot_blocks(c.nodes)) * 8) + al(4);
      b += al(size_t(c.nodes) * 8) + al(size_t(c.nodes));
      b += al(size_t(nslots) * ans->chip * esz) + al(size_t(c.entries) * sizeof(LogProd<double>));
      if (ans->cplx)
        b += al(size_t(c.entries) * 2 * mantissa_bytes(opts->precision)) + al(size_t(c.nodes) * 8);
      b += al(size_t(rows) * 4) + al(size_t(rows)) + al(size_t(rows) * 4);
      b += al(size_t(order_blocks(rows)) * (K + 1) * 4) + al(size_t(K + 1) * 8);
    }
  }
  b += 3 * al(size_t(N) * 8) + al(64);     // outputs the caller did not provide, batch sums
  b += al(4);                              // sample validation flag
  *bytes = b;
  return NQS_OK;
}

nqs_status nqs_vmc_step(nqs_ctx* ctx, const nqs_instance* inst, nqs_ansatz* ans, const nqs_vmc_opts* opts,
                        double* params, double* adam_m, double* adam_v, double* grad, nqs_vmc_stats* stats,
                        hipStream_t stream) {
  if (!ctx || !inst || !ans || !opts || !params || !adam_m || !adam_v) return fail(NQS_EINVAL, "NULL argument");
  if (opts->n_draws < 1) return fail(NQS_EINVAL, "n_draws < 1");
  if (opts->step < 1) return fail(NQS_EINVAL, "AdamW step numbers start at 1");
  if (!(opts->lr >= 0) || !(opts->beta1 >= 0 && opts->beta1 < 1) || !(opts->beta2 >= 0 && opts->beta2 < 1) ||
      !(opts->adam_eps > 0) || !(opts->weight_decay >= 0))
    return fail(NQS_EINVAL, "bad AdamW hyperparameters");
  if (!ans->bound) return fail(NQS_EINVAL, "parameters not bound");
  const int32_t prec = opts->eloc.precision;
  const int32_t low = prec == NQS_F64 ? NQS_F64 : NQS_F32;   // sampler and adjoint precision
  const int64_t np = ans->n_params;
  DeviceGuard g(ctx->device);
  auto now = [] { return std::chrono::steady_clock::now(); };
  auto ms = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
  };
  const int64_t D = opts->n_draws;
  Scratch S(ctx, stream);
  uint64_t* smp = S.get<uint64_t>(size_t(D) * 2);
  int64_t* cnt = S.get<int64_t>(D);
  double* cd = S.get<double>(D);
  double* etn = S.get<double>(D);
  double* f2 = S.get<double>(D);
  double* cot = S.get<double>(D);
  double* etn_i = ans->cplx ? S.get<double>(D) : nullptr;
  double* cotq = ans->cplx ? S.get<double>(D) : nullptr;
  double* gbuf = grad ? grad : S.get<double>(np);
  double* red = S.get<double>(4);
  if (S.oom) return fail(NQS_ENOMEM, "workspace allocation failed");
  nqs_status st;
  // 1. exact draws from Phi^2, merged into unique samples with counts
  const auto t0 = now();
  int64_t U = 0;
  if ((st = nqs_sample(ctx, ans, D, opts->sample_seed, opts->draw_base, low, opts->max_draws_per_pass, D, smp, cnt,
                       nullptr, nullptr, &U, stream)) != NQS_OK)
    return st;
  HIPCHK(launch_i64_to_f64(U, cnt, cd, stream));
  // 2. semi-stochastic local energies of the unique samples, weighted by counts
  const auto t1 = now();
  nqs_eloc_stats es;
  if (ans->cplx)
    st = nqs_eloc_complex(ctx, inst, ans, smp, cd, U, &opts->eloc, nullptr, nullptr, etn, etn_i, nullptr, nullptr, f2,
                          &es, stream);
  else
    st = nqs_eloc(ctx, inst, ans, smp, cd, U, &opts->eloc, nullptr, etn, nullptr, nullptr, f2, &es, stream);
  if (st != NQS_OK) return st;
  // 3. the reweighted gradient (Eq. (19)) as the VJP of ln|Psi| with cotangent
  // cot (and of the phase with cotq for complex parameters)
  const auto t2 = now();
  if (ans->cplx)
    HIPCHK(launch_vmc_cotangent_cx(U, cd, etn, etn_i, f2, cot, cotq, red, stream));
  else
    HIPCHK(launch_vmc_cotangent(U, cd, etn, f2, cot, red, stream));
  HIPCHK(hipMemsetAsync(gbuf, 0, sizeof(double) * np, stream));
  if ((st = nqs_logpsi_vjp_phase(ctx, ans, smp, U, cot, cotq, low, gbuf, stream)) != NQS_OK) return st;
  // 4. AdamW on the packed parameters, then the kernels' layouts are rebuilt
  const auto t3 = now();
  HIPCHK(launch_sumsq(np, gbuf, red + 2, stream));
  HIPCHK(launch_adamw(np, params, gbuf, adam_m, adam_v, opts->step, opts->lr, opts->beta1, opts->beta2,
                      opts->adam_eps, opts->weight_decay, stream));
  // projected step: eta >= 0 (Sec. 2.1); the caller's packed layout (complex: cEta of the map)
  if (ans->cplx)
    HIPCHK(launch_project_eta(ans->K, ans->chi_c, ans->d_cx + 5 * ans->K, params, stream));
  else
    HIPCHK(launch_project_eta(ans->K, ans->chi, ans->d_offEta, params, stream));
  double hred[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(hred, red, sizeof hred, hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if ((st = nqs_ansatz_bind_params(ans, params, stream)) != NQS_OK) return st;
  const auto t4 = now();
  if (stats) {
    stats->n_unique = U;
    stats->E = hred[0];
    stats->var = es.var;
    stats->B = es.B;
    stats->grad_norm = std::sqrt(hred[2]);
    stats->ms_sample = ms(t0, t1);
    stats->ms_eloc = ms(t1, t2);
    stats->ms_grad = ms(t2, t3);
    stats->ms_update = ms(t3, t4);
  }
  return NQS_OK;
}

}  // extern "C"
