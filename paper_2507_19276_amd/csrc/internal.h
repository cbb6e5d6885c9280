// Internal declarations shared by the HIP kernels and the host runtime of
// libnqs.  Nothing here is part of the C ABI (include/nqs.h).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "nqs.h"

namespace nqs {

constexpr int kWave = 64;

// Hamiltonian of one instance as the kernels see it.  Ranks of the connected
// determinants of a sample run over five blocks (alpha singles, beta
// singles, alpha-alpha doubles, beta-beta doubles, alpha-beta doubles); the
// block sizes depend only on (K, n_alpha, n_beta), so every sample of an
// instance has the same rank space [0, n_conn).
struct HamDev {
  const double* h;     // [K][K]
  const double* eri;   // [K][K][K][K] chemist (pq|rs), exactly 8-fold symmetric
  const double* jk;    // [2][K][K]: (pp|qq) and (pq|qp), copies of eri entries for the diagonal
  const double* s3;    // [K][K][K][2]: (ai|jj) and (aj|ji) at [a][i][j], copies of eri entries for the singles
  double ecore;
  int K, na, nb, va, vb;                 // va = K - na, vb = K - nb
  uint32_t off_sb, off_daa, off_dbb, off_dab, n_conn;
  uint32_t npa_v, npb_v, nsb;            // C(va,2), C(vb,2), nb*vb
  // ceil(2^32 / d) for exact division q = (x * m) >> 32 of the operands the
  // unranking meets (x * d < 2^32 holds for every K <= 64, checked on the host)
  uint64_t mg_va, mg_vb, mg_npa_v, mg_npb_v, mg_nsb;
};

// Geometry of the chunked enumeration: a chunk is 64 consecutive ranks of one
// sample (one wavefront); the chunks of a sample are split into S contiguous
// segments processed by different wavefronts.
struct EnumGeom {
  int nchunks;   // ceil(n_conn / 64)
  int S;         // segments per sample
  int cps;       // chunks per segment
};

struct DrawKeys {
  uint32_t key0, key1;       // Philox key (seed lo, hi)
  uint32_t ctr2, ctr3;       // stream id lo, hi
  uint32_t sample_base;
};

// Ansatz parameters in kernel layouts for one precision T (double or float).
// chip = chi rounded up to 16; padded entries are zero so they never change
// a result.
template <typename T>
struct PsiParams {
  int K, chi, chip, na, nb, W;   // W = LDS ring slots (the most carried states live at once)
  const int* pptr;               // [K+1] forward edges of site i: pptr[i]..pptr[i+1]-1 (never empty)
  const int* slot;               // [edges] ring slot read by each edge (W: a parentless site's zero edge)
  const int* wsl;                // [K] ring slot receiving site i's carried state
  const uint64_t* live;          // [K+1] bit s: the state of site s < i is read by a site >= i (live[K] = 0:
                                 // rows with no change below K, the samples' own rows among them, resume at K)
  const T* A;                    // [edges + 1][CH/4][CH/4][64] k-permuted MFMA A operands, see runtime.cpp
  const T* v;                    // [K][4][chip]
  const T* eta;                  // [K][chip]
  const T* w;                    // [K][chip]
  const T* c;                    // [K]
  bool folded;                   // operands carry sqrt(eta) (see k_psi_mt); never with a carried-state store
  bool d1 = false;               // every site has exactly one edge (pptr[i+1] - pptr[i] == 1)
  const T* w2 = nullptr;         // complex parameters (realified state): [K][chip] vector of Im z
  const T* c2 = nullptr;         // [K] Im c
  // BDG-TensorRNN term on MFMA (chip <= 32, chi' <= 8): the operand stream
  // (per tensor site: projections [parent][k-step][lane], core
  // [k-step][tile 0..1][lane], output factor [state][tile][v][lane], built in
  // runtime.cpp) and per site {chi' (0: none), offsets of the three parts}
  const T* TA = nullptr;
  const int* tsite = nullptr;    // [K][4]
};

// BDG-TensorRNN forward (tensor_rnn.hip), one precision T.
template <typename T>
struct TnParams {
  int K, chi, chip, rw, na, nb, W;   // rw = ceil4(chi): units of a carried state in the ring
  int qp;                            // padded width of the projections and of U's last index (8 or 16)
  const T* prm;                  // kernel layout: per edge M^T [4][chip][chip]; per site v [4][chip],
                                 // eta, w [chip], c; per tensor site K0^T [chi'][chip],
                                 // K_j [d][chip][qp], U [4][chi'^d][qp]
  const int* pptr;               // [K+1] parents of site i: pptr[i]..pptr[i+1]-1
  const int* edge;               // [edges][2]: offset of M^T, ring slot of the parent
  const int* site;               // [K][8]: offV, offEta, offW, offC, chi' (0: none), offK0, offKj, offU
};

// Adjoint (backward) layouts for one precision T.
template <typename T>
struct AdjParams {
  int K, chi, chip, na, nb;
  const int* pptr;               // device [K+1]
  const int* pidx;               // device
  const int* pptr_host;          // host copy, launch sizing only
  const T* AF;                   // recompute A operands, k-permuted (see adjoint.hip)
  const int64_t* afoff;          // device [K]
  const T* BT;                   // M^T operands for the parent cotangents
  const int64_t* btoff;          // device [K]
  const T* v;                    // [K][4][chip]
  const T* eta;                  // [K][chip]
  const int64_t* offM;           // device: packed offset of each edge's M block
  const int64_t* offV;           // device [K]
  const int64_t* offEta;         // device [K]
  // complex parameters (realified state): the phase factor z_i = (w^T x + c)
  // + i (w2^T x + c2) of the stored state x, the phase cotangent, per-row
  // scratch for the current site, and the offsets of w, c, w2, c2 in the
  // realified gradient (device [K] each); cotp == nullptr: no phase term
  const T* w = nullptr;
  const T* c = nullptr;
  const T* w2 = nullptr;
  const T* c2 = nullptr;
  const double* cotp = nullptr;  // [Rpad]
  T* ab = nullptr;               // [Rpad][2]
  const int64_t* offW = nullptr;
  const int64_t* offC = nullptr;
  const int64_t* offW2 = nullptr;
  const int64_t* offC2 = nullptr;
  const T* tadd = nullptr;       // tensor term of the current site's candidates [Rpad][4][chip] (nullable)
};

// The tensor term's part of the adjoint sweep (host-side description; the
// row scratch is device memory of the current site)
template <typename T>
struct TnAdj {
  TnParams<T> P;                 // the forward's kernel layout
  const int* tq_host;            // [K] chi' of each site (0: no tensor term)
  const int* d_host;             // [K] in-degrees
  const int64_t* offTK_host;     // [K] packed offsets of K^(0..d)
  const int64_t* offTU_host;     // [K] packed offsets of U^s
  T* TT;                         // [Rpad][4][chip] tensor term of the candidates
  T* PJ;                         // [Rpad][3][16] projections
  T* QS;                         // [Rpad][4][16] core contractions
  T* DQ;                         // [Rpad][4][16]
  T* DP;                         // [Rpad][3][16]
};

// Map of a gradient over the realified parameters onto the packed complex
// layout (adjoint.hip): per site the offsets in both vectors (device).
struct CxMap {
  int K, chi, n_edges;           // chi: complex units (the realified state has 2 chi)
  const int* pptr;               // device [K+1]
  const int64_t* rM;             // realified: per edge [4][2chi][2chi]
  const int64_t* rV;             // [K] [4][2chi]
  const int64_t* rEta;           // [K] [2chi]
  const int64_t* rW;             // [K] [2chi] vector of Re z
  const int64_t* rC;             // [K]
  const int64_t* rW2;            // [K] [2chi] vector of Im z
  const int64_t* rC2;            // [K]
  const int64_t* cM;             // complex: per edge [4][chi][chi] pairs
  const int64_t* cV;             // [K] [4][chi] pairs
  const int64_t* cEta;           // [K] [chi]
  const int64_t* cW;             // [K] [chi] pairs
  const int64_t* cC;             // [K] one pair
  int64_t r_corr, c_corr, n_corr;// the real correlator block: offsets and length
};

// BF16 forward (psi_bf16.hip): same edge tables as PsiParams; FP32 vectors.
struct B16Params {
  int K, chi, chip, na, nb, W;   // W, slot, wsl, live: the ring as in PsiParams
  const int* pptr;               // [K+1] forward edges (never empty per site)
  const int* slot;               // [edges] ring slot read by each edge (W: a parentless site's zero edge)
  const int* wsl;                // [K]
  const uint64_t* live;          // [K+1]
  const uint16_t* A;             // BF16 A stream, per forward edge + one zero edge (runtime.cpp)
  const uint16_t* Alo = nullptr; // the same stream's lo parts (split form)
  const float* v;                // [K][4][chip]
  const float* eta;              // [K][chip]
  const float* w;                // [K][chip]
  const float* c;                // [K]
  bool folded;                   // operands carry sqrt(eta)
  bool d1 = false;               // every site has exactly one edge
};
// States of the BF16 forward's STORE / SEED modes (as PsiStates): carried
// states as BF16 with one power-of-two exponent per (site, row).
struct B16States {
  uint16_t* hs = nullptr;        // [K][ns][chip] BF16 carried state / 2^he
  uint16_t* hs_lo = nullptr;     // split form: the lo parts of hs
  int32_t* he = nullptr;         // [K][ns]
  float* pm = nullptr;           // [K+1][ns]
  int32_t* pe = nullptr;         // [K+1][ns]
  int8_t* pg = nullptr;          // [K+1][ns]
  int64_t ns = 0;
  const int32_t* perm = nullptr;
  const uint8_t* t0 = nullptr;
  const int32_t* owner = nullptr;
};

struct CorrParams {
  int K, nh;
  const double* b;   // [nh]
  const double* W;   // [nh][2K]
  const double* W1t = nullptr;   // W transposed [2K][nh]
  // Ising-RBM (ising != 0): the symmetric part of the quadratic couplings
  // S[P][Q][k] = (W2[k][P][Q] + W2[k][Q][P]) / 2
  int ising = 0;
  const double* S = nullptr;
  const float* S32 = nullptr;   // S rounded to FP32 (reduced-precision paths)
};

// Row list of one local-energy call (structure of arrays).
struct Rows {
  uint64_t* m;       // [R][2]
  double* coef;      // [R]
  int32_t* owner;    // [R]
  int64_t* rank;     // [R]   (-1 for the sample's own row)
  uint8_t* t0;       // [R]   first site where m differs from its sample (K when equal); may be null
  uint32_t* sec;     // [R]   c2 | state at c1 << 8 | c3 << 16 | state at c2 << 24 (next changed sites,
                     //       K when absent); may be null
};

// ---- launchers (enumerate.hip) ----------------------------------------
hipError_t launch_validate(const uint64_t* samples, int64_t N, int K, int na, int nb, int* bad,
                           hipStream_t st);
hipError_t launch_enum_count(const HamDev& H, const EnumGeom& G, const uint64_t* samples, int64_t N,
                             double eps, int qshift, uint64_t* masks, uint64_t* qpref, uint64_t* segq,
                             uint32_t* segd, hipStream_t st);
hipError_t launch_sample_scan(const EnumGeom& G, int64_t N, uint64_t* segq, uint32_t* segd,
                              uint64_t* Qn, int64_t* Dn, hipStream_t st);
hipError_t launch_draw(const HamDev& H, const EnumGeom& G, const uint64_t* samples, int64_t N,
                       double eps, int qshift, int n_eps, DrawKeys keys, const uint64_t* qpref,
                       const uint64_t* segq_off, const uint64_t* Qn, int32_t* urank, double* ucoef,
                       uint64_t* um, int64_t* Un, hipStream_t st);
hipError_t launch_row_counts(int64_t N, const int64_t* Dn, const int64_t* Un, int64_t* rowptr,
                             hipStream_t st);
hipError_t launch_fill(const HamDev& H, const EnumGeom& G, const uint64_t* samples, int64_t n0, int64_t n1,
                       const uint64_t* masks, const uint32_t* segd_off, const int64_t* rowptr,
                       int64_t row_base, const int64_t* Dn, const int64_t* Un, const int32_t* urank,
                       const double* ucoef, const uint64_t* um, int n_eps, Rows rows, hipStream_t st);
hipError_t launch_diag(const HamDev& H, const uint64_t* samples, int64_t N, double* hdiag,
                       hipStream_t st);
hipError_t launch_connected(const HamDev& H, const uint64_t* samples, int64_t N, uint64_t* m_out,
                            double* h_out, hipStream_t st);

// ---- launchers (amplitude.hip) -----------------------------------------
// hstore (nullable): carried states h_i^{s_i} of every row, [K][rpad][chip]
// Forward modes.  PLAIN: rows 0..R-1 from site 0.  STORE: as PLAIN, and for
// rows r < X.ns the carried state after every site goes to X.hs and, when
// X.pm is set, the log-product state (mantissa, exponent, sign) before every
// site and after the last to X.pm/pe/pg.  SEED: position p evaluates row
// X.perm[p]; positions are sorted by the row's first changed site X.t0[p],
// and each wavefront resumes at the site of its first position from the state
// that a STORE pass left for the row's sample X.owner[row].
// Sampling (psi.hip, sampling mode of the forward): particle p = p0 + row
// draws its local state at site i with the uniform of Philox4x32-10 counter
// (p lo, p hi, i, kSampleTag) and key (k0, k1); out receives its ONV.
constexpr uint32_t kSampleTag = 0x53414D50u;
struct SampleArgs {
  uint32_t k0 = 0, k1 = 0;
  int64_t p0 = 0;
  uint64_t* out = nullptr;       // [R][2]
};
template <typename T> struct PsiParams;
// PSI_NODE: SEED for the units of a node list (resumed from their samples)
// plus the compact store of nodes.hip.
enum { PSI_PLAIN = 0, PSI_STORE = 1, PSI_SEED = 2, PSI_NODE = 3 };
// what the amplitude kernels read of a node (one 32-byte record, a single
// cache line): log-product entries from off, carried-state slots from coff
// for the sites marked in need, the changed site c1 and the last resume site e1
struct alignas(32) NodeRec {
  int64_t off, coff;
  uint64_t need;
  int32_t c1, e1;
};
// a node's log-product state before a site (mantissa, power of two, sign) in
// one 16-byte store: the node pass writes them scattered, one per unit
template <typename T>
struct alignas(16) LogProd {
  T m;
  int32_t e, s;
};
static_assert(sizeof(LogProd<float>) == 16 && sizeof(LogProd<double>) == 16, "one 16-byte store per entry");
template <typename T>
struct PsiStates {
  T* hs = nullptr;               // [K][ns][chip] carried states
  T* pm = nullptr;               // [K+1][ns] product mantissa before site i
  int32_t* pe = nullptr;         // [K+1][ns] product exponent
  int8_t* pg = nullptr;          // [K+1][ns] sign
  T* pz = nullptr;               // complex parameters: [K+1][ns][2] phase-factor product before site i
  int64_t ns = 0;                // sample stride
  const int32_t* perm = nullptr; // SEED: [R] row of each position
  const uint8_t* t0 = nullptr;   // SEED: [R] first changed site of each position (ascending)
  const int32_t* owner = nullptr;// SEED: [rows] sample of each row
  // one level of shared prefixes (nodes.hip), per node u with record
  // nrec[u]: entry off + k holds the log-product state before site c1 + k
  // (k <= e1 - c1); the carried state after site s (c1 <= s < e1) is in slot
  // coff + popcount(need & bits below s), stored only where need has bit s
  T* nhs = nullptr;              // [slots][chip]
  LogProd<T>* nlp = nullptr;     // [entries]
  T* npz = nullptr;              // complex parameters: [entries][2]
  const NodeRec* nrec = nullptr; // [nodes]
  const int32_t* unode = nullptr;// SEED rows: [rows] node the row resumes from (-1: its sample)
};
// node list written by nodes.hip
struct NodeList {
  uint64_t* m;                   // [nodes][2] ONV: the sample with its rows' first (two) changes
  int32_t* owner;                // [nodes] sample
  uint8_t* c1;                   // [nodes] changed site
  uint8_t* e1;                   // [nodes] largest resume site of its rows
  int64_t* off;                  // [nodes] first storage entry (log-product states)
  uint64_t* need;                // [nodes] bit s: some row reads the carried state after site s
};
// capacities of one pass's node storage: nodes, log-product entries, and the
// carried-state slots the rows read at their own resume sites (the scan keeps
// whole samples in order while all three fit)
struct NodeCaps {
  int64_t nodes, entries, own_slots;
};
// whether nodes can be keyed by the first two changes (the pair table fits the
// LDS of a workgroup on the current device; else by the first change)
bool node_pairs(int K);
// slots beyond the rows' own reads that the wavefront starts can add: 64 K^2
int64_t slot_reserve(int K);
hipError_t launch_node_count(const uint8_t* t0, const uint32_t* sec, const uint64_t* samples, const int64_t* rowptr,
                             int64_t n0, int64_t n1, int64_t row_base, int K, int W, bool pair, int32_t* ncnt,
                             int64_t* nent, int64_t* nslt, hipStream_t st);
hipError_t launch_node_scan(int64_t ns, const NodeCaps& cap, const int32_t* ncnt, const int64_t* nent,
                            const int64_t* nslt, int64_t* nbase, int64_t* ebase, int64_t* totals, hipStream_t st);
hipError_t launch_node_assign(const uint8_t* t0, const uint32_t* sec, const uint64_t* samples,
                              const int64_t* rowptr, int64_t n0, int64_t n1, int64_t row_base, int K, int W,
                              bool pair, const int64_t* nbase, const int64_t* ebase, const NodeList& nl,
                              int32_t* row_node, uint8_t* row_site, hipStream_t st);
// need[row_node[perm[p]]] |= the sites below the row's wavefront start whose
// carried states the row pass reads from the node, for rows whose wavefront
// starts below their own resume site (rows sorted by resume site t0s; at most
// 64 rows per wavefront of the forward kernels)
hipError_t launch_node_need(const int32_t* perm, const uint8_t* t0s, int64_t R, int W, const int32_t* row_node,
                            const uint8_t* nc1, uint64_t* need, hipStream_t st);
// the records of the nn nodes of a pass.  compact: coff = sum over v < u of
// popcount(need[v]) (bsum: slot_blocks(nn) entries, total: 1); beyond cap
// slots every need and coff is zeroed and *overflow set.  Otherwise (the
// tensor-term kernels) a slot per entry: coff = off, need = every site >= c1.
int64_t slot_blocks(int64_t nn);
hipError_t launch_node_records(const NodeList& nl, int64_t nn, bool compact, int64_t cap, int64_t* bsum,
                               int64_t* total, NodeRec* rec, int* overflow, hipStream_t st);
// phs (complex parameters, PSI_PLAIN only): the phase of each row
hipError_t launch_psi_f64(const PsiParams<double>& P, const uint64_t* m, int64_t R, double* lphi,
                          int8_t* sphi, hipStream_t st, const PsiStates<double>& X = PsiStates<double>(),
                          int mode = PSI_PLAIN, double* phs = nullptr);
hipError_t launch_psi_f32(const PsiParams<float>& P, const uint64_t* m, int64_t R, double* lphi,
                          int8_t* sphi, hipStream_t st, const PsiStates<float>& X = PsiStates<float>(),
                          int mode = PSI_PLAIN, double* phs = nullptr);
hipError_t launch_sample_f64(const PsiParams<double>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                             const SampleArgs& SA);
hipError_t launch_sample_f32(const PsiParams<float>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                             const SampleArgs& SA);
// ---- unique ONVs with counts (unique.hip) ------------------------------
struct UniqueScratch {
  void* temp;                    // hipCUB temporary storage
  size_t temp_bytes;
  uint64_t *key_a, *key_b;       // [N]
  uint32_t *ord_a, *ord_b;       // [N]
  int32_t *flag, *pos;           // [N]
  int64_t* start;                // [N]
  int64_t* wsum;                 // [N], used with weights
};
hipError_t unique_temp_bytes(int64_t N, size_t* bytes);
// merges m [N][2] into unique ONVs (ascending high, low word), their counts
// (entries, or the sum of the entries' weights when weights is not null) and
// the lphi/sphi of a representative; *nu (device) = number of unique ONVs,
// at most cap written
hipError_t launch_unique(const uint64_t* m, const double* lphi, const int8_t* sphi, const int64_t* weights,
                         int64_t N, bool two_words, const UniqueScratch& w, int64_t cap, uint64_t* um, int64_t* ucnt,
                         double* ul, int8_t* us, int64_t* nu, hipStream_t st);
hipError_t launch_fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t st);
// ---- BDG-TensorRNN (tensor_rnn.hip) --------------------------------------
size_t tn_lds_bytes(int W, int rw, int precision);
// hs (nullable): store the carried state of every row r < ns and site for the adjoint
hipError_t launch_psi_tn_f64(const TnParams<double>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                             hipStream_t st, double* hs = nullptr, int64_t ns = 0);
hipError_t launch_psi_tn_f32(const TnParams<float>& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                             hipStream_t st, float* hs = nullptr, int64_t ns = 0);
// adjoint of the tensor term at site i (tensor_rnn.hip): stage 0 = the
// projections, core contraction and t^s of every row (into A.TT, added to the
// recomputed candidates), stage 1 = the cotangents of the parents' states and
// the gradient of K0, K_j, U into gpart
hipError_t launch_tn_bwd_site(const TnAdj<double>& A, const int* pidx, int i, int stage, int64_t Rpad,
                              const double* Hbuf, const double* Dc, double* dcarry, int rows_per_split, int nsplit,
                              double* gpart, int64_t n_params, hipStream_t st);
hipError_t launch_tn_bwd_site(const TnAdj<float>& A, const int* pidx, int i, int stage, int64_t Rpad,
                              const float* Hbuf, const float* Dc, float* dcarry, int rows_per_split, int nsplit,
                              double* gpart, int64_t n_params, hipStream_t st);
hipError_t launch_sample_tn_f64(const TnParams<double>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                                const SampleArgs& SA);
hipError_t launch_sample_tn_f32(const TnParams<float>& P, int64_t R, double* lphi, int8_t* sphi, hipStream_t st,
                                const SampleArgs& SA);
// ---- VMC step (vmc.hip) -------------------------------------------------
hipError_t launch_i64_to_f64(int64_t n, const int64_t* a, double* b, hipStream_t st);
// cot_n = 2 c_n (etnum_n - fsq_n E) / S with S = sum c fsq, E = sum c etnum / S;
// out (device double[2]) = {E, S}
hipError_t launch_vmc_cotangent(int64_t N, const double* c, const double* etnum, const double* fsq, double* cot,
                                double* out, hipStream_t st);
// complex parameters: also cotp_n = 2 c_n etnum_im_n / S
hipError_t launch_vmc_cotangent_cx(int64_t N, const double* c, const double* etnum, const double* etnum_im,
                                   const double* fsq, double* cot, double* cotp, double* out, hipStream_t st);
hipError_t launch_adamw(int64_t n, double* p, const double* g, double* m, double* v, int64_t t, double lr, double b1,
                        double b2, double eps, double wd, hipStream_t st);
hipError_t launch_sumsq(int64_t n, const double* g, double* out, hipStream_t st);
// eta >= 0 (Sec. 2.1): p[off[i] + u] = 0 where it is negative, i < K, u < chi
hipError_t launch_project_eta(int K, int chi, const int64_t* off, double* p, hipStream_t st);
// ---- static workspace of the allocation-free entry point (static_ws.hip) --
constexpr size_t kStaticWorkspaceBytes = size_t(NQS_STATIC_WORKSPACE_BYTES);
// look up the device address of this device's array (with `device` current), once per device
hipError_t static_workspace_setup(int device);
// that address (nullptr before the setup)
void* static_workspace(int device);
// ---- row order by first changed site (order.hip) ----------------------
// chunk of rows per block of the counting sort
constexpr int kOrderChunk = 16384;
inline int64_t order_blocks(int64_t R) { return (R + kOrderChunk - 1) / kOrderChunk; }
// Stable counting sort of rows 0..R-1 by their first changed site t0[r] in
// [0, K].  cnt: [blocks][K+1] int32 scratch; tot: [K+1] int64 bucket totals
// (device); perm: [R] rows in (t0, row) order; t0s: [R] t0 of each position.
hipError_t launch_order_t0(const uint8_t* t0, int64_t R, int K, int32_t* cnt, int64_t* tot, int32_t* perm,
                           uint8_t* t0s, hipStream_t st);
// The same in (t0, t1, row) order (t1[r] in [0, K]); tmp_perm: [2 R] int32,
// tmp_key: [2 R] bytes of scratch.
hipError_t launch_order_t0_t1(const uint8_t* t0, const uint8_t* t1, int64_t R, int K, int32_t* cnt, int64_t* tot,
                              int32_t* tmp_perm, uint8_t* tmp_key, int32_t* perm, uint8_t* t0s, hipStream_t st);
hipError_t launch_psi_bf16(const B16Params& P, const uint64_t* m, int64_t R, double* lphi, int8_t* sphi,
                           hipStream_t st, const B16States& X, int mode, bool split);
// theta[N][nh] of the samples; with the Ising-RBM also (when E is not null) the
// per-sample row-update table E[N][2K][nh] (see energy.hip), FP64 for
// precision NQS_F64, else FP32
hipError_t launch_corr_theta(const CorrParams& C, const uint64_t* samples, int64_t N, double* theta,
                             void* E, int precision, hipStream_t st);
hipError_t launch_corr_rows(const CorrParams& C, const uint64_t* m, const int32_t* owner,
                            const uint64_t* samples, const double* theta, const void* E, int64_t R,
                            int precision, double* lf, int8_t* sf, hipStream_t st);
hipError_t launch_corr_direct(const CorrParams& C, const uint64_t* m, int64_t R, double* lf, int8_t* sf,
                              hipStream_t st);
hipError_t launch_reduce(int64_t n0, int64_t n1, const int64_t* rowptr, int64_t row_base, const double* coef,
                         const double* lphi, const int8_t* sphi, const double* lf, const int8_t* sf,
                         const double* hdiag, double* eloc, double* etnum, double* logabs, int8_t* sign,
                         double* fsq, hipStream_t st);
// eloc_im, etnum_im (nullable): complex local energies; then the variance
// takes |E_loc - E|^2 and out[7] = sum c Im Etilde_num / sum c |f|^2
hipError_t launch_batch_sums(int64_t N, const double* counts, const double* eloc, const double* etnum,
                             const double* fsq, double* out /*[8]*/, hipStream_t st,
                             const double* eloc_im = nullptr, const double* etnum_im = nullptr);
hipError_t launch_gather_logpsi(int64_t N, const double* lphi, const int8_t* sphi, const double* lf,
                                const int8_t* sf, double* logabs, int8_t* sign, hipStream_t st);
// phases: the rows' phases of Phi (phs, nullable: 0 or pi by sphi) with the
// correlator's sign
hipError_t launch_reduce_cx(int64_t n0, int64_t n1, const int64_t* rowptr, int64_t row_base, const double* coef,
                            const double* lphi, const int8_t* sphi, const double* phs, const double* lf,
                            const int8_t* sf, const double* hdiag, double* eloc, double* eloc_im, double* etnum,
                            double* etnum_im, double* logabs, double* phase, double* fsq, hipStream_t st);
hipError_t launch_gather_logpsi_phase(int64_t N, const double* lphi, const int8_t* sphi, const double* phs,
                                      const double* lf, const int8_t* sf, double* logabs, double* phase,
                                      hipStream_t st);

// ---- launchers (adjoint.hip) -------------------------------------------
// tn (nullable): the tensor term's part of the sweep
hipError_t launch_bwd_sweep_f64(const AdjParams<double>& P, const uint64_t* m, int64_t R, int64_t Rpad,
                                const double* cot, const double* Hbuf, double* dcarry, double* Dc,
                                double* Eeta, int rows_per_split, int nsplit, double* gpart,
                                int64_t n_params, hipStream_t st, const TnAdj<double>* tn = nullptr);
hipError_t launch_bwd_sweep_f32(const AdjParams<float>& P, const uint64_t* m, int64_t R, int64_t Rpad,
                                const double* cot, const float* Hbuf, float* dcarry, float* Dc,
                                float* Eeta, int rows_per_split, int nsplit, double* gpart,
                                int64_t n_params, hipStream_t st, const TnAdj<float>* tn = nullptr);
hipError_t launch_corr_backward(const CorrParams& C, const uint64_t* m, int64_t R, const double* cot,
                                double* dth, int rows_per_split, int nsplit, int64_t offB, int64_t offW,
                                int64_t offW2, double* gpart, int64_t n_params, hipStream_t st);
hipError_t launch_sum_parts(int64_t n_params, int nsplit, const double* gpart, double* grad, hipStream_t st);
// grad (packed complex layout) += the realified gradient gr mapped through M
hipError_t launch_cx_grad_map(const CxMap& M, const double* gr, double* grad, hipStream_t st);

}  // namespace nqs
