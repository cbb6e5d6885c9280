/*
 * nqs.h — C ABI of the MI355X (gfx950) semi-stochastic local-energy library.
 *
 * The library evaluates, for a batch of sampled occupation-number vectors n,
 *
 *   E_loc(n) = sum_m H_nm Psi(m) / Psi(n)                (Sec. 2.1, Eq. (6))
 *
 * split into a deterministic part over |H_nm| >= eps (Sec. 2.4, Eq. (20)) and
 * a stochastic part that draws N_eps connected determinants with probability
 * proportional to |H_nm| among the rest (Sec. 2.4, Eqs. (21)-(22)).  Psi = f Phi
 * where Phi is a BDG-RNN / MPS-RNN amplitude (Sec. 2.1 Eq. (10), Sec. 2.2
 * Eq. (12) without the tensor term) with particle-number / S_z masking (Sec. 3,
 * Eqs. (23)-(24)) and f the optional cos-RBM correlator (Sec. 2.3, Eq. (15)).
 * It also returns the reweighted numerator of Sec. 2.3 Eq. (18), log|Psi| and
 * the vector-Jacobian product of log|Psi| used by the gradients of Eqs. (7)
 * and (19).
 *
 * Conventions
 *  - K spatial orbitals (K <= 64), spin orbital P = 2p + sigma (sigma 0 alpha,
 *    1 beta), interleaved as in Sec. 3.  An ONV is two uint64 words
 *    (little-endian 128-bit integer), bit P = occupation of spin orbital P.
 *  - |n> = prod_{P ascending} (a+_P)^{x_P} |vac>; fermionic signs follow.
 *  - Integrals: h[p*K+q] = h_pq and eri[((p*K+q)*K+r)*K+s] = (pq|rs) (chemist
 *    notation, real orbitals, 8-fold symmetric); <PQ|RS> = (pr|qs) for matching
 *    spins.  Row-major FP64 host arrays.
 *  - Graph: parents N(i) of site i as CSR (parent_ptr[K+1], parent_idx[]),
 *    every parent index lower than i, ascending within a site.
 *  - Packed FP64 parameters, per site i ascending: for each parent j (in
 *    parent_idx order) and local state s = 0..3 (s = n_alpha + 2 n_beta), the
 *    chi x chi matrix M_ij^s row-major (h_out[u] = sum_k M[u][k] h_in[k]);
 *    then v_i^s (4 x chi), eta_i (chi, >= 0), w_i (chi), c_i (1).  After all
 *    sites, when n_hidden > 0: b (n_hidden) then W (n_hidden x 2K row-major).
 *
 * Errors: every call returns an nqs_status; nothing else crosses the ABI.
 * nqs_last_error() returns a thread-local message describing the last
 * failure of a call made by the calling thread.
 *
 * Streams: device work is ordered on the hipStream_t passed in (0 = the null
 * stream).  Every call has completed its device work when it returns, unless
 * stated otherwise; the host waits on that stream (and only on it) at the
 * points each call lists.  nqs_eloc / nqs_eloc_complex wait
 *   1. after validating the samples (the result decides EINVAL),
 *   2. after enumeration, screening and draws, to read the row count of
 *      every sample (it sizes the row buffers and the passes),
 *   3. once per amplitude pass in FP64 / FP32 with resumed rows, to read the
 *      number of shared-prefix nodes of the pass (it sizes the node pass),
 *   4. at the end;
 * with a stats pointer also once per pass for the stage timers and the
 * per-site row totals.  nqs_ansatz_bind_params waits to copy the parameters
 * to the host, where they are laid out per precision.  Workspace blocks go
 * back to the context's pool behind the work queued on the call's stream
 * (an event recorded on it), on error paths too, so a block is never handed
 * to another call while a queued kernel may still use it.
 */
#ifndef NQS_H
#define NQS_H

#include <stdint.h>
#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int nqs_status;
enum {
  NQS_OK = 0,
  NQS_EINVAL = 1,       /* bad shape, bad argument, sample outside the sector */
  NQS_ENOMEM = 2,       /* device memory exhausted (or the allocation hook fired) */
  NQS_EDEVICE = 3,      /* a HIP runtime error; the message holds the HIP string */
  NQS_EUNSUPPORTED = 4, /* combination not implemented (e.g. chi > 64) */
  NQS_EBUSY = 5         /* serving: no request completed yet / queue full */
};

typedef enum {
  NQS_F64 = 0,   /* bond contractions in FP64 (the paper's precision, Sec. 3) */
  NQS_F32 = 1,   /* FP32 operands on MFMA, FP32 accumulate */
  NQS_BF16 = 2,  /* BF16 operands on MFMA, FP32 accumulate, per-row scaled hidden states */
  NQS_BF16X3 = 3 /* the same with every operand split into two BF16 parts (hi + lo) and three
                    MFMAs per product (hi.hi + hi.lo + lo.hi): relative errors near 2^-15 */
} nqs_precision;

typedef struct nqs_ctx nqs_ctx;
typedef struct nqs_instance nqs_instance;
typedef struct nqs_ansatz nqs_ansatz;

/* Options of one local-energy call (Sec. 2.4 hyperparameters and RNG keys). */
typedef struct {
  double eps;          /* deterministic cutoff: |H_nm| >= eps is summed exactly; eps >= 0 */
  int32_t n_eps;       /* number of i.i.d. draws from the remainder per sample; >= 0 */
  int32_t precision;   /* nqs_precision of the amplitude evaluation */
  uint64_t seed;       /* Philox4x32-10 key (low word, high word) */
  uint64_t stream_id;  /* third and fourth Philox counter words */
  int32_t sample_base; /* added to the sample index in the Philox counter */
  int32_t max_rows_per_pass; /* 0 = evaluate all amplitude rows at once; otherwise rows are
                                evaluated in passes over whole samples holding at most
                                max(max_rows_per_pass, 1 + n_conn + n_eps) rows, which bounds
                                the device memory of the call (nqs_eloc_workspace_bytes) */
  int32_t flags;       /* NQS_ELOC_* bits; 0 = defaults */
} nqs_eloc_opts;

/* nqs_eloc_opts.flags.  By default the FP64 and FP32 amplitude rows resume at
 * their first changed site from the state their sample reached there (the
 * conditionals of Eqs. (9)-(10) below that site see the sample's
 * occupations); the results are bit-identical to evaluating every row from
 * site 0, which this flag selects. */
#define NQS_ELOC_FULL_RECOMPUTE 1

/* Per-call statistics (host struct, filled when a non-NULL pointer is passed). */
typedef struct {
  int64_t n_samples;
  int64_t n_conn;        /* connected determinants per sample (same for all samples) */
  int64_t n_rows;        /* amplitude rows evaluated (samples + deterministic + unique drawn) */
  int64_t n_det_rows;    /* total |D_n| */
  int64_t n_draw_rows;   /* total unique drawn determinants */
  int64_t n_zero_amp;    /* samples with Psi(n) = 0 (their E_loc is NaN) */
  double sum_c;          /* sum of counts */
  double B;              /* sum c |f|^2 / sum c                       (Sec. 2.3) */
  double E;              /* sum c Etilde_num / sum c |f|^2           (Eq. (17)) */
  double var;            /* sum c |f|^2 (E_loc - E)^2 / sum c |f|^2 */
  double ms_enumerate, ms_draw, ms_rows, ms_amplitude, ms_reduce;  /* stage times (device events) */
  int64_t n_passes;      /* amplitude passes (see max_rows_per_pass) */
  int64_t n_site_rows;   /* per-site amplitude evaluations executed: sum over rows of the
                            sites computed (K per row without resumption), plus the
                            samples' own pass when rows resume */
  double ms_psi;         /* device time of the row amplitude kernel launches alone */
  double psi_flops;      /* their algorithmic flops: 8 chi^2 d_i per evaluated site i with
                            d_i parents (32 chi^2 d_i with complex parameters), plus for a
                            tensor-RNN site 2 (d chi chi' + 4 chi'^(d+1) + 4 chi chi') */
  double E_im;           /* nqs_eloc_complex: sum c Im Etilde_num / sum c |f|^2; else 0 */
} nqs_eloc_stats;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device`; all objects made from it live on
 * that device.  The context owns a pool of device workspaces. */
nqs_status nqs_ctx_create(int device, nqs_ctx** out);
/* Destroy a context.  No call may use an object created from it afterwards,
 * except nqs_instance_destroy and nqs_ansatz_destroy (they keep the device
 * and free their own memory, so garbage-collected handles may outlive the
 * context); a server must be destroyed before its context. */
nqs_status nqs_ctx_destroy(nqs_ctx* ctx);
/* Message of the calling thread's last failed call ("" if none). */
const char* nqs_last_error(void);
/* Library version string. */
const char* nqs_version(void);

/* ---- instance: the Hamiltonian of Sec. 2.1 Eq. (2) ------------------- */

/* Copy h (K*K) and eri (K^4) from host memory to the device and keep them
 * resident.  EINVAL if K < 1 or K > 64, n_alpha/n_beta outside [0,K], an
 * entry of h or eri or e_core not finite, h not symmetric or eri not 8-fold
 * symmetric within 1e-10 * max|eri| (values are replaced by their canonical
 * representative). */
nqs_status nqs_instance_create(nqs_ctx* ctx, int K, int n_alpha, int n_beta, const double* h1,
                               const double* eri, double e_core, nqs_instance** out);
nqs_status nqs_instance_destroy(nqs_instance* inst);
/* Number of S_z-conserving singles + doubles of any ONV of the sector. */
int64_t nqs_instance_n_conn(const nqs_instance* inst);

/* Hamiltonian engine (Sec. 2.4, Slater-Condon rules): for each of the N
 * samples (device, [N][2] uint64), all n_conn connected determinants in the
 * canonical order (alpha singles, beta singles, alpha-alpha doubles,
 * beta-beta doubles, alpha-beta doubles; holes outer, particles inner,
 * ascending orbitals, pairs lexicographic) with H_mn, plus H_nn.
 * m_out: device [N][n_conn][2] uint64; h_out: device [N][n_conn] double;
 * hdiag_out: device [N] double (any may be NULL).  EINVAL for a sample outside
 * the (n_alpha, n_beta) sector. */
nqs_status nqs_connected(nqs_ctx* ctx, const nqs_instance* inst, const uint64_t* samples, int64_t N,
                         uint64_t* m_out, double* h_out, double* hdiag_out, hipStream_t stream);

/* ---- ansatz: BDG-RNN / MPS-RNN (Sec. 2.1-2.2) x RBM correlator (Sec. 2.3) */

/* Correlators of Sec. 2.3: f(n) = prod_k cos(theta_k(n)) with
 * theta_k = b_k + sum_P W_kP x_P (cos-RBM, Eq. (15)), or with the Ising-RBM
 * term (1/2) sum_{P,Q} W2_kPQ x_P x_Q added (Eq. (16), a full 2K x 2K matrix
 * per hidden unit, all ordered pairs and the diagonal). */
#define NQS_CORR_COS_RBM 0
#define NQS_CORR_ISING_RBM 1
/* Flag added to the correlator kind: BDG-TensorRNN (Sec. 2.2, Eqs. (12)-(13)),
 * the tensor term in Tucker form at every site with d = 2 or 3 parents,
 * chi' = ceil(chi^(2/(d+1))); its parameters follow everything else: per such
 * site ascending, K^(0) (output mode) and K^(1..d) (one per parent, ascending),
 * each chi x chi' row-major, then U^s for s = 0..3, each chi'^(d+1) with index
 * order [i', a_1, .., a_d].  Forward, local energy, sampling, the adjoint
 * (nqs_logpsi_vjp, the factor matrices and cores included) and the VMC step
 * run in FP64 and FP32 (rows evaluated from site 0; NQS_EUNSUPPORTED for BF16,
 * for a site with more than 3 parents, and when a thread's ring of
 * W x ceil4(chi) states does not fit the LDS). */
#define NQS_ANSATZ_TENSOR 0x10
/* Flag added to the correlator kind: complex parameters (Sec. 2.1, the
 * MPS-RNN over C^chi): M, v, w, c complex, eta real and >= 0; the conditional
 * P^s = h^dagger eta h and the phase of Phi(n) = sum_i arg(w_i^T h_i + c_i)
 * (no conjugation of w; arg 0 = 0).  Packed layout per site as for real
 * parameters, with every complex entry stored as (re, im): M (per parent,
 * 4 x chi x chi pairs), v (4 x chi pairs), eta (chi reals), w (chi pairs),
 * c (one pair); the correlator block after the sites stays real (its sign
 * adds 0 or pi to the phase).  chi <= 32.  The amplitudes run in FP64 and
 * FP32 (the realified form: a real 2chi state with block matrices
 * [[Re M, -Im M], [Im M, Re M]] on the same MFMA kernels, the phase factors
 * multiplied per row and carried with the resumed rows' prefix states);
 * NQS_EUNSUPPORTED for BF16; not combined with NQS_ANSATZ_TENSOR.  Signs are replaced by phases:
 * nqs_logpsi, nqs_eloc and the sign output of nqs_sample refuse a complex
 * ansatz (EINVAL); use nqs_logpsi_phase, nqs_eloc_complex and
 * nqs_logpsi_vjp_phase. */
#define NQS_ANSATZ_COMPLEX 0x20

/* Describe the ansatz: K sites, electron counts of the sector (they define the
 * mask of Sec. 3), bond dimension chi (1..64), parent CSR (host arrays),
 * n_hidden correlator units (0 = no correlator) and the variant: the
 * correlator kind, optionally | NQS_ANSATZ_TENSOR or | NQS_ANSATZ_COMPLEX.
 * Packed parameters: the BDG-RNN block, then b (n_hidden), W (n_hidden x 2K),
 * and for the Ising-RBM W2 (n_hidden x 2K x 2K, row-major).  EINVAL for a
 * malformed graph or an unknown correlator.  The Ising-RBM local energy keeps
 * a table of N x 2K x n_hidden doubles (8 N 2K n_hidden bytes of workspace). */
nqs_status nqs_ansatz_create(nqs_ctx* ctx, int K, int n_alpha, int n_beta, int chi,
                             const int32_t* parent_ptr, const int32_t* parent_idx, int n_hidden,
                             int32_t variant, nqs_ansatz** out);
nqs_status nqs_ansatz_destroy(nqs_ansatz* ans);
/* Length of the packed parameter vector. */
int64_t nqs_ansatz_n_params(const nqs_ansatz* ans);
/* Copy the packed FP64 parameters (device pointer, nqs_ansatz_n_params
 * doubles) into the library's kernel layouts for every precision.  The caller's
 * buffer may be freed or changed afterwards; call again after an update.
 * EINVAL if some eta < 0 or NaN (nothing changes then).  A failure after the
 * old layouts were released (device memory) leaves the ansatz unbound: every
 * call refuses it with EINVAL until a bind succeeds. */
nqs_status nqs_ansatz_bind_params(nqs_ansatz* ans, const double* params, hipStream_t stream);

/* log|Psi(n)| (device double[N]) and sign Psi(n) (device int8[N]) of N samples.
 * A sample outside the sector is EINVAL; Psi(n) = 0 gives -inf and sign 0. */
nqs_status nqs_logpsi(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                      int32_t precision, double* logabs, int8_t* sign, hipStream_t stream);

/* log|Psi(n)| and the phase of Psi(n) in [-pi, pi] (device double[N] each,
 * either may be NULL) for any ansatz: with real parameters the phase is 0 or
 * pi by the sign.  precision NQS_F64 or NQS_F32 for a complex ansatz (the
 * phase factors are multiplied in that precision, the final arg in FP64).  A
 * sample outside the sector is EINVAL; Psi(n) = 0 gives -inf and phase 0. */
nqs_status nqs_logpsi_phase(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                            int32_t precision, double* logabs, double* phase, hipStream_t stream);

/* Vector-Jacobian product of log|Psi| (Eqs. (7), (19)): grad[k] +=
 * sum_n cot[n] d log|Psi(n)| / d theta_k over the packed parameters (device
 * double[n_params], accumulated, not overwritten).  cot: device double[N].
 * precision NQS_F64 or NQS_F32 (the FP32 path accumulates in FP32 per block and
 * in FP64 across blocks). */
nqs_status nqs_logpsi_vjp(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                          const double* cot, int32_t precision, double* grad, hipStream_t stream);

/* The same with the phase: grad[k] += sum_n (cot_abs[n] d log|Psi(n)| +
 * cot_phase[n] d phase(n)) / d theta_k, where for a complex ansatz theta runs
 * over the real and imaginary parts of the packed parameters (the gradient
 * of a real loss, entry by entry of the packed vector).  With real
 * parameters the phase is locally constant and cot_phase is ignored;
 * cot_phase may be NULL (= 0).  The gradient of the energy over complex
 * parameters, 2 Re <(E_loc - E)^* d ln Psi>, takes cot_abs from Re E_loc and
 * cot_phase from Im E_loc (see nqs_vmc_step). */
nqs_status nqs_logpsi_vjp_phase(nqs_ctx* ctx, const nqs_ansatz* ans, const uint64_t* samples, int64_t N,
                                const double* cot_abs, const double* cot_phase, int32_t precision, double* grad,
                                hipStream_t stream);

/* ---- sampling (Sec. 2.1 autoregressive sampling, masks of Sec. 3) ------ */

/* Exact autoregressive draws from Phi^2 (the BDG-RNN / MPS-RNN modulus of
 * Eqs. (9)-(10); the correlator is left to reweighting, Sec. 2.3), with the
 * particle-number / S_z mask of Eqs. (23)-(24).  Draw t (t = draw_base ..
 * draw_base + n_draws - 1) takes site i's local state s from the masked
 * conditionals p_s (s = 0..3, n_alpha + 2 n_beta): with the uniform u of
 * words 0 and 1 of Philox4x32-10 at counter (t lo, t hi, i, 0x53414D50) under
 * key (seed lo, seed hi) as a 53-bit fraction, the first s whose running sum of
 * the allowed p exceeds u * sum p (the last allowed s if none).  Draws are
 * independent of each other and of how they are split into calls.  Equal
 * draws are merged: samples (device uint64[cap][2], ascending by high then
 * low word), counts (device int64[cap]), logabs (device double[cap],
 * log|Phi|, nullable), sign (device int8[cap], sign of Phi, nullable);
 * *n_unique (host) receives the number of unique draws, of which at most cap
 * are written.  precision NQS_F64 or NQS_F32 (the conditionals' precision).
 * Memory: the draws run in passes of at most max_draws_per_pass (0 = one
 * pass, at most 2^31 - 1 draws); each pass is merged with the unique draws of
 * the passes before it, so the workspace is about 25 B per draw of a pass plus
 * about 150 B per unique draw, independent of n_draws.  The result does not
 * depend on the pass size.  NQS_EUNSUPPORTED for BF16 or a pass (plus the
 * unique draws so far) above 2^31 - 1; NQS_ENOMEM when the pool limit is hit.
 * Synchronises `stream`. */
nqs_status nqs_sample(nqs_ctx* ctx, const nqs_ansatz* ans, int64_t n_draws, uint64_t seed, int64_t draw_base,
                      int32_t precision, int64_t max_draws_per_pass, int64_t cap, uint64_t* samples,
                      int64_t* counts, double* logabs, int8_t* sign, int64_t* n_unique, hipStream_t stream);

/* ---- local energy (Sec. 2.4) ------------------------------------------ */

/* Semi-stochastic local energies of N samples (device [N][2] uint64).
 * counts: device double[N] weights of the batch sums (NULL = all 1).
 * Outputs (device, length N, any may be NULL):
 *   eloc  = H_nn + sum_{D_n} H_nm r_m + (1/N_eps) sum_k H_nm_k / P(m_k) r_mk,
 *           r = Psi(m)/Psi(n)                                   (Eq. (22))
 *   etnum = f_n sum_m H_nm f_m Phi(m)/Phi(n) = |f_n|^2 E_loc(n)  (numerator of Eq. (18))
 *   logabs = log|Psi(n)|, sign = sign Psi(n), fsq = |f_n|^2.
 * The proposal is P(m) = q_m / sum q with q_m = ceil(|H_nm| 2^(40-e)),
 * eps = f 2^e, f in [0.5,1); draw k of sample s uses Philox4x32-10 with key
 * (seed lo, seed hi) and counter (sample_base + s, k, stream_id lo, hi).
 * stats (host, nullable) receives the batch sums of Sec. 2.3.  Host waits on
 * `stream`: see "Streams" above.  Combinations the amplitude kernels do not
 * run (BF16 with complex parameters or the tensor term) fail with
 * NQS_EUNSUPPORTED before any work is queued. */
nqs_status nqs_eloc(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans,
                    const uint64_t* samples, const double* counts, int64_t N,
                    const nqs_eloc_opts* opts, double* eloc, double* etnum, double* logabs,
                    int8_t* sign, double* fsq, nqs_eloc_stats* stats, hipStream_t stream);

/* The same local energies for an ansatz with complex parameters (or any
 * ansatz: real parameters give zero imaginary parts and phases 0 or pi):
 * Psi(m)/Psi(n) = e^{log|Psi(m)| - log|Psi(n)|} e^{i (phase(m) - phase(n))}, so
 * E_loc and Etilde_num are complex (eloc_re/eloc_im, etnum_re/etnum_im); phase
 * = the phase of Psi(n) in [-pi, pi] replaces the sign.  All outputs device
 * double[N], nullable.  The batch sums use Re Etilde_num for E, |E_loc - E|^2
 * for the variance, and stats->E_im receives sum c Im Etilde_num / sum c |f|^2
 * (zero in expectation, H being Hermitian).  Complex amplitudes run in FP64
 * or FP32; rows resume as in nqs_eloc, bit-identical to NQS_ELOC_FULL_RECOMPUTE. */
nqs_status nqs_eloc_complex(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans,
                            const uint64_t* samples, const double* counts, int64_t N,
                            const nqs_eloc_opts* opts, double* eloc_re, double* eloc_im, double* etnum_re,
                            double* etnum_im, double* logabs, double* phase, double* fsq,
                            nqs_eloc_stats* stats, hipStream_t stream);

/* The amplitude rows of the same computation, for inspection: per sample
 * its own ONV (rank -1, coefficient 0), the deterministic set in canonical
 * rank order (coefficient H_nm) and the unique drawn determinants in rank
 * order (coefficient multiplicity * H_nm Q / (N_eps q_m)).  row_ptr: device
 * int64[N+1]; n_det: device int64[N]; Q: device uint64[N] (remainder weight
 * sum); rank: device int64[cap]; coef: device double[cap]; m: device
 * uint64[cap][2].  *n_rows (host) receives the total; rows beyond cap are not
 * written. */
nqs_status nqs_rows(nqs_ctx* ctx, const nqs_instance* inst, const uint64_t* samples, int64_t N,
                    const nqs_eloc_opts* opts, int64_t cap, int64_t* row_ptr, int64_t* n_det,
                    uint64_t* Q, int64_t* rank, double* coef, uint64_t* m, int64_t* n_rows,
                    hipStream_t stream);

/* Device bytes an nqs_eloc call of this shape takes from the context's pool
 * at most.  With opts->max_rows_per_pass > 0 the bound holds for any sample
 * data; otherwise pass the number of amplitude rows the call will evaluate
 * (n_rows; 0 gives the row-independent part).  Used for admission by
 * footprint in the serving loop. */
nqs_status nqs_eloc_workspace_bytes(const nqs_instance* inst, const nqs_ansatz* ans, int64_t N,
                                    const nqs_eloc_opts* opts, int64_t n_rows, size_t* bytes);

/* ---- allocation-free local energies ------------------------------------ */

/* Bytes of the static device workspace of nqs_eloc_noalloc: one array per GPU,
 * in the library's code object, held from the first context created on that
 * GPU until the process ends. */
#define NQS_STATIC_WORKSPACE_BYTES (256u << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid it.
 * The same computation, arguments and results as nqs_eloc (bit for bit),
 * without the stats pointer, with every workspace block taken from the static
 * array above instead of the context's pool: no hipMalloc, hipFree or other
 * allocating call is made.  NQS_ENOMEM with a message when the call needs more
 * than NQS_STATIC_WORKSPACE_BYTES; with opts->max_rows_per_pass > 0 a call
 * whose nqs_eloc_workspace_bytes is at most that size always fits.  Every
 * call on a GPU shares that GPU's array, which keeps the last call's contents
 * (the kernels write what they read before reading it); calls that overlap on
 * one GPU (any context, thread or stream) race on it, so the caller must
 * serialise them.  On an error after work was queued the call waits for
 * `stream` before returning.  Host waits otherwise as nqs_eloc. */
nqs_status nqs_eloc_noalloc(nqs_ctx* ctx, const nqs_instance* inst, const nqs_ansatz* ans,
                            const uint64_t* samples, const double* counts, int64_t N,
                            const nqs_eloc_opts* opts, double* eloc, double* etnum, double* logabs,
                            int8_t* sign, double* fsq, hipStream_t stream);

/* ---- one VMC step (Sec. 2.1 Eq. (7), Sec. 2.3 Eq. (19), AdamW of Sec. 3) - */

typedef struct {
  int64_t n_draws;            /* exact draws from Phi^2 in this step (>= 1) */
  uint64_t sample_seed;       /* sampler key (see nqs_sample) */
  int64_t draw_base;          /* index of the step's first draw, e.g. step * n_draws */
  int64_t max_draws_per_pass; /* sampler passes (0 = one pass) */
  nqs_eloc_opts eloc;         /* local-energy options; eloc.precision NQS_F64 also selects FP64
                                 sampling and adjoint, anything else FP32 for both */
  double lr, beta1, beta2, adam_eps, weight_decay;   /* AdamW (decoupled weight decay) */
  int64_t step;               /* AdamW step number t >= 1 (bias corrections 1 - beta^t) */
} nqs_vmc_opts;

typedef struct {
  int64_t n_unique;           /* unique samples of the step */
  double E, var, B;           /* reweighted energy, variance and <|f|^2> of the step's samples */
  double grad_norm;           /* Euclidean norm of the gradient */
  double ms_sample, ms_eloc, ms_grad, ms_update;   /* host wall time of the four stages */
} nqs_vmc_stats;

/* One variational step: draw n_draws samples from Phi^2
 * (nqs_sample), merge them into unique samples with counts, evaluate the
 * semi-stochastic local energies weighted by the counts (nqs_eloc), form the
 * reweighted gradient of Eq. (19),
 *   g = sum_n cot_n d ln|Psi(n)|/d theta,  cot_n = 2 c_n (Etilde_num(n) - |f_n|^2 E) / sum c |f|^2
 * (for f = 1 the plain VMC gradient of Eq. (7)), through nqs_logpsi_vjp, apply
 * one AdamW update to params (device double[n_params], in place) with the
 * moment estimates adam_m, adam_v (device, in place, zero before the first
 * step), project eta onto eta >= 0 (negative entries become 0: the
 * constraint of Sec. 2.1, a projected gradient step), and re-bind the ansatz
 * to the new parameters.  grad (device
 * double[n_params], nullable) receives g.  With complex parameters the
 * local energies come from nqs_eloc_complex and the gradient over the real
 * and imaginary parts is 2 Re <(E_loc - E)^* d ln Psi> reweighted as above:
 * cot_abs_n = 2 c_n (Re Etilde_num(n) - |f_n|^2 E) / sum c |f|^2 and
 * cot_phase_n = 2 c_n Im Etilde_num(n) / sum c |f|^2 through
 * nqs_logpsi_vjp_phase; AdamW treats every real entry of the packed vector as
 * one parameter.  Synchronises `stream`. */
nqs_status nqs_vmc_step(nqs_ctx* ctx, const nqs_instance* inst, nqs_ansatz* ans, const nqs_vmc_opts* opts,
                        double* params, double* adam_m, double* adam_v, double* grad, nqs_vmc_stats* stats,
                        hipStream_t stream);

/* ---- serving: continuous batching of local-energy requests ------------- */

typedef struct nqs_server nqs_server;

/* One local-energy request.  samples and the outputs are caller-owned device
 * buffers that must stay valid until the request's completion is returned;
 * inst/ans must outlive it too. */
typedef struct {
  const nqs_instance* inst;
  const nqs_ansatz* ans;
  const uint64_t* samples;   /* device [N][2] */
  int64_t N;
  nqs_eloc_opts opts;        /* opts.max_rows_per_pass = 0: the server's default */
  double* eloc;              /* device outputs as in nqs_eloc (nullable) */
  double* etnum;
  double* logabs;
  int8_t* sign;
  double* fsq;
  double t_arrival;          /* host monotonic seconds (nqs_monotonic_seconds); 0 = now */
  uint64_t user_tag;
} nqs_request;

typedef struct {
  int64_t ticket;
  uint64_t user_tag;
  nqs_status status;         /* the nqs_eloc status of the request */
  int32_t pad;
  double t_submit;           /* arrival (host monotonic seconds) */
  double t_start;            /* admission to a slot */
  double t_end;              /* completion; latency = t_end - t_submit */
  size_t footprint;          /* device bytes reserved for the request */
  nqs_eloc_stats stats;
  char message[256];         /* error message when status != NQS_OK */
} nqs_completion;

typedef struct {
  size_t budget, reserved, peak_reserved;
  int32_t in_flight, peak_in_flight;
  int64_t queued, skips;
} nqs_serve_status;

/* Host monotonic clock used for arrival and completion times (seconds). */
double nqs_monotonic_seconds(void);
/* Device of a context. */
int nqs_ctx_device(const nqs_ctx* ctx);

/* Start a server on ctx with n_slots concurrent requests (one device stream
 * each, 1..64) and a device-memory budget in bytes for all admitted requests;
 * the context's pool is capped at the budget while the server lives.
 * max_rows_per_pass (> 0) bounds the amplitude rows held per pass and hence
 * each request's footprint (see nqs_eloc_opts). */
nqs_status nqs_serve_create(nqs_ctx* ctx, int n_slots, size_t budget_bytes, int32_t max_rows_per_pass,
                            nqs_server** out);
/* Finish every queued and running request, then stop (completions not yet
 * polled are dropped). */
nqs_status nqs_serve_destroy(nqs_server* srv);
/* Queue a request; *ticket identifies its completion.  A request is admitted
 * when a slot is free and its footprint fits the unreserved budget (FIFO; a
 * later request that fits may go ahead of a head that does not, at most 8
 * times per head).  NQS_ENOMEM if its footprint exceeds the whole budget. */
nqs_status nqs_serve_submit(nqs_server* srv, const nqs_request* req, int64_t* ticket);
/* Device bytes the server would reserve for req. */
nqs_status nqs_serve_footprint(nqs_server* srv, const nqs_request* req, size_t* bytes);
/* Next completion, without blocking (NQS_EBUSY if none) or waiting up to
 * timeout_s seconds (NQS_EBUSY on timeout). */
nqs_status nqs_serve_poll(nqs_server* srv, nqs_completion* out);
nqs_status nqs_serve_wait(nqs_server* srv, double timeout_s, nqs_completion* out);
/* Budget, reserved bytes (current and peak), slots in use (current and
 * peak), queue length and skip-ahead count. */
nqs_status nqs_serve_info(nqs_server* srv, nqs_serve_status* out);

/* ---- test hooks --------------------------------------------------------- */

/* Make the k-th subsequent workspace allocation of this context fail with
 * NQS_ENOMEM (k >= 1; 0 disables).  For failure-handling tests. */
nqs_status nqs_ctx_fail_alloc_at(nqs_ctx* ctx, int64_t k);
/* Scale the node storage capacities of this context's later local-energy
 * calls by scale (0 < scale <= 1; 1 restores them; NQS_EINVAL otherwise):
 * whole samples past a capacity get no nodes and their rows resume at their
 * first changed site, with the same results.  For tests of that path. */
nqs_status nqs_ctx_set_node_capacity(nqs_ctx* ctx, double scale);
/* Bytes currently held by the context's workspace pool (in use, cached). */
nqs_status nqs_ctx_pool_bytes(const nqs_ctx* ctx, size_t* in_use, size_t* cached);
/* High-water mark of the pool's in-use bytes; reset != 0 restarts it at the
 * current in-use value. */
nqs_status nqs_ctx_pool_peak(nqs_ctx* ctx, size_t* peak, int reset);
/* Cap the pool's device memory (in use + cached, bytes; 0 = no cap).  Cached
 * blocks are released to stay under the cap; an allocation that cannot fit
 * fails with NQS_ENOMEM. */
nqs_status nqs_ctx_set_pool_limit(nqs_ctx* ctx, size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* NQS_H */
