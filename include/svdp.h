/*
 * svdp -- differentiable SVD via polar decomposition on AMD Instinct MI355X
 * (gfx950).  C ABI.
 *
 * Method ("Fast Differentiable SVD on GPU via Polar Decomposition"):
 *   forward  (Algorithm 1): normalise A (Algorithm 3), compute the polar
 *            factor W by the CANS polynomial iteration (chains of batched
 *            GEMMs), H = sym(W^T A), eigendecomposition H = V Sigma V^T,
 *            U = W V, rank-deficiency test on the column norms of U;
 *   backward (Algorithm 4, and Algorithm 2 for the polar factors): the
 *            regularised adjoint, a Sylvester solve in the eigenbasis of H.
 *
 * Conventions for every entry point:
 *   - Matrices are dense FP32, row-major, batched: matrix b of an argument X
 *     starts at X + b * sX, and entry (i, j) is X[b * sX + i * ldX + j]
 *     (ld >= number of columns).  Vectors (S, dS) use only a batch stride.
 *   - All array pointers are DEVICE pointers owned by the caller, except
 *     where a comment says host.  The library allocates no device memory per
 *     call: scratch comes from the caller's workspace `ws` of `ws_bytes`
 *     bytes, sized by svdp_workspace_size() (alignment 256 bytes).
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; null =
 *     the default stream).  Calls return after enqueueing: the iteration
 *     control of CANS, of the bounded schedule and refinement, of the Jacobi
 *     sweeps and of the eigensolver restarts runs on the device (fixed
 *     budgets of launches whose workgroups skip converged matrices).  Three
 *     forward steps read device values back, which synchronises `stream`:
 *     the bounded paths' fallback test (learned / user bounds), the QR step
 *     of Algorithm 1 when it runs blocked (n > 512), and the EVD step of a
 *     single FP32 matrix from n = 2048, which runs by the divide and conquer
 *     of svdp_eigh_dc (two reads per split); svdp_host_syncs() counts them.
 *     That EVD route also enlarges svd_polar_fwd's workspace by the
 *     divide and conquer's (SVDP_OP_EIGH_DC's for batch 1).
 *   - Errors: arguments are checked before anything is launched; a non-OK
 *     status means no work was enqueued, except SVDP_ERR_HIP, which reports
 *     a failed launch or copy (svdp_last_error() gives the HIP message).
 *     Numerical trouble never fails a call: it is reported per matrix in
 *     `info` (svdp_info flags).
 *   - A null upstream gradient (dU, dS, dV, dW, dH) means zero.
 */
#ifndef SVDP_H
#define SVDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SVDP_OK = 0,
  SVDP_ERR_INVALID_ARG = 1, /* null pointer, bad precision/bound/op, ld too small */
  SVDP_ERR_SHAPE = 2,       /* m < n, n < 1, batch < 0 or > 65535, n > 8192, m*n > 2^31 */
  SVDP_ERR_WORKSPACE = 3,   /* ws_bytes below svdp_workspace_size() */
  SVDP_ERR_HIP = 4,         /* a HIP launch or copy failed */
  SVDP_ERR_NO_MODEL = 5     /* learned bounds requested, no model loaded */
} svdp_status;

/* arithmetic of the CANS polar iteration */
typedef enum {
  SVDP_PREC_FP32 = 0, /* FP32 GEMMs on FP32 MFMA throughout */
  SVDP_PREC_BF16 = 1  /* BF16 MFMA (FP32 accumulate), then FP32 refinement steps */
} svdp_precision;

/* how the spectral interval of A is bounded before CANS */
typedef enum {
  SVDP_BOUND_CONSERVATIVE = 0, /* sqrt(|A|_1 |A|_inf) scale + delta preprocessing */
  SVDP_BOUND_LEARNED = 1,      /* sketch features -> MLP -> [sigma_min, sigma_max] */
  SVDP_BOUND_USER = 2          /* caller's [sigma_min, sigma_max] per matrix */
} svdp_bound;

/* Iteration polynomial of the conservative FP32 path (the appendix's
 * ablation of polar iterations built on matrix products). */
typedef enum {
  SVDP_POLY_CANS3 = 0, /* interval-optimal odd cubic (CANS), the method's default */
  SVDP_POLY_NS = 1,    /* classical Newton-Schulz 1.5 x - 0.5 x^3, no preprocessing */
  SVDP_POLY_CANS5 = 2, /* interval-optimal odd quintic (Remez exchange): three products
                          per step (X^T X, G G, X P), with its own preprocessing */
  SVDP_POLY_PE = 3     /* Polar Express (cited by the paper's ablation of polar
                          iterations): X0 = A / |A|_F, per-step minimax odd quintics on the
                          interval recursion from [pe_lo, 1], the cushioned interval
                          [max(l, u / 10), u], the input divided by 1.01 on every step but
                          the last; a fixed number of steps (svdp_pe_table), no stop test */
} svdp_poly;

/* per-matrix result flags (svdp_info.flags) */
#define SVDP_FLAG_NOT_CONVERGED 1        /* CANS stopped at max_iters above tol */
#define SVDP_FLAG_FALLBACK_USED 2        /* learned/user bound failed; conservative CANS rerun */
#define SVDP_FLAG_NEG_EIGENVALUE 4       /* H had an eigenvalue below -1e-4 max|lambda| */
#define SVDP_FLAG_RANK_DEFICIENT 8       /* some | |U_i| - 1 | > eps_qr; U was orthogonalised by QR
                                            (Algorithm 1), zero columns completed */
#define SVDP_FLAG_NONFINITE 16           /* non-finite input or result */
#define SVDP_FLAG_EIGH_NOT_CONVERGED 32  /* Jacobi hit max_sweeps */

typedef struct {
  int64_t batch, m, n;     /* m >= n >= 1 */
  int32_t precision;       /* svdp_precision */
  int32_t bound;           /* svdp_bound */
  int32_t max_iters;       /* CANS step cap, preprocessing included (50) */
  int32_t pre_iters;       /* conservative preprocessing steps (2) */
  int32_t refine_steps;    /* bounded paths: FP32 refinement steps taken unconditionally (2); the
                              refinement then continues per matrix until the relative change is
                              <= tol, for at most refine_steps + 8 steps, else NOT_CONVERGED and
                              the conservative fallback */
  int32_t max_sweeps;      /* Jacobi sweep budget (16): launched whatever the convergence */
  int32_t inner_sweeps;    /* repetitions of a block step's scalar rounds per 32 x 32 Jacobi
                              subproblem (1) */
  int32_t fp64_sweeps;     /* final Jacobi sweeps with FP64 subproblem solves, and the sweeps of
                              each restart (1) */
  double delta;            /* CANS preprocessing target [1-delta, 1+delta] (0.99) */
  double tol;              /* CANS stop: |X_k+1 - X_k|_F <= tol |X_k+1|_F (1e-5) */
  double eps_qr;           /* column-norm tolerance of U (1e-5) */
  double bf16_handoff;     /* BF16 phase ends when the interval error <= this (1e-2) */
  double refine_tol;       /* bounded paths fall back when |W^T W - I|_F / sqrt(n) after the
                              refinement exceeds this (1e-2) */
  double jacobi_tol;       /* Jacobi stops after a sweep whose largest rotated |h_pq| is
                              <= jacobi_tol sqrt(|h_pp h_qq|); by quadratic convergence that
                              sweep leaves about jacobi_tol^2 and the final FP64 sweep about
                              its square; tightly clustered spectra need the margin (3e-3) */
  double jacobi_abs;       /* entries below jacobi_abs |H|_F are ignored by that test (1e-9) */
  double bf16_from;        /* bounded paths: FP32 steps until the interval's lower end
                              reaches this value, BF16 steps after it (0.2).  BF16 rounding
                              while a singular value is still small rotates its singular
                              vectors and moves the small singular values; the BF16
                              correction (bf16_correct) removes that to first order.  With
                              it, on 256 x 512^2 with sigma in [1e-3, 1], the largest
                              per-value relative sigma error against the FP32 path is 1e-4
                              from 0.5 down to 0.2 and 2e-4 at 0.1; at 0.01 it is 2e-2.
                              Below 0.1 the column-norm test starts flagging (eps_qr) */
  double eps_K, eps_R, eps_T; /* backward regularisers (absolute, units of sigma^2):
                              K_ij = (s_i - s_j)/((s_i - s_j)^2 + eps_K),
                              R = V S (S^2 + eps_R)^-1 V^T,
                              T_ij = (s_i + s_j)/((s_i + s_j)^2 + eps_T).
                              Algorithm 4 takes (eps^1/2, eps^1/2, eps^1/4). */
  double margin_max;       /* learned/user sigma_max is multiplied by this (1.1) */
  double margin_min;       /* learned/user sigma_min is multiplied by this (1.0: the learned
                              bound is already a 0.98 quantile; values it overestimates are
                              finished by the refinement's stop test) */
  const float* user_bounds; /* device, batch x 2 (sigma_min, sigma_max), bound == USER */
  const float* probe;      /* device, batch x n Gaussian probe vectors, bound == LEARNED */
  double eigh_off_tol;     /* eigensolver restarts: T = V^T H V is re-formed from the input and
                              swept again from V' = I (V <- V V') while |off(T)|_F > eigh_off_tol
                              |H|_F; the last T gives the eigenvalues (6e-6: about the FP32
                              floor of a restart at n = 4096) */
  int32_t eigh_restarts;   /* cap on those restarts (2) */
  double jacobi_fro_tol;   /* Jacobi also stops after a sweep whose rotated entries have
                              sqrt(sum h_pq^2) <= jacobi_fro_tol |H|_F: a normwise test, met
                              sweeps before the relative one when small eigenvalues need many
                              sweeps for relative accuracy (3e-4; 0 disables it) */
  int32_t poly;            /* svdp_poly (CANS3); other values need bound CONSERVATIVE and
                              precision FP32 */
  int32_t bf16_correct;    /* precision BF16: correct svd_polar_fwd's U, V and S, and polar_fwd's
                              W, H and cached (S, V) when the cache is requested, for the BF16
                              rounding of the polar iterate (1; 0 = off).  That rounding
                              leaves W = W_t (I + S) with S skew of order 2^-9 / sigma_min of
                              the iterate, which the FP32 refinement cannot remove.  With
                              (lam, V) = eig(sym(W^T A)) and P = V^T W^T A V, S~ = V^T S V
                              solves S~ L + L S~ = -(P - P^T) elementwise; U = W V (I - S~/2)
                              and V (I + S~/2) are then right to second order, and
                              sigma_i = diag((I + S~/2) P (I + S~/2)) to third, plus the
                              2 x 2 shift of the coupling the eigensolver's stop leaves in
                              P.  P is the eigensolver's last restart measure; the cost is
                              one n^3 GEMM and two element-wise passes (polar_fwd: three more
                              GEMMs, W <- W (V Mu) V^T and H = sym(W^T A)).  polar_fwd without
                              the cache is not corrected; tall matrices keep W's error outside
                              A's column space unless tall_qr is on */
  double pe_lo;            /* poly PE: lower end of the interval assumed to hold the singular
                              values of A / |A|_F (1e-3); values below it still converge, more
                              slowly, and the step count grows as it falls */
  int32_t tall_qr;         /* svd_polar_fwd with m >= 2 n: 1 = QR preprocessing (the paper's
                              rectangular experiments): an orthonormal basis Q of A's columns
                              by block Gram-Schmidt with CholeskyQR blocks (FP32 Grams: a
                              64-column block of condition beyond about 1e7 loses its smallest
                              directions; set 0 for such inputs), then the SVD of the n x n
                              matrix B = Q^T A, U = Q U_B; 0 = CANS on A itself.  Default 1 */
} svdp_params;

/* per-matrix diagnostics, device array of `batch` records */
typedef struct {
  int32_t iters;    /* CANS steps taken (BF16 + FP32) */
  int32_t sweeps;   /* Jacobi sweeps: the FP32 phase plus the sweeps of eigensolver restarts */
  int32_t flags;    /* SVDP_FLAG_* */
  float residual;   /* |X^T X - I|_F / sqrt(n) of the iterate entering the last CANS step */
} svdp_info;

typedef struct svdp_handle svdp_handle;

/* Fill `p` with the defaults quoted in the field comments (the paper's CANS
 * hyperparameters from its reproducibility appendix; eps triple zero). */
void svdp_default_params(svdp_params* p, int64_t batch, int64_t m, int64_t n);

/* Library handle: owns the predictor model (device copy) and a pinned host
 * word for counter read-back.  One handle per thread / stream. */
svdp_status svdp_create(svdp_handle** h);
svdp_status svdp_destroy(svdp_handle* h);

/* Load the interval predictor: `host_model` (HOST pointer) holds
 * SVDP_MODEL_FLOATS floats: the MLP parameters (layout of svdp_mlp_fwd)
 * followed by 8 feature means and 8 feature standard deviations. */
#define SVDP_MLP_PARAMS 4866
#define SVDP_MODEL_FLOATS (SVDP_MLP_PARAMS + 16)
svdp_status svdp_set_model(svdp_handle* h, const float* host_model);

/* op codes of svdp_workspace_size */
#define SVDP_OP_SVD_FWD 0
#define SVDP_OP_SVD_BWD 1
#define SVDP_OP_POLAR_FWD 2
#define SVDP_OP_POLAR_BWD 3
#define SVDP_OP_EIGH 4
#define SVDP_OP_FEATURES 5
#define SVDP_OP_EIGH_BWD 6
#define SVDP_OP_EIGH_DC 7
svdp_status svdp_workspace_size(const svdp_params* p, int32_t op, size_t* bytes);

/* name of a status code; any other value gives "unknown status" (the code
 * is taken as an int, so a value from a foreign caller outside svdp_status
 * is defined behaviour) */
const char* svdp_status_string(int32_t status);
/* message of the last failing call on this thread (static storage) */
const char* svdp_last_error(void);

/* Number of host synchronisations the library has made so far (all
 * threads): each is one device count read back by a forward pass. */
int64_t svdp_host_syncs(void);

/* Forward SVD A = U diag(S) V^T (Algorithm 1).
 * A: m x n.  U: m x n.  S: n values, descending.  V: n x n (V, not V^T).
 * info: device, batch records (may be null). */
svdp_status svd_polar_fwd(svdp_handle* h, const svdp_params* p,
                          const float* A, int64_t lda, int64_t sA,
                          float* U, int64_t ldu, int64_t sU,
                          float* S, int64_t sS,
                          float* V, int64_t ldv, int64_t sV,
                          svdp_info* info, void* ws, size_t ws_bytes, void* stream);

/* Backward of svd_polar_fwd (Algorithm 4, regularisers from p->eps_*), in
 * the eigenbasis of H: with Ahat = U^T dU and P = V^T dV it forms
 * C = sym(diag dS + K^T o skew(P + Ahat) - diag(D S) Ahat diag(D)),
 * D = S / (S^2 + eps_R), Y = T o C, and dA = (dU diag(D) + 2 U S Y) V^T,
 * which equals Algorithm 4's dW R + 2 M X with M = U S V^T.
 * U, S, V: the forward's outputs.  dU (m x n), dS (n), dV (n x n, the
 * gradient of V; for a loss on V^T pass its transpose).  dA: m x n. */
svdp_status svd_polar_bwd(svdp_handle* h, const svdp_params* p,
                          const float* U, int64_t ldu, int64_t sU,
                          const float* S, int64_t sS,
                          const float* V, int64_t ldv, int64_t sV,
                          const float* dU, int64_t lddu, int64_t sdU,
                          const float* dS, int64_t sdS,
                          const float* dV, int64_t lddv, int64_t sdV,
                          float* dA, int64_t ldda, int64_t sdA,
                          void* ws, size_t ws_bytes, void* stream);

/* svd_polar_bwd without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): its scratch is a file-scope device
 * array of 128 MiB, one per GPU, resolved once per device and held until
 * the process ends.  The call allocates nothing (no hipMalloc / hipFree, no
 * allocating library routine).  Same arguments and results as
 * svd_polar_bwd otherwise.  SVDP_ERR_WORKSPACE when the batch needs more
 * than 128 MiB of scratch (svdp_workspace_size with SVDP_OP_SVD_BWD gives the
 * need; e.g. 64 matrices of 256 x 256 need 84 MB).  All calls on one GPU
 * share that GPU's array and nothing in it carries over between calls:
 * calls that overlap on one GPU (other streams or threads) race. */
svdp_status svd_polar_bwd_noalloc(svdp_handle* h, const svdp_params* p,
                                  const float* U, int64_t ldu, int64_t sU,
                                  const float* S, int64_t sS,
                                  const float* V, int64_t ldv, int64_t sV,
                                  const float* dU, int64_t lddu, int64_t sdU,
                                  const float* dS, int64_t sdS,
                                  const float* dV, int64_t lddv, int64_t sdV,
                                  float* dA, int64_t ldda, int64_t sdA, void* stream);

/* Polar decomposition A = W H (Algorithm 1 up to the symmetric factor).
 * W: m x n with orthonormal columns.  H: n x n, sym(W^T A).  Optional
 * S_cache (n) / V_cache (n x n): eigenvalues (descending) and eigenvectors
 * of H for polar_bwd; both null to skip the eigendecomposition. */
svdp_status polar_fwd(svdp_handle* h, const svdp_params* p,
                      const float* A, int64_t lda, int64_t sA,
                      float* W, int64_t ldw, int64_t sW,
                      float* H, int64_t ldh, int64_t sH,
                      float* S_cache, int64_t sS,
                      float* V_cache, int64_t ldv, int64_t sV,
                      svdp_info* info, void* ws, size_t ws_bytes, void* stream);

/* Backward of the polar decomposition (Algorithm 2 with regularisers eps_R,
 * eps_T from p): dA = (dW V D + 2 (A V) Xt) V^T with
 * Xt = T o (sym(V^T dH V) - D sym((A V)^T (dW V)) D), D = S/(S^2 + eps_R).
 * A: the forward input.  H: n x n.  S_cache / V_cache: the eigenpairs of H
 * from polar_fwd, or both null to compute them here first (Algorithm 2,
 * step 1).  dW: m x n, dH: n x n (either may be null).  dA: m x n. */
svdp_status polar_bwd(svdp_handle* h, const svdp_params* p,
                      const float* A, int64_t lda, int64_t sA,
                      const float* H, int64_t ldh, int64_t sH,
                      const float* S_cache, int64_t sS,
                      const float* V_cache, int64_t ldv, int64_t sV,
                      const float* dW, int64_t lddw, int64_t sdW,
                      const float* dH, int64_t lddh, int64_t sdH,
                      float* dA, int64_t ldda, int64_t sdA,
                      void* ws, size_t ws_bytes, void* stream);

/* Symmetric eigendecomposition H = V diag(lam) V^T (the EVD step of
 * Algorithm 1) by batched block Jacobi; lam descending (signed), V n x n.
 * Uses p->batch, p->n (m ignored), max_sweeps, inner_sweeps, fp64_sweeps,
 * jacobi_tol, jacobi_abs, jacobi_fro_tol, eigh_off_tol, eigh_restarts.
 * info: sweeps and flags (may be null). */
svdp_status svdp_eigh(svdp_handle* h, const svdp_params* p,
                      const float* H, int64_t ldh, int64_t sH,
                      float* lam, int64_t slam,
                      float* V, int64_t ldv, int64_t sV,
                      svdp_info* info, void* ws, size_t ws_bytes, void* stream);

/* Symmetric eigendecomposition by polar-based spectral divide and conquer
 * (the stable QDWH-eig-type method the paper's related work cites for
 * relieving the EVD bottleneck at large n), with the same results as
 * svdp_eigh: lam descending, V n x n.  H is taken as its symmetric part
 * (H + H^T) / 2: inside the SVD, the symmetric matrix nearest to W^T A.
 * A split of a symmetric piece M (s x s):
 *   sigma = trace(M) / s; W = polar(M - sigma I) = sign(M - sigma I) by
 *   conservative FP32 CANS (the same iteration as Algorithm 1); P = (I + W)/2
 *   projects onto the eigenvectors above sigma, of rank k = (s + trace W)/2;
 *   Q = [Q1 Q2] spans P's range and its complement: the polar factors (the
 *   same CANS) of P Om1 and of (I - P) Om2 with P Om1's span projected out,
 *   Om a seeded pseudo-random matrix, then one step of subspace iteration,
 *   [P Q1, (I - P) Q2] orthonormalised block by block by Newton-Schulz;
 *   T = Q^T M Q (symmetrised), whose diagonal blocks
 *   T[:k, :k] and T[k:, k:] are the two new pieces; V = [Q1 V1, Q2 V2] once
 *   they are solved.  The dropped coupling T[:k, k:] is held to
 *   10 tol |T|_F (tol: the CANS stop test).
 * Each matrix is split once; pieces above 1024 are split again, to 4 levels
 * (16 pieces at most).  Every piece is solved by svdp_eigh's solver shifted
 * by its mean eigenvalue: those of at most 1024, zero-padded to the largest,
 * as one batch; a larger one (at the depth limit, or one that does not
 * split) alone.  A piece does not split when k = 0 or s, the polar
 * iteration is unconverged, |W|_F^2 is off s by more than 1/2, a
 * Newton-Schulz block stays off orthonormal, or the coupling is larger; when
 * that happens to the first split, the matrix runs svdp_eigh's solver on H
 * itself and gets SVDP_FLAG_FALLBACK_USED.  Two host reads per split (k,
 * then the coupling and orthonormality checks).  Uses p->batch, p->n (m
 * ignored), the CANS settings (delta, tol, max_iters, pre_iters) and the
 * eigensolver settings of svdp_eigh; workspace op SVDP_OP_EIGH_DC (one
 * matrix's worth, reused across the batch: about 32 n^2 floats at
 * n = 4096, 27 n^2 at 8192).  info: sweeps (the largest over the pieces)
 * and flags. */
svdp_status svdp_eigh_dc(svdp_handle* h, const svdp_params* p,
                         const float* H, int64_t ldh, int64_t sH,
                         float* lam, int64_t slam,
                         float* V, int64_t ldv, int64_t sV,
                         svdp_info* info, void* ws, size_t ws_bytes, void* stream);

/* Backward of the symmetric eigendecomposition: the EVD pseudo-gradient
 * (theorem on the EVD backward, Section 4.2) with the regularised K of the
 * same section, K_ij = (l_i - l_j) / ((l_i - l_j)^2 + eps_K):
 *   dH = V (S + diag(dlam)) V^T,  S = K^T o (V^T dV - dV^T V) / 2.
 * eps_K = 0 gives K_ij = 1 / (l_i - l_j), and 0 for equal eigenvalues
 * (rotations inside an eigenspace do not contribute).  lam, V: the forward
 * eigenpairs (any order, as svdp_eigh returns them); dlam (batch x n) and
 * dV (n x n) may be null (zero).  dH: n x n, symmetric.  Uses p->batch,
 * p->n (m ignored), eps_K; workspace op SVDP_OP_EIGH_BWD. */
svdp_status svdp_eigh_bwd(svdp_handle* h, const svdp_params* p,
                          const float* lam, int64_t slam,
                          const float* V, int64_t ldv, int64_t sV,
                          const float* dlam, int64_t sdlam,
                          const float* dV, int64_t lddv, int64_t sdV,
                          float* dH, int64_t lddh, int64_t sdH,
                          void* ws, size_t ws_bytes, void* stream);

/* Sketch features of each matrix (the learned interval predictor's input).
 * probe: batch x n.  With y0 = probe, y1 = A y0, y2 = A^T y1, ... up to y7
 * and r_k = |y_k| / |y_(k-1)|:  F[b] = (log(|A|_F / r_7),
 * log(r_2 / r_3), ..., log(r_6 / r_7), log(n), log(m / n)) (8 floats);
 * aux[b] = (r_7, |A|_F).  F: batch x 8, aux: batch x 2.  The sequence is
 * computed on A / |A|_F (the ratios scale back exactly), so no norm
 * overflows FP32 whatever the scale of A. */
svdp_status svdp_bound_features(svdp_handle* h, const svdp_params* p,
                                const float* A, int64_t lda, int64_t sA,
                                const float* probe, float* F, float* aux,
                                void* ws, size_t ws_bytes, void* stream);

/* The same features for A = Q1 diag(s) Q2^T with probe Q2 z, which depend on
 * (s, z) only: |y_k| = |s^k * z|.  s, z: rows x n; m_over_n: rows (host
 * scalar semantics per row, device array).  Used to build training sets. */
svdp_status svdp_spectral_features(const float* s, const float* z, int64_t rows, int64_t n,
                                   const float* m_over_n, float* F, float* aux, void* stream);

/* Training targets of the interval predictor (Section 3, learned bounds:
 * the network predicts how far sigma_max lies above the sketch estimate r_7
 * and the log condition number): for each row of s (rows x n, a spectrum)
 * and aux (rows x 2 from svdp_spectral_features, aux[r][0] = r_7),
 * T[r] = (log(max s / r_7), log(max s / min s)) (min s clamped at 1e-30).
 * T: rows x 2, device.  rows = 0 is a no-op; SVDP_ERR_SHAPE for rows < 0,
 * rows > 2^26 or n < 1. */
svdp_status svdp_training_targets(const float* s, const float* aux, int64_t rows, int64_t n, float* T,
                                  void* stream);
/* Feature standardisation of the predictor's inputs (Section 3, learned
 * bounds): mu[f] = mean and sd[f] = sample standard deviation (divisor
 * rows - 1, clamped at 1e-3) of column f of F (rows x 8, device), summed in
 * FP64 in a fixed order, so repeated calls agree bit for bit.  mu, sd: 8
 * floats each, device.  SVDP_ERR_SHAPE unless 1 <= rows <= 2^26. */
svdp_status svdp_feature_stats(const float* F, int64_t rows, float* mu, float* sd, void* stream);

/* MLP 8 -> 64 -> 64 -> 2 with tanh hidden layers.  params (4866 floats):
 * W1 (64 x 8), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2), weights
 * row-major (out x in).  Inputs are standardised as (X - mu) / sd when mu, sd
 * (8 floats each) are given.  X: rows x 8.  out: rows x 2.  act: rows x 128
 * (hidden activations, kept for the backward; may be null in forward-only
 * use). */
svdp_status svdp_mlp_fwd(const float* params, const float* mu, const float* sd,
                         const float* X, int64_t rows, float* out, float* act, void* stream);
/* dparams = d(sum dout * out)/d params (overwritten).  ws: at least
 * svdp_mlp_bwd_ws_bytes(rows) bytes. */
size_t svdp_mlp_bwd_ws_bytes(int64_t rows);
svdp_status svdp_mlp_bwd(const float* params, const float* mu, const float* sd,
                         const float* X, const float* act, const float* dout, int64_t rows,
                         float* dparams, void* ws, size_t ws_bytes, void* stream);
/* Pinball (quantile) loss mean_rows sum_j rho_tau_j(target_j - out_j),
 * rho_tau(u) = max(tau u, (tau - 1) u): dout (rows x 2) and *loss (device,
 * accumulated: clear it first). */
svdp_status svdp_pinball(const float* out, const float* target, int64_t rows, float tau0,
                         float tau1, float* dout, float* loss, void* stream);
/* One Adam step (bias-corrected, step count t >= 1) on n parameters. */
svdp_status svdp_adam_step(float* params, float* m, float* v, const float* grad, int64_t n,
                           float lr, float beta1, float beta2, float eps, int64_t t,
                           void* stream);

/* HOST helper: the coefficient table (alpha_k, beta_k) of p(x) = alpha x +
 * beta x^3 for `steps` CANS steps into host `table` (steps x 2 doubles).
 * kind 0: conservative (pre_iters steps on [t, 1], t the smallest value they
 * map into [1-delta, 1+delta], then the interval recursion from
 * [1-delta, 1+delta]); kind 1: interval recursion from [lo, 1].
 * Returns the preprocessing t (kind 0) or lo (kind 1) in *t_out. */
svdp_status svdp_cans_table(int32_t kind, double delta, int32_t pre_iters, double lo,
                            int32_t steps, double* table, double* t_out);

/* HOST helper: the conservative coefficient table (c1, c3, c5) of
 * p(x) = c1 x + c3 x^3 + c5 x^5 for `steps` steps of iteration polynomial
 * `poly` into host `table` (steps x 3 doubles): CANS3 as svdp_cans_table
 * kind 0 with c5 = 0; NS (1.5, -0.5, 0) throughout, t = 0; CANS5 the
 * interval-optimal quintics, pre_iters of them on [t, 1] (t the smallest
 * value they map into [1-delta, 1+delta]), then the interval recursion from
 * [1-delta, 1+delta].  Returns t in *t_out (may be null). */
svdp_status svdp_poly_table(int32_t poly, double delta, int32_t pre_iters, int32_t steps, double* table,
                            double* t_out);

/* HOST helper: the Polar Express schedule (poly SVDP_POLY_PE) from [lo, 1]:
 * the coefficients (c1, c3, c5) of each step, with the step's 1 / 1.01 input
 * scaling folded in (c_k / 1.01^k on every step but the last), into host
 * `table` (max_steps x 3 doubles), and the number of steps in *steps.  Step t
 * takes the odd quintic closest to 1 in max norm on [max(l_t, u_t / 10), u_t];
 * [l_t+1, u_t+1] is the image of [l_t / 1.01, u_t / 1.01] under it.  The
 * damped steps continue until u - l <= 1e-4, then one undamped step ends the
 * schedule.  INVALID_ARG if lo is not in (0, 1) or the schedule needs more
 * than max_steps (<= 64) steps. */
svdp_status svdp_pe_table(double lo, int32_t max_steps, double* table, int32_t* steps);

/* Kernel timing for benchmarks: while enabled, every launch of the kernel
 * classes below is bracketed by HIP events on its stream.  read() waits for
 * the recorded events and returns, for one class, the summed milliseconds,
 * the launch count and the summed algorithmic work in flops (the method's
 * operation count for the matrices each launch processed); reset() forgets
 * the records. */
#define SVDP_PROF_JAC_SOLVE_F32 0 /* Jacobi 64 x 64 pair solves, FP32 */
#define SVDP_PROF_JAC_SOLVE_F64 1 /* Jacobi pair solves of the FP64 sweep */
#define SVDP_PROF_JAC_APPLY 2     /* Jacobi block rotations on MFMA */
#define SVDP_PROF_GEMM_F32 3      /* batched GEMMs on FP32 MFMA */
#define SVDP_PROF_GEMM_BF16 4     /* batched GEMMs on BF16 MFMA */
/* phases of the forward and backward calls (wall time on the caller's
 * stream between the phase's first and last launch; work 0) */
#define SVDP_PROF_PHASE_BOUND 5    /* normalisation, sketch features, predictor, schedule */
#define SVDP_PROF_PHASE_CANS 6     /* CANS steps before the FP32 refinement */
#define SVDP_PROF_PHASE_REFINE 7   /* FP32 refinement and the final residual */
#define SVDP_PROF_PHASE_H 8        /* H = W^T A */
#define SVDP_PROF_PHASE_EIGH 9     /* eigendecomposition of H */
#define SVDP_PROF_PHASE_U 10       /* BF16 correction, U = W V, column-norm test, QR step */
#define SVDP_PROF_PHASE_FALLBACK 11 /* conservative reruns of the bounded paths */
#define SVDP_PROF_PHASE_BWD 12     /* svd_polar_bwd, polar_bwd */
#define SVDP_PROF_PHASE_QR 13      /* QR preprocessing of tall matrices */
#define SVDP_PROF_JAC_VSWEEP 14    /* Jacobi: the once-per-sweep update of V from every phase's
                                      group rotations (n <= 1024) */
void svdp_profile_enable(int on);
void svdp_profile_reset(void);
int svdp_profile_read(int kind, double* total_ms, int64_t* launches, double* work);

#ifdef __cplusplus
}
#endif
#endif /* SVDP_H */
