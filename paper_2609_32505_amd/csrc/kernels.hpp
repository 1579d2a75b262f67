// Launchers of the element-wise, reduction and small-network kernels.
#pragma once
#include "common.hpp"
#include "svdp.h"

// ---- normalisation (Algorithm 3): s_b = sqrt(|A_b|_1 |A_b|_inf) ----------
// colsum: batch x n scratch, rowmax/colmax/fro2: batch floats (all cleared here).
// per-matrix partial sums of the column pass (norms_launch's part buffer)
inline int norms_blocks(int64_t n) { return (int)((n + 63) / 64); }
hipError_t norms_launch(const float* A, int64_t lda, int64_t sA, int batch, int m, int n,
                        float* colsum, float* rowmax, float* fro2, float* part, int* flags, const int* mask,
                        hipStream_t st);
// scale[b] = sqrt(max_j colsum[b, j] * rowmax[b]) (1 for a zero matrix)
hipError_t transpose_bf16_launch(const void* X, int batch, int m, int n, void* Xt, const int* mask,
                                 hipStream_t st);
hipError_t training_targets_launch(const float* s, const float* aux, int rows, int n, float* T, hipStream_t st);
hipError_t feature_stats_launch(const float* F, int rows, float* mu, float* sd, hipStream_t st);
hipError_t fro_scale_launch(const float* fro2, int batch, float* scale, const int* mask, hipStream_t st);
hipError_t ns_scale_launch(const float* colsum, const float* rowmax, int batch, int n,
                           float* scale, const int* mask, hipStream_t st);
// X[b] = A[b] / scale[b], contiguous m x n, FP32 or BF16
hipError_t scale_copy_launch(const float* A, int64_t lda, int64_t sA, int batch, int m, int n,
                             const float* scale, void* X, int out_bf16, const int* mask,
                             hipStream_t st);

// ---- CANS bookkeeping ------------------------------------------------------
// Broadcast a coefficient table of up to 64 steps into coef (kcap x 2 floats).
hipError_t set_coef_launch(float* coef, const double* tab, int steps, hipStream_t st);
// After step k: matrices whose relative change is <= tol stop (active = 0),
// where[b] = parity of the buffer holding their last iterate;
// iters[b] = iter_base[b * base_stride] + k + 1 (base 0 when iter_base is
// null); conv: per matrix `slots` (change, output) sums of squares written by
// the update GEMM's sub-tiles (gemm_conv_slots), added in slot order;
// *counter = number still active.
hipError_t cans_check_launch(int batch, const float* conv, int slots, float tol, int k, int* active, int* where,
                             int* iters, const int* iter_base, int base_stride, int* flags,
                             int* counter, hipStream_t st);
// residual[b] = |G - I|_F / sqrt(n) from a Gram matrix G (FP32 or BF16);
// part: residual_part_floats(batch) floats of per-workgroup partial sums
size_t residual_part_floats(int64_t batch);
hipError_t residual_launch(const void* G, int gbf16, int batch, int n, float* part, float* resid,
                           const int* mask, hipStream_t st);

// ---- U column-norm check (Algorithm 1, rank-deficiency test) --------------
hipError_t colnorm_check_launch(const float* U, int64_t ldu, int64_t sU, int batch, int m, int n,
                                float* colnorm2, float eps_qr, int* flags, const int* mask,
                                hipStream_t st);
// Algorithm 1's QR orthogonalisation of U for the matrices flagged
// RANK_DEFICIENT (R_ii >= 0; zero columns completed); scratch: 2 m floats
// per matrix.
hipError_t qr_complete_launch(float* U, int64_t ldu, int64_t sU, int batch, int m, int n, float eps_qr,
                              const int* flags, float* scratch, const int* mask, hipStream_t st);
// blocked QR pieces (flagged matrices only): the CholeskyQR factor of one
// block of bc <= 64 columns from its Gram matrix, the replacement of columns
// without direction (sigma_j <= eps_qr sigma_1) and the eps_qr perturbation
// of other deficient columns, and the mask (and count) of the flagged matrices
hipError_t qr_chol_launch(const float* G, float* Rinv, int batch, int bc, const int* qmask, int zero_dep,
                          hipStream_t st);
hipError_t qr_perturb_launch(float* U, int64_t ldu, int64_t sU, int batch, int m, int n, const float* S,
                             int64_t sS, const float* colnorm2, float eps_qr, const int* qmask, hipStream_t st);
hipError_t qr_mask_launch(int batch, const int* flags, const int* mask, int* qmask, int* counter, hipStream_t st);

// ---- backward element-wise steps -------------------------------------------
// D[b, j] = s_j / (s_j^2 + eR) in FP64
hipError_t dvec_launch(const float* S, int64_t sS, int batch, int n, double eR, float* D,
                       hipStream_t st);
// mode 0 (SVD, Algorithm 4 in the eigenbasis): X1 = U^T dU, X2 = V^T dV,
//   out = diag(s) (T o sym(diag dS + K^T o skew(X2 + X1) - diag(D s) X1 diag(D)))
// mode 1 (polar, Algorithm 2): X1 = V^T dH V, X2 = (M V)^T (dW V),
//   out = T o (sym(X1) - diag(D) sym(X2) diag(D))
// X1 / X2 may be null (zero).  n x n, contiguous per matrix.
hipError_t sylvester_launch(int mode, const float* X1, const float* X2, const float* S, int64_t sS,
                            const float* dS, int64_t sdS, const float* D, int batch, int n,
                            double eK, double eT, float* out, hipStream_t st);
// out = (in + in^T) / 2 into a strided destination
hipError_t symmetrize_launch(const float* in, int batch, int n, float* out, int64_t ldo,
                             int64_t so, hipStream_t st);
// First-order correction of a BF16-rounded polar factor from
// P = V^T (W^T A) V, gathered as T[perm_i, perm_j] from the eigensolver's
// last T (working order, leading dimension ldt, batch stride sT), and the
// eigenpairs (lam, V) of sym(W^T A): lam = sgn * S (S magnitudes, snew a
// magnitude) or, with signed_lam, lam = S (snew signed).  Scratch P, Pt: n x n contiguous per
// matrix; dP: batch x n.  Leaves Mu = I - S~/2 in P (S~_ij = -2 skew(P)_ij /
// (lam_i + lam_j)) and the corrected singular values in snew (batch x n).
// U = W V Mu and V (2 I - Mu) replace W V and V.
hipError_t polar_fix_launch(const float* T, int ldt, int64_t sT, const int* perm, const float* S, int64_t sS,
                            const float* sgn, int signed_lam, int batch, int n, float* P, float* Pt, float* dP,
                            float* snew, const int* mask, hipStream_t st);
// V <- 2 V - Vu (Vu contiguous n x n per matrix)
hipError_t vcorr_launch(float* V, int64_t ldv, int64_t sV, const float* Vu, int batch, int n, hipStream_t st);
// S = snew, made non-increasing per matrix
hipError_t sigma_store_launch(const float* snew, int n, float* S, int64_t sS, int batch, const int* mask,
                              hipStream_t st);
// strided batch copy (m x n); matrix b reads src_alt when sel[b], and is
// skipped when mask is given and mask[b] == 0
hipError_t copy_launch(const float* src, int64_t lds, int64_t ss, const int* sel,
                       const float* src_alt, float* dst, int64_t ldd, int64_t sd, int batch, int m,
                       int n, hipStream_t st, const int* mask = nullptr);

// ---- sketch features and the interval predictor ---------------------------
// y[b] = c A[b] x[b] (trans = 0, length m) or c A[b]^T x[b] (trans = 1, length n),
// c = 1 / sqrt(fro2[b]) when fro2 is given, else 1
hipError_t matvec_launch(const float* A, int64_t lda, int64_t sA, int batch, int m, int n,
                         const float* x, int64_t sx, float* y, int64_t sy, int trans,
                         const float* fro2, hipStream_t st);
// nrm[b * 8 + slot] = |v[b]|_2 (v length len, stride sv)
hipError_t vnorm_launch(const float* v, int64_t sv, int batch, int len, float* nrm, int slot,
                        hipStream_t st);
// features from |A|_F^2 and the 8 power-sequence norms (see svdp_bound_features)
hipError_t features_launch(const float* fro2, const float* nrm, int batch, int m, int n,
                           float* F, float* aux, hipStream_t st);
// features of A = Q1 diag(s) Q2^T with probe Q2 z, from (s, z)
hipError_t spectral_features_launch(const float* s, const float* z, int rows, int n,
                                    const float* m_over_n, float* F, float* aux, hipStream_t st);
hipError_t mlp_fwd_launch(const float* P, const float* mu, const float* sd, const float* X, int rows,
                          float* out, float* act, hipStream_t st);
hipError_t mlp_bwd_launch(const float* P, const float* mu, const float* sd, const float* X,
                          const float* act, const float* dout, int rows, float* partial,
                          float* dP, hipStream_t st);
size_t mlp_bwd_partial_floats(int rows);
hipError_t pinball_launch(const float* out, const float* target, int rows, float tau0, float tau1,
                          float* dout, float* loss, hipStream_t st);
hipError_t adam_launch(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t st);
// Learned / user bounds -> per-matrix scale, interval-optimal coefficient
// table and BF16 step count (FP64 scalar recursion): ksteps[2b] = steps of
// matrix b to the hand-off (K), ksteps[2b+1] = FP32 steps before its
// interval's lower end reaches bf16_from (K1).
hipError_t bounds_launch(int batch, int mode, const float* mlp_out, const float* aux,
                         const float* user_bounds, double margin_max, double margin_min,
                         double handoff, double bf16_from, int kcap, float* scale, float* coef,
                         int* ksteps, const int* mask, hipStream_t st);

// ---- info ------------------------------------------------------------------
hipError_t info_pack_launch(int batch, const int* iters, const int* sweeps, const int* flags,
                            const float* resid, svdp_info* info, const int* mask, hipStream_t st);
// mask[b] = 1 if flags[b] & bits or resid[b] > rtol; *counter = count
hipError_t fallback_mask_launch(int batch, int* flags, int bits, const float* resid,
                                float rtol, int* mask, int* counter, hipStream_t st);
hipError_t or_flags_launch(int batch, int* flags, int bits, const int* mask, hipStream_t st);
// p[b] = v where mask[b] != 0 (all b when mask is null)
hipError_t fill_masked_launch(int* p, int v, int n, const int* mask, hipStream_t st);
// *counter = number of nonzero mask entries
hipError_t count_mask_launch(int batch, const int* mask, int* counter, hipStream_t st);
// mask[b] = schedule starts in FP32 (what 0), in BF16 (1), or K is odd (2)
hipError_t sched_mask_launch(int batch, const int* ksteps, int bf16, int what, int* mask, hipStream_t st);
// iters[b] = K
hipError_t sched_iters_launch(int batch, const int* ksteps, int* iters, hipStream_t st);
// dst[b] = src[b] (per_matrix floats, a multiple of 4) where mask[b] != 0
hipError_t copy_masked_launch(const float* src, float* dst, int batch, int64_t per_matrix, const int* mask,
                              hipStream_t st);

// ---- spectral divide and conquer (svdp_eigh_dc), one matrix per call -------
// *sigma = trace(H) / n, A = (H + H^T) / 2 - sigma I (A n x n, pitch lda)
hipError_t dc_shift_launch(const float* H, int64_t ldh, float* A, int64_t lda, int n, float* sigma,
                           hipStream_t st);
// dst (rows x cols, pitch ldd) <- sel[0] ? X1 : X0 (pitch lds)
hipError_t dc_copy_sel_launch(const float* X0, const float* X1, const int* sel, int64_t lds, float* dst,
                              int64_t ldd, int rows, int cols, hipStream_t st);
// x[i] += *mu, i < n
hipError_t dc_add_launch(float* x, int n, const float* mu, hipStream_t st);
// The SVD's order of one eigendecomposition (lam descending by value, V n x n
// pitch ldv, n <= 8192): lam <- |lam| descending, sgn = the signs, V's columns
// permuted to match (perm: n ints of scratch); *flags |= NONFINITE and
// NEG_EIGENVALUE (an eigenvalue below -neg_tol max |lam|)
hipError_t dc_abs_order_launch(float* lam, float* V, int64_t ldv, int n, float* sgn, int* perm, float neg_tol,
                               int* flags, hipStream_t st);
// T <- (T + T^T) / 2 in place (n x n, pitch ldt), exactly symmetric
hipError_t dc_sym_launch(float* T, int64_t ldt, int n, hipStream_t st);
// *k = round((n + trace W) / 2) clamped to [0, n], W = sel[0] ? X1 : X0 (n x n);
// 0 when flags[0] reports an unconverged or non-finite polar iteration or
// when |wn2[1] - n| > 1/2 (wn2[1] = |W|_F^2)
hipError_t dc_rank_launch(const float* X0, const float* X1, const int* sel, const double* wn2, const int* flags,
                          int n, int* k, hipStream_t st);
// *flags |= NEG_EIGENVALUE when some lam[i] < -neg_tol max |lam|
hipError_t dc_neg_launch(const float* lam, int n, float neg_tol, int* flags, hipStream_t st);
// *sweeps = max of sw[0 .. count), *flags |= the or of fl[0 .. count) without
// NEG_EIGENVALUE (the pieces are shifted)
hipError_t dc_info_launch(const int* sw, const int* fl, int count, int* sweeps, int* flags, hipStream_t st);
// A piece of size s solved zero-padded to P x P (V, lam: the solver's output,
// P <= 1024): its s eigenpairs, in the solver's order, to lam_out (plus *mu)
// and the s x s V_out (pitch ldo); padding columns are told apart by their
// weight in rows s.. (map: P ints of scratch); *flags gets
// EIGH_NOT_CONVERGED if they are not exactly P - s
hipError_t dc_leaf_launch(const float* V, const float* lam, const float* mu, int P, int s, int* map, float* lam_out,
                          float* V_out, int64_t ldo, int* flags, hipStream_t st);
// out[i] uniform in [-1, 1), a hash of (seed, i)
hipError_t dc_random_launch(float* out, int64_t count, uint32_t seed, hipStream_t st);
// cs[j] = j < *k ? 1 : -1
hipError_t dc_signs_launch(float* cs, int n, const int* k, hipStream_t st);
// out[0] = |G - I|_F^2, out[1] = 0 (G n x n; part: 2 n doubles of row sums)
hipError_t dc_dev_launch(const float* G, int n, double* part, double* out, hipStream_t st);
// out[0] = |T[:k, k:]|_F^2, out[1] = |T|_F^2 with T = sel && sel[0] ? T1 : T0
// (n x n; k null: k = 0; part: 2 n doubles of row sums)
hipError_t dc_coupling_launch(const float* T0, const float* T1, const int* sel, int n, const int* k, double* part,
                              double* out, hipStream_t st);
