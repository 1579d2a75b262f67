/*
 * FP64 CPU oracle for differentiable SVD via polar decomposition.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the GPU library.
 *
 * What is here, each function citing the passage of the paper it follows:
 *   orc_svd        thin SVD by one-sided (Hestenes) Jacobi, the classical
 *                  algorithm the paper cites in its introduction and related
 *                  work; singular values sorted descending (Sec. 2, SVD
 *                  definition under the polar-decomposition definition).
 *   orc_eigh       symmetric eigendecomposition by two-sided cyclic Jacobi
 *                  (textbook: Golub & Van Loan, "Matrix Computations",
 *                  Sec. 8.5), eigenvalues sorted descending.
 *   orc_svd_bwd    Algorithm 4 ("CANS SVD with a regularized backward
 *                  pass"), backward part, literally, step by step.
 *   orc_polar_bwd  Algorithm 2 ("Polar Decomposition Backward"), literally.
 *   orc_townsend   the classical full-rank SVD backward (theorem on low-rank
 *                  SVD backward in the appendix on existing formulas, with
 *                  k = n), used only as a cross-check.
 *
 * All matrices are dense, row-major, double precision.  Batched entry points
 * loop over matrices with OpenMP, one matrix per thread.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* small dense helpers (plain loops)                                   */
/* ------------------------------------------------------------------ */

/* C (p x r) = op(A) * op(B); op(A) is p x q, op(B) is q x r.
 * ta: A is stored q x p (use its transpose); tb likewise. */
static void mm(double *C, const double *A, const double *B, int p, int q, int r,
               int ta, int tb) {
  for (int i = 0; i < p * r; ++i) C[i] = 0.0;
  for (int i = 0; i < p; ++i)
    for (int k = 0; k < q; ++k) {
      double a = ta ? A[(size_t)k * p + i] : A[(size_t)i * q + k];
      if (a == 0.0) continue;
      double *c = C + (size_t)i * r;
      if (tb) {
        for (int j = 0; j < r; ++j) c[j] += a * B[(size_t)j * q + k];
      } else {
        const double *b = B + (size_t)k * r;
        for (int j = 0; j < r; ++j) c[j] += a * b[j];
      }
    }
}

static void sym_inplace(double *A, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double s = 0.5 * (A[i * n + j] + A[j * n + i]);
      A[i * n + j] = s;
      A[j * n + i] = s;
    }
}

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* ------------------------------------------------------------------ */
/* SVD by one-sided Jacobi (Hestenes)                                   */
/* ------------------------------------------------------------------ */

/* Thin SVD A = U diag(S) V^T of an m x n matrix (m >= n).
 * Columns of a working copy are orthogonalised pairwise by plane rotations
 * that zero their inner product; V accumulates the rotations.  A rotation is
 * skipped when |a_i . a_j| <= 1e-15 sqrt(|a_i|^2 |a_j|^2); the iteration
 * stops after a sweep with no rotation (at most 60 sweeps).  Then
 * sigma_i = |a_i|, u_i = a_i / sigma_i (u_i = 0 when sigma_i = 0).
 * Returns the number of sweeps. */
int orc_svd(int m, int n, const double *A, double *U, double *S, double *V) {
  /* column-major working copy: column j is G[j*m .. j*m+m) */
  double *G = dalloc((size_t)m * n);
  double *Vc = dalloc((size_t)n * n); /* column-major V */
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) G[(size_t)j * m + i] = A[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) Vc[(size_t)j * n + j] = 1.0;
  int sweep = 0;
  for (sweep = 1; sweep <= 60; ++sweep) {
    int rotated = 0;
    for (int i = 0; i < n - 1; ++i)
      for (int j = i + 1; j < n; ++j) {
        double *gi = G + (size_t)i * m, *gj = G + (size_t)j * m;
        double al = 0, be = 0, ga = 0;
        for (int k = 0; k < m; ++k) {
          al += gi[k] * gi[k];
          be += gj[k] * gj[k];
          ga += gi[k] * gj[k];
        }
        if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
        rotated = 1;
        double zeta = (be - al) / (2.0 * ga);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int k = 0; k < m; ++k) {
          double x = gi[k], y = gj[k];
          gi[k] = c * x - s * y;
          gj[k] = s * x + c * y;
        }
        double *vi = Vc + (size_t)i * n, *vj = Vc + (size_t)j * n;
        for (int k = 0; k < n; ++k) {
          double x = vi[k], y = vj[k];
          vi[k] = c * x - s * y;
          vj[k] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  /* singular values and order (descending; ties keep column order) */
  double *sig = dalloc(n);
  int *ord = (int *)malloc(sizeof(int) * (n ? n : 1));
  for (int j = 0; j < n; ++j) {
    double s2 = 0;
    for (int k = 0; k < m; ++k) s2 += G[(size_t)j * m + k] * G[(size_t)j * m + k];
    sig[j] = sqrt(s2);
    ord[j] = j;
  }
  for (int a = 1; a < n; ++a) { /* insertion sort, stable */
    int x = ord[a], b = a - 1;
    while (b >= 0 && sig[ord[b]] < sig[x]) { ord[b + 1] = ord[b]; --b; }
    ord[b + 1] = x;
  }
  for (int c = 0; c < n; ++c) {
    int j = ord[c];
    S[c] = sig[j];
    for (int k = 0; k < m; ++k)
      U[(size_t)k * n + c] = sig[j] > 0 ? G[(size_t)j * m + k] / sig[j] : 0.0;
    for (int k = 0; k < n; ++k) V[(size_t)k * n + c] = Vc[(size_t)j * n + k];
  }
  free(G); free(Vc); free(sig); free(ord);
  return sweep > 60 ? 60 : sweep;
}

/* ------------------------------------------------------------------ */
/* symmetric eigendecomposition by two-sided cyclic Jacobi               */
/* ------------------------------------------------------------------ */

/* H = V diag(lam) V^T, H symmetric n x n (only read).  Row-cyclic Jacobi:
 * for each (p, q) with |h_pq| > 1e-15 sqrt(|h_pp h_qq|) (and h_pq != 0) the
 * 2x2 symmetric Schur rotation zeroing h_pq is applied on both sides and
 * accumulated in V.  Stops after a sweep without rotations (max 60).
 * Eigenvalues sorted descending.  Returns sweeps. */
int orc_eigh(int n, const double *H, double *lam, double *V) {
  double *A = dalloc((size_t)n * n), *Q = dalloc((size_t)n * n);
  memcpy(A, H, sizeof(double) * n * n);
  sym_inplace(A, n);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  int sweep;
  for (sweep = 1; sweep <= 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0 || fabs(apq) <= 1e-15 * sqrt(fabs(A[p * n + p] * A[q * n + q]))) continue;
        rotated = 1;
        double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        /* A <- J^T A J with J = [[c, s], [-s, c]] acting on (p, q) */
        for (int k = 0; k < n; ++k) { /* columns p, q */
          double x = A[k * n + p], y = A[k * n + q];
          A[k * n + p] = c * x - s * y;
          A[k * n + q] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) { /* rows p, q */
          double x = A[p * n + k], y = A[q * n + k];
          A[p * n + k] = c * x - s * y;
          A[q * n + k] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {
          double x = Q[k * n + p], y = Q[k * n + q];
          Q[k * n + p] = c * x - s * y;
          Q[k * n + q] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  int *ord = (int *)malloc(sizeof(int) * (n ? n : 1));
  for (int i = 0; i < n; ++i) ord[i] = i;
  for (int a = 1; a < n; ++a) {
    int x = ord[a], b = a - 1;
    while (b >= 0 && A[ord[b] * n + ord[b]] < A[x * n + x]) { ord[b + 1] = ord[b]; --b; }
    ord[b + 1] = x;
  }
  for (int c = 0; c < n; ++c) {
    lam[c] = A[ord[c] * n + ord[c]];
    for (int k = 0; k < n; ++k) V[k * n + c] = Q[k * n + ord[c]];
  }
  free(A); free(Q); free(ord);
  return sweep > 60 ? 60 : sweep;
}

/* ------------------------------------------------------------------ */
/* Algorithm 4: regularised SVD backward, literal                        */
/* ------------------------------------------------------------------ */

/* Ratio x / (x^2 + e), defined as 0 when both x and e vanish (the paper's
 * masks K and T set the entry to 0 exactly where the denominator would). */
static double reg_ratio(double x, double e) {
  double d = x * x + e;
  return d == 0.0 ? 0.0 : x / d;
}

/* Inputs: M (m x n), U (m x n), S (n), V (n x n, NOT V^T), incoming
 * gradients dU (m x n), dS (n), dV (n x n; the gradient of V, i.e. the
 * transpose of the gradient of V^T), any of which may be NULL (= zero).
 * eK, eR, eT are the three regularisers; the paper's Algorithm 4 uses
 * (eps^(1/2), eps^(1/2), eps^(1/4)) and its main text eps^2 for K.
 * Output dM (m x n).  Steps follow Algorithm 4 in order. */
void orc_svd_bwd(int m, int n, const double *M, const double *U, const double *S,
                 const double *V, const double *dU, const double *dS, const double *dV,
                 double eK, double eR, double eT, double *dM) {
  size_t mn = (size_t)m * n, nn = (size_t)n * n;
  double *W = dalloc(mn), *dW = dalloc(mn), *Vt = dalloc(nn), *B = dalloc(nn);
  double *t1 = dalloc(nn), *t2 = dalloc(nn), *dH = dalloc(nn), *R = dalloc(nn);
  double *C = dalloc(nn), *X = dalloc(nn), *tm = dalloc(mn), *tn = dalloc(mn);
  double *zU = dalloc(mn), *zV = dalloc(nn);
  if (!dU) dU = zU;
  if (!dV) dV = zV;
  /* W = U V^T */
  mm(W, U, V, m, n, n, 0, 1);
  /* dW = dU V^T */
  mm(dW, dU, V, m, n, n, 0, 1);
  /* Vtot = dV + W^T dU */
  mm(Vt, W, dU, n, m, n, 1, 0);
  for (size_t i = 0; i < nn; ++i) Vt[i] += dV[i];
  /* B = (V^T Vtot - Vtot^T V) / 2 */
  mm(t1, V, Vt, n, n, n, 1, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[i * n + j] = 0.5 * (t1[i * n + j] - t1[j * n + i]);
  /* dH = V (diag(dS) + K_eps^T o B) V^T, (K_eps)_ij = (si - sj)/((si - sj)^2 + eK) */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double kji = reg_ratio(S[j] - S[i], eK); /* (K^T)_ij = K_ji */
      t1[i * n + j] = kji * B[i * n + j] + (i == j && dS ? dS[i] : 0.0);
    }
  mm(t2, V, t1, n, n, n, 0, 0);
  mm(dH, t2, V, n, n, n, 0, 1);
  /* R = V Sigma (Sigma^2 + eR)^-1 V^T */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t1[i * n + j] = V[i * n + j] * reg_ratio(S[j], eR);
  mm(R, t1, V, n, n, n, 0, 1);
  /* C = (dH - R M^T dW R)_sym */
  mm(t1, M, dW, n, m, n, 1, 0);  /* M^T dW */
  mm(t2, R, t1, n, n, n, 0, 0);  /* R M^T dW */
  mm(t1, t2, R, n, n, n, 0, 0);  /* R M^T dW R */
  for (size_t i = 0; i < nn; ++i) C[i] = dH[i] - t1[i];
  sym_inplace(C, n);
  /* X = V (T_eps o (V^T C V)) V^T, (T_eps)_ij = (si + sj)/((si + sj)^2 + eT) */
  mm(t1, V, C, n, n, n, 1, 0);
  mm(t2, t1, V, n, n, n, 0, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t2[i * n + j] *= reg_ratio(S[i] + S[j], eT);
  mm(t1, V, t2, n, n, n, 0, 0);
  mm(X, t1, V, n, n, n, 0, 1);
  /* dM = dW R + 2 M X */
  mm(tm, dW, R, m, n, n, 0, 0);
  mm(tn, M, X, m, n, n, 0, 0);
  for (size_t i = 0; i < mn; ++i) dM[i] = tm[i] + 2.0 * tn[i];
  free(W); free(dW); free(Vt); free(B); free(t1); free(t2); free(dH); free(R);
  free(C); free(X); free(tm); free(tn); free(zU); free(zV);
}

/* ------------------------------------------------------------------ */
/* Algorithm 2: regularised polar backward, literal                      */
/* ------------------------------------------------------------------ */

/* Inputs: M (m x n), H (n x n) from M = W H, incoming dW (m x n) and
 * dH (n x n), either may be NULL (= zero).  eR, eT as in Algorithm 2,
 * which uses (eps^(1/2), eps^(1/4)).  With eR = eT = 0 this is the exact
 * backward of the polar-decomposition theorem.  Output dM (m x n). */
void orc_polar_bwd(int m, int n, const double *M, const double *H, const double *dW,
                   const double *dH, double eR, double eT, double *dM) {
  size_t mn = (size_t)m * n, nn = (size_t)n * n;
  double *lam = dalloc(n), *V = dalloc(nn), *Hi = dalloc(nn), *t1 = dalloc(nn);
  double *t2 = dalloc(nn), *Bm = dalloc(nn), *X = dalloc(nn), *tm = dalloc(mn);
  double *tn = dalloc(mn), *zW = dalloc(mn), *zH = dalloc(nn);
  if (!dW) dW = zW;
  if (!dH) dH = zH;
  /* step 1: EVD H = V Sigma V^T */
  orc_eigh(n, H, lam, V);
  /* step 2: H_eps^-1 = V Sigma (Sigma^2 + eR I)^-1 V^T */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t1[i * n + j] = V[i * n + j] * reg_ratio(lam[j], eR);
  mm(Hi, t1, V, n, n, n, 0, 1);
  /* step 3: B = (dH - H_eps^-1 M^T dW H_eps^-1)_sym */
  mm(t1, M, dW, n, m, n, 1, 0);
  mm(t2, Hi, t1, n, n, n, 0, 0);
  mm(t1, t2, Hi, n, n, n, 0, 0);
  for (size_t i = 0; i < nn; ++i) Bm[i] = dH[i] - t1[i];
  sym_inplace(Bm, n);
  /* step 4: Xt_ij = (si + sj)/((si + sj)^2 + eT) (V^T B V)_ij */
  mm(t1, V, Bm, n, n, n, 1, 0);
  mm(t2, t1, V, n, n, n, 0, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) t2[i * n + j] *= reg_ratio(lam[i] + lam[j], eT);
  /* step 5: X = V Xt V^T */
  mm(t1, V, t2, n, n, n, 0, 0);
  mm(X, t1, V, n, n, n, 0, 1);
  /* step 6: dM = dW H_eps^-1 + 2 M X */
  mm(tm, dW, Hi, m, n, n, 0, 0);
  mm(tn, M, X, m, n, n, 0, 0);
  for (size_t i = 0; i < mn; ++i) dM[i] = tm[i] + 2.0 * tn[i];
  free(lam); free(V); free(Hi); free(t1); free(t2); free(Bm); free(X); free(tm);
  free(tn); free(zW); free(zH);
}

/* ------------------------------------------------------------------ */
/* classical full-rank SVD backward (cross-check only)                   */
/* ------------------------------------------------------------------ */

/* Low-rank SVD backward theorem of the appendix on existing formulas with
 * k = n (distinct positive singular values):
 *   dA = [U (F o (U^T dU - dU^T U)) S + (I - U U^T) dU S^-1] V^T
 *        + U (I o dS) V^T + U S (F o (V^T dV - dV^T V)) V^T,
 * F_ij = 1/(s_j^2 - s_i^2) off the diagonal, 0 on it.  (The last term of the
 * theorem with I - V V^T vanishes for k = n.)  The "+" sign of the
 * (I - U U^T) term is the theorem's. */
void orc_townsend(int m, int n, const double *U, const double *S, const double *V,
                  const double *dU, const double *dS, const double *dV, double *dA) {
  size_t mn = (size_t)m * n, nn = (size_t)n * n;
  double *a = dalloc(nn), *b = dalloc(nn), *inner = dalloc(nn), *P = dalloc(mn);
  double *t = dalloc(mn), *zU = dalloc(mn), *zV = dalloc(nn);
  if (!dU) dU = zU;
  if (!dV) dV = zV;
  mm(a, U, dU, n, m, n, 1, 0); /* U^T dU */
  mm(b, V, dV, n, n, n, 1, 0); /* V^T dV */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double F = (i == j) ? 0.0 : 1.0 / (S[j] * S[j] - S[i] * S[i]);
      double v = F * (a[i * n + j] - a[j * n + i]) * S[j];         /* (F o ..) S */
      v += S[i] * F * (b[i * n + j] - b[j * n + i]);               /* S (F o ..) */
      if (i == j && dS) v += dS[i];
      inner[i * n + j] = v;
    }
  /* P = U inner + (I - U U^T) dU S^-1 */
  mm(P, U, inner, m, n, n, 0, 0);
  mm(t, U, a, m, n, n, 0, 0); /* U U^T dU */
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j)
      P[(size_t)i * n + j] += (dU[(size_t)i * n + j] - t[(size_t)i * n + j]) / S[j];
  mm(dA, P, V, m, n, n, 0, 1);
  free(a); free(b); free(inner); free(P); free(t); free(zU); free(zV);
}

/* ------------------------------------------------------------------ */
/* batched drivers (one matrix per OpenMP thread)                        */
/* ------------------------------------------------------------------ */

void orc_svd_batch(int batch, int m, int n, const double *A, double *U, double *S,
                   double *V, int *sweeps, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int b = 0; b < batch; ++b) {
    int sw = orc_svd(m, n, A + (size_t)b * m * n, U + (size_t)b * m * n, S + (size_t)b * n,
                     V + (size_t)b * n * n);
    if (sweeps) sweeps[b] = sw;
  }
}

void orc_svd_bwd_batch(int batch, int m, int n, const double *M, const double *U,
                       const double *S, const double *V, const double *dU,
                       const double *dS, const double *dV, double eK, double eR,
                       double eT, double *dM, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int b = 0; b < batch; ++b) {
    size_t mn = (size_t)m * n, nn = (size_t)n * n;
    orc_svd_bwd(m, n, M + b * mn, U + b * mn, S + (size_t)b * n, V + b * nn,
                dU ? dU + b * mn : NULL, dS ? dS + (size_t)b * n : NULL,
                dV ? dV + b * nn : NULL, eK, eR, eT, dM + b * mn);
  }
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
