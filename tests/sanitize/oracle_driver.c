/* Runs every entry point of the FP64 C oracle on small matrices in
 * exactly sized heap buffers, for AddressSanitizer / UndefinedBehavior-
 * Sanitizer builds (tests/test_host_sanitizers.py).  Prints "ok". */
#include <stdio.h>
#include <stdlib.h>

int orc_svd(int m, int n, const double *A, double *U, double *S, double *V);
int orc_eigh(int n, const double *H, double *lam, double *V);
void orc_svd_bwd(int m, int n, const double *M, const double *U, const double *S, const double *V,
                 const double *dU, const double *dS, const double *dV, double eK, double eR, double eT,
                 double *dM);
void orc_polar_bwd(int m, int n, const double *M, const double *H, const double *dW, const double *dH,
                   double eR, double eT, double *dM);
void orc_townsend(int m, int n, const double *U, const double *S, const double *V, const double *dU,
                  const double *dS, const double *dV, double *dA);
void orc_svd_batch(int batch, int m, int n, const double *A, double *U, double *S, double *V, int *sweeps,
                   int nthreads);
void orc_svd_bwd_batch(int batch, int m, int n, const double *M, const double *U, const double *S,
                       const double *V, const double *dU, const double *dS, const double *dV, double eK,
                       double eR, double eT, double *dM, int nthreads);
int orc_num_threads(void);

static unsigned state = 12345u;

static double *rnd(size_t n) {
  double *p = (double *)malloc((n ? n : 1) * sizeof(double));
  for (size_t i = 0; i < n; ++i) {
    state = state * 1103515245u + 12345u;
    p[i] = (double)((state >> 8) & 0xffff) / 32768.0 - 1.0;
  }
  return p;
}

static double *zeros(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

int main(void) {
  const int shapes[][2] = {{7, 5}, {5, 5}, {9, 1}, {1, 1}, {6, 3}};
  for (size_t t = 0; t < sizeof(shapes) / sizeof(shapes[0]); ++t) {
    const int m = shapes[t][0], n = shapes[t][1];
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    double *A = rnd(mn), *U = zeros(mn), *S = zeros(n), *V = zeros(nn);
    orc_svd(m, n, A, U, S, V);
    double *dU = rnd(mn), *dS = rnd(n), *dV = rnd(nn), *dM = zeros(mn);
    orc_svd_bwd(m, n, A, U, S, V, dU, dS, dV, 1e-6, 1e-6, 1e-3, dM);
    orc_svd_bwd(m, n, A, U, S, V, NULL, NULL, NULL, 0.0, 0.0, 0.0, dM);
    orc_townsend(m, n, U, S, V, dU, dS, dV, dM);
    double *H = zeros(nn); /* H = V diag(S) V^T */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        for (int k = 0; k < n; ++k) H[i * n + j] += V[i * n + k] * S[k] * V[j * n + k];
    double *dW = rnd(mn), *dH = rnd(nn);
    orc_polar_bwd(m, n, A, H, dW, dH, 1e-6, 1e-3, dM);
    orc_polar_bwd(m, n, A, H, NULL, NULL, 0.0, 0.0, dM);
    free(A); free(U); free(S); free(V); free(dU); free(dS); free(dV); free(dM); free(H); free(dW); free(dH);
  }
  const int sizes[] = {1, 2, 6};
  for (size_t t = 0; t < sizeof(sizes) / sizeof(sizes[0]); ++t) {
    const int n = sizes[t];
    double *R = rnd((size_t)n * n), *H = zeros((size_t)n * n), *lam = zeros(n), *V = zeros((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) H[i * n + j] = R[i * n + j] + R[j * n + i];
    orc_eigh(n, H, lam, V);
    free(R); free(H); free(lam); free(V);
  }
  {
    const int B = 3, m = 6, n = 4;
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    double *A = rnd(B * mn), *U = zeros(B * mn), *S = zeros(B * n), *V = zeros(B * nn);
    int *sw = (int *)calloc(B, sizeof(int));
    orc_svd_batch(B, m, n, A, U, S, V, sw, 1);
    double *dU = rnd(B * mn), *dS = rnd(B * n), *dV = rnd(B * nn), *dM = zeros(B * mn);
    orc_svd_bwd_batch(B, m, n, A, U, S, V, dU, dS, dV, 1e-6, 1e-6, 1e-3, dM, 1);
    orc_svd_bwd_batch(B, m, n, A, U, S, V, NULL, NULL, NULL, 0.0, 0.0, 0.0, dM, 1);
    free(A); free(U); free(S); free(V); free(sw); free(dU); free(dS); free(dV); free(dM);
  }
  if (orc_num_threads() < 1) return 1;
  printf("ok\n");
  return 0;
}
