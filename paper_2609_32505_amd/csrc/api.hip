// C-ABI entry points: argument checks, workspace carving and the host-side
// orchestration of the kernels (no arithmetic of the method runs on the host
// except the scalar CANS coefficient recursion).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "eigh.hpp"
#include "kernels.hpp"
#include "prof.hpp"
#include "svdp.h"

struct svdp_handle {
  float* model = nullptr;  // device: SVDP_MODEL_FLOATS
  bool has_model = false;
  int* host_word = nullptr;  // pinned: counter read-back
  EighAux aux{};  // extra streams of the eigensolver
};

namespace {

thread_local std::string g_last_error;

svdp_status fail(svdp_status s, const char* msg) {
  g_last_error = msg;
  return s;
}
svdp_status hip_fail(hipError_t e, const char* where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return SVDP_ERR_HIP;
}
#define HIPCHK(x, where)                      \
  do {                                        \
    hipError_t _e = (x);                      \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

// Bump allocator over the caller's workspace (null base = size query).
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 1);
    size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return base ? (T*)(base + o) : nullptr;
  }
  void* take_bytes(size_t bytes) { return take<char>(bytes); }
};

// ---------------------------------------------------------------- CANS tables

// Degree-3 odd polynomial closest to 1 in max norm on [a, b]: the error
// equioscillates at a, at the stationary point x*, and at b.
void cans_poly(double a, double b, double& al, double& be, double& lo, double& hi) {
  double s = a * a + a * b + b * b;
  double xs = std::sqrt(s / 3.0);
  be = -2.0 / (a * b * (a + b) + 2.0 * xs * xs * xs);
  al = -be * s;
  lo = al * a + be * a * a * a;
  hi = al * xs + be * xs * xs * xs;
}

// smallest t whose `steps` optimal steps from [t, 1] land in [1-delta, 1+delta]
double preprocess_t(double delta, int steps) {
  auto err = [&](double t) {
    double a = t, b = 1.0, al, be;
    for (int k = 0; k < steps; ++k) cans_poly(a, b, al, be, a, b);
    return std::max(1.0 - a, b - 1.0);
  };
  double lo = 1e-16, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = std::sqrt(lo * hi);
    if (err(mid) <= delta) hi = mid;
    else lo = mid;
  }
  return hi;
}

void table_conservative(double delta, int pre, int steps, double* tab, double* t_out) {
  double t = preprocess_t(delta, pre);
  double a = t, b = 1.0;
  int k = 0;
  for (; k < std::min(pre, steps); ++k) cans_poly(a, b, tab[2 * k], tab[2 * k + 1], a, b);
  a = 1.0 - delta;
  b = 1.0 + delta;
  for (; k < steps; ++k) cans_poly(a, b, tab[2 * k], tab[2 * k + 1], a, b);
  if (t_out) *t_out = t;
}

// The bound kernel clamps the interval's lower end at this value (a singular
// value below 1e-9 of the largest is not resolved in FP32 anyway: such a
// matrix misses the refinement's stop test and falls back).
constexpr double kLoFloor = 1e-9;

// Steps of the interval recursion from [kLoFloor, 1] until its error is
// <= handoff: an upper bound of every matrix's K in the bounded schedule.
int bounded_budget(double handoff) {
  double a = kLoFloor, b = 1.0, al, be;
  for (int k = 0; k < 64; ++k) {
    cans_poly(a, b, al, be, a, b);
    if (std::max(1.0 - a, b - 1.0) <= handoff) return k + 1;
  }
  return 64;
}

void table_interval(double lo, int steps, double* tab) {
  double a = lo, b = 1.0;
  for (int k = 0; k < steps; ++k) cans_poly(a, b, tab[2 * k], tab[2 * k + 1], a, b);
}

// Odd quintic p(x) = c1 x + c3 x^3 + c5 x^5 closest to 1 in max norm on
// [a, b], the degree-5 analogue of cans_poly: the error 1 - p equioscillates
// (signs +, -, +, -) at a, at the two interior stationary points and at b.
// Remez exchange in FP64 from Chebyshev-spaced points: solve
// p(x_i) + s_i E = 1 for (c1, c3, c5, E), move the interior points to the
// roots of p' (a quadratic in x^2), repeat.  A very narrow interval takes the
// limit q(x / x0), q(u) = (15 u - 10 u^3 + 3 u^5) / 8 (p = 1, p' = p'' = 0 at
// x0), which is increasing.  [lo, hi] is the image of [a, b].
static bool solve4(double M[4][5], double x[4]) {
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
    if (M[piv][col] == 0.0) return false;
    for (int k = 0; k < 5; ++k) std::swap(M[col][k], M[piv][k]);
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      const double f = M[r][col] / M[col][col];
      for (int k = col; k < 5; ++k) M[r][k] -= f * M[col][k];
    }
  }
  for (int r = 0; r < 4; ++r) x[r] = M[r][4] / M[r][r];
  return true;
}

void cans5_poly(double a, double b, double* c, double& lo, double& hi) {
  auto p = [&](double x) { const double x2 = x * x; return x * (c[0] + x2 * (c[1] + x2 * c[2])); };
  auto limit = [&]() {
    const double x0 = 0.5 * (a + b);
    c[0] = 15.0 / (8.0 * x0);
    c[1] = -10.0 / (8.0 * x0 * x0 * x0);
    c[2] = 3.0 / (8.0 * x0 * x0 * x0 * x0 * x0);
    lo = p(a);
    hi = p(b);
  };
  if (b - a <= 1e-6 * b) { limit(); return; }
  const double pi = 3.14159265358979323846;
  double x[4] = {a, a + (b - a) * (1.0 - std::cos(pi / 3.0)) / 2.0, a + (b - a) * (1.0 - std::cos(2.0 * pi / 3.0)) / 2.0, b};
  const double s[4] = {1.0, -1.0, 1.0, -1.0};
  double sol[4] = {0, 0, 0, 0};
  for (int it = 0; it < 100; ++it) {
    double M[4][5];
    for (int i = 0; i < 4; ++i) {
      const double x2 = x[i] * x[i];
      M[i][0] = x[i]; M[i][1] = x[i] * x2; M[i][2] = x[i] * x2 * x2; M[i][3] = s[i]; M[i][4] = 1.0;
    }
    if (!solve4(M, sol)) { limit(); return; }
    c[0] = sol[0]; c[1] = sol[1]; c[2] = sol[2];
    // p'(x) = c1 + 3 c3 x^2 + 5 c5 x^4 = 0
    const double disc = 9.0 * c[1] * c[1] - 20.0 * c[0] * c[2];
    if (!(disc > 0.0) || c[2] == 0.0) { limit(); return; }
    double y1 = (-3.0 * c[1] - std::sqrt(disc)) / (10.0 * c[2]);
    double y2 = (-3.0 * c[1] + std::sqrt(disc)) / (10.0 * c[2]);
    if (y1 > y2) std::swap(y1, y2);
    if (!(y1 > a * a && y2 < b * b)) { limit(); return; }
    const double n1 = std::sqrt(y1), n2 = std::sqrt(y2);
    const double move = std::max(std::fabs(n1 - x[1]), std::fabs(n2 - x[2]));
    x[1] = n1;
    x[2] = n2;
    if (move <= 1e-15 * b) break;
  }
  lo = std::min(p(a), p(x[2]));
  hi = std::max(p(x[1]), p(b));
}

// smallest t whose `steps` optimal quintic steps from [t, 1] land in [1-delta, 1+delta]
double preprocess_t5(double delta, int steps) {
  auto err = [&](double t) {
    double a = t, b = 1.0, c[3];
    for (int k = 0; k < steps; ++k) cans5_poly(a, b, c, a, b);
    return std::max(1.0 - a, b - 1.0);
  };
  double lo = 1e-16, hi = 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = std::sqrt(lo * hi);
    if (err(mid) <= delta) hi = mid;
    else lo = mid;
  }
  return hi;
}

// Conservative coefficient table (c1, c3, c5) per step for each iteration
// polynomial: CANS cubic (c5 = 0), classical Newton-Schulz (1.5, -0.5, 0)
// from the first step (no preprocessing, t = 0), or the CANS quintic with its
// own preprocessing.
void table_poly(int poly, double delta, int pre, int steps, double* tab, double* t_out) {
  if (poly == SVDP_POLY_NS) {
    for (int k = 0; k < steps; ++k) { tab[3 * k] = 1.5; tab[3 * k + 1] = -0.5; tab[3 * k + 2] = 0.0; }
    if (t_out) *t_out = 0.0;
    return;
  }
  if (poly == SVDP_POLY_CANS5) {
    const double t = preprocess_t5(delta, pre);
    double a = t, b = 1.0;
    int k = 0;
    for (; k < std::min(pre, steps); ++k) cans5_poly(a, b, tab + 3 * k, a, b);
    a = 1.0 - delta;
    b = 1.0 + delta;
    for (; k < steps; ++k) cans5_poly(a, b, tab + 3 * k, a, b);
    if (t_out) *t_out = t;
    return;
  }
  double tab2[128];
  table_conservative(delta, pre, steps, tab2, t_out);
  for (int k = 0; k < steps; ++k) { tab[3 * k] = tab2[2 * k]; tab[3 * k + 1] = tab2[2 * k + 1]; tab[3 * k + 2] = 0.0; }
}

// Polar Express schedule from [lo, 1] (the iteration the paper's ablation of
// polar iterations compares CANS with; reading of its published
// construction): step t takes the odd quintic closest to 1 in max norm on
// the cushioned interval [max(l, u / 10), u] and applies it to X / 1.01, so
// the interval moves to the image of [l / 1.01, u / 1.01]; once the
// interval is narrower than 1e-4 one undamped step ends the schedule.  The
// image of an interval under an odd quintic is read off its ends and its
// stationary points (the roots of p' in x^2).  tab: (c1, c3, c5) per step,
// the 1.01 folded in.  Returns the step count, or -1 above max_steps.
static void quintic_image(const double* c, double x0, double x1, double& lo, double& hi) {
  auto p = [&](double x) { const double x2 = x * x; return x * (c[0] + x2 * (c[1] + x2 * c[2])); };
  lo = std::min(p(x0), p(x1));
  hi = std::max(p(x0), p(x1));
  const double disc = 9.0 * c[1] * c[1] - 20.0 * c[0] * c[2];
  if (c[2] != 0.0 && disc >= 0.0)
    for (int sg = -1; sg <= 1; sg += 2) {
      const double y = (-3.0 * c[1] + sg * std::sqrt(disc)) / (10.0 * c[2]);
      if (y <= 0.0) continue;
      const double x = std::sqrt(y);
      if (x > x0 && x < x1) { lo = std::min(lo, p(x)); hi = std::max(hi, p(x)); }
    }
}

int pe_table(double lo, int max_steps, double* tab) {
  constexpr double kDamp = 1.01, kCushion = 0.1, kWidth = 1e-4;
  double l = lo, u = 1.0;
  for (int t = 0; t < max_steps; ++t) {
    double c[3], ilo, ihi;
    cans5_poly(std::max(l, kCushion * u), u, c, ilo, ihi);
    const bool last = u - l <= kWidth;
    if (last) {
      for (int k = 0; k < 3; ++k) tab[3 * t + k] = c[k];
      return t + 1;
    }
    tab[3 * t] = c[0] / kDamp;
    tab[3 * t + 1] = c[1] / (kDamp * kDamp * kDamp);
    tab[3 * t + 2] = c[2] / (kDamp * kDamp * kDamp * kDamp * kDamp);
    quintic_image(c, l / kDamp, u / kDamp, l, u);
  }
  return -1;
}

// ---------------------------------------------------------------- checks

bool bad_shape(const svdp_params* p) {
  return p->batch < 0 || p->n < 1 || p->m < p->n || p->batch > 65535 || p->m > (1 << 20) ||
         p->n > 8192 || p->m * p->n > (int64_t)1 << 31;
}
bool bad_ld(int64_t ld, int64_t cols, int64_t stride, int64_t rows) {
  return ld < cols || stride < 0 || (stride > 0 && stride < (rows - 1) * ld + cols);
}
svdp_status check_common(const svdp_params* p) {
  if (!p) return fail(SVDP_ERR_INVALID_ARG, "null params");
  if (bad_shape(p)) return fail(SVDP_ERR_SHAPE, "need batch >= 0, m >= n >= 1 (n <= 8192)");
  if (p->precision != SVDP_PREC_FP32 && p->precision != SVDP_PREC_BF16)
    return fail(SVDP_ERR_INVALID_ARG, "unknown precision");
  if (p->bound < 0 || p->bound > 2) return fail(SVDP_ERR_INVALID_ARG, "unknown bound mode");
  if (p->max_iters < 1 || p->max_iters > 64) return fail(SVDP_ERR_INVALID_ARG, "max_iters must be in [1, 64]");
  if (p->pre_iters < 0 || p->pre_iters > p->max_iters) return fail(SVDP_ERR_INVALID_ARG, "bad pre_iters");
  if (p->refine_steps < 0 || p->refine_steps > 8) return fail(SVDP_ERR_INVALID_ARG, "refine_steps must be in [0, 8]");
  if (p->max_sweeps < 1 || p->max_sweeps > 100) return fail(SVDP_ERR_INVALID_ARG, "max_sweeps must be in [1, 100]");
  if (p->inner_sweeps < 1 || p->inner_sweeps > 16) return fail(SVDP_ERR_INVALID_ARG, "inner_sweeps must be in [1, 16]");
  if (p->fp64_sweeps < 0 || p->fp64_sweeps > 4) return fail(SVDP_ERR_INVALID_ARG, "fp64_sweeps must be in [0, 4]");
  if (p->eigh_restarts < 0 || p->eigh_restarts > 8)
    return fail(SVDP_ERR_INVALID_ARG, "eigh_restarts must be in [0, 8]");
  if (!(p->eigh_off_tol >= 0)) return fail(SVDP_ERR_INVALID_ARG, "eigh_off_tol must be >= 0");
  if (!(p->jacobi_fro_tol >= 0)) return fail(SVDP_ERR_INVALID_ARG, "jacobi_fro_tol must be >= 0");
  if (!(p->delta > 0 && p->delta < 1)) return fail(SVDP_ERR_INVALID_ARG, "delta must be in (0, 1)");
  if (!(p->tol > 0)) return fail(SVDP_ERR_INVALID_ARG, "tol must be > 0");
  if (p->eps_K < 0 || p->eps_R < 0 || p->eps_T < 0) return fail(SVDP_ERR_INVALID_ARG, "eps must be >= 0");
  if (p->poly < SVDP_POLY_CANS3 || p->poly > SVDP_POLY_PE) return fail(SVDP_ERR_INVALID_ARG, "unknown poly");
  if (p->bf16_correct != 0 && p->bf16_correct != 1) return fail(SVDP_ERR_INVALID_ARG, "bf16_correct must be 0 or 1");
  if (p->tall_qr != 0 && p->tall_qr != 1) return fail(SVDP_ERR_INVALID_ARG, "tall_qr must be 0 or 1");
  if (p->poly == SVDP_POLY_PE) {
    if (!(p->pe_lo > 0 && p->pe_lo < 1)) return fail(SVDP_ERR_INVALID_ARG, "pe_lo must be in (0, 1)");
    double tab[3 * 64];
    if (pe_table(p->pe_lo, p->max_iters, tab) < 0)
      return fail(SVDP_ERR_INVALID_ARG, "the Polar Express schedule from pe_lo needs more than max_iters steps");
  }
  if (p->poly != SVDP_POLY_CANS3 && (p->bound != SVDP_BOUND_CONSERVATIVE || p->precision != SVDP_PREC_FP32))
    return fail(SVDP_ERR_INVALID_ARG, "poly variants run on the conservative FP32 path");
  return SVDP_OK;
}

EighOpts eigh_opts(const svdp_params* p) {
  EighOpts o;
  o.inner_sweeps = p->inner_sweeps;
  o.fp64_sweeps = p->fp64_sweeps;
  o.fp64_inner = p->inner_sweeps;
  o.tol = (float)p->jacobi_tol;
  o.abs_tol = (float)p->jacobi_abs;
  o.fro_tol = (float)p->jacobi_fro_tol;
  o.neg_tol = 1e-4f;
  o.off_tol = (float)p->eigh_off_tol;
  o.restarts = p->eigh_restarts;
  return o;
}

// ---------------------------------------------------------------- forward workspace

// Refinement steps allowed beyond refine_steps before a bounded-path matrix
// is declared unconverged (and rerun with conservative CANS).
constexpr int kRefineExtra = 8;

// Algorithm 1's QR step: one workgroup runs CGS2 over all columns of a
// flagged matrix up to this n; beyond it, blocks of kQrBlock columns are
// projected against the earlier ones by GEMMs (twice) and orthonormalised
// among themselves by CholeskyQR (twice).
constexpr int kQrBlockedFrom = 512;
constexpr int kQrBlock = 64;

// QR preprocessing for matrices at least twice as tall as wide (below that
// the QR costs about what it saves on the CANS steps)
bool use_tall_qr(const svdp_params* p) { return p->tall_qr && p->m >= 2 * p->n; }

struct FwdWs {
  float *X0, *X1, *G;
  void *Y0, *Y1;  // BF16 iterates (never aliasing the FP32 ones)
  void *Yt0, *Yt1;  // their transposes (n x m, BF16): the Gram's operands, contiguous in k
  void* eigh;
  float *scale, *conv, *resid, *rpart, *colsum, *rowmax, *fro2, *fpart, *coef, *rcoef, *F, *aux, *mlpout, *nrm, *y0, *y1;
  float* qr;   // QR completion scratch: 2 m per matrix
  float* qrc;  // blocked QR: projection coefficients, n x kQrBlock per matrix
  float *qrg, *qrr;  // blocked QR: a block's Gram matrix and CholeskyQR factor
  float* P;    // quintic steps: c3 G + c5 G^2, n x n per matrix
  float *Qt, *Bq, *UBq;  // QR preprocessing of tall matrices: Q (m x n), B = Q^T A and U_B (n x n)
  int* qmask;  // blocked QR: the flagged matrices
  int *active, *where, *iters, *flags, *sweeps, *mask, *counter, *ksteps, *gmask;
  void* dc;     // divide-and-conquer eigensolver workspace (dc_route)
  float* dsgn;  // ... the signs of its eigenvalues, n
  int* dperm;   // ... its order by magnitude, n
};

// Single FP32 matrices from kDcFrom up take the EVD step by spectral divide
// and conquer (eigh_dc_one) instead of the batch-1 block Jacobi: at 4096
// about 2x faster, with the same or smaller error.  The BF16 path keeps the
// Jacobi: its correction reads the Jacobi's working copies.
constexpr int64_t kDcFrom = 2048;
bool dc_route(const svdp_params* p) {
  return p->batch == 1 && p->n >= kDcFrom && p->precision == SVDP_PREC_FP32;
}
size_t dc_ws_bytes(const svdp_params* p);
// H (n x n) = V diag(lam) V^T by divide and conquer for the SVD (workspace:
// dc_ws_bytes(p) at ws); no FALLBACK_USED flag
svdp_status svd_eigh_dc(svdp_handle* h, const svdp_params* p, void* ws, const float* H, float* lam, float* V,
                        int64_t ldv, int* sweeps, int* flags, hipStream_t st);

// dc = false for the divide and conquer's own polar workspace
FwdWs carve_fwd(void* base, const svdp_params* p, size_t* total, bool dc = true) {
  Carver c(base);
  FwdWs w;
  const size_t b = p->batch, m = p->m, n = p->n;
  w.X0 = c.take<float>(b * m * n);
  w.X1 = c.take<float>(b * m * n);
  w.Y0 = c.take<uint16_t>(b * m * n);
  w.Y1 = c.take<uint16_t>(b * m * n);
  const bool bf16 = p->precision == SVDP_PREC_BF16;
  w.Yt0 = c.take<uint16_t>(bf16 ? b * m * n : 0);
  w.Yt1 = c.take<uint16_t>(bf16 ? b * m * n : 0);
  w.G = c.take<float>(b * n * n);
  w.eigh = c.take_bytes(eigh_ws_bytes(b, n, p->max_sweeps));
  w.scale = c.take<float>(b);
  w.conv = c.take<float>(2 * b * gemm_conv_slots(m, n));
  w.resid = c.take<float>(b);
  w.rpart = c.take<float>(residual_part_floats(b));
  w.colsum = c.take<float>(b * n);
  w.rowmax = c.take<float>(b);
  w.fro2 = c.take<float>(b);
  w.fpart = c.take<float>(b * norms_blocks(n));
  w.coef = c.take<float>(b * 64 * 2);
  w.rcoef = c.take<float>(64 * 2);
  w.F = c.take<float>(b * 8);
  w.aux = c.take<float>(b * 2);
  w.mlpout = c.take<float>(b * 2);
  w.nrm = c.take<float>(b * 8);
  w.y0 = c.take<float>(b * m);
  w.y1 = c.take<float>(b * m);
  w.qr = c.take<float>(b * 2 * m);
  const bool tall_qr = use_tall_qr(p);
  const bool blocked_qr = n > (size_t)kQrBlockedFrom || tall_qr;
  w.qrc = c.take<float>(blocked_qr ? b * n * kQrBlock : 0);
  w.qrg = c.take<float>(blocked_qr ? b * kQrBlock * kQrBlock : 0);
  w.qrr = c.take<float>(blocked_qr ? b * kQrBlock * kQrBlock : 0);
  w.P = c.take<float>(p->poly == SVDP_POLY_CANS5 || p->poly == SVDP_POLY_PE ? b * n * n : 0);
  w.qmask = c.take<int>(b);
  w.active = c.take<int>(b);
  w.where = c.take<int>(b);
  w.iters = c.take<int>(b);
  w.flags = c.take<int>(b);
  w.sweeps = c.take<int>(b);
  w.mask = c.take<int>(b);
  w.gmask = c.take<int>(b);
  w.counter = c.take<int>(16);
  w.ksteps = c.take<int>(2 * b);
  w.Qt = c.take<float>(tall_qr ? b * m * n : 0);
  w.Bq = c.take<float>(tall_qr ? b * n * n : 0);
  w.UBq = c.take<float>(tall_qr ? b * n * n : 0);
  const bool route = dc && dc_route(p);
  w.dc = c.take_bytes(route ? dc_ws_bytes(p) : 0);
  w.dsgn = c.take<float>(route ? n : 0);
  w.dperm = c.take<int>(route ? n : 0);
  if (total) *total = c.off;
  return w;
}

GemmArgs gemm_base(int M, int N, int K, int batch) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.alpha = 1.f; g.beta = 0.f;
  return g;
}

struct Ctx {
  svdp_handle* h;
  const svdp_params* p;
  FwdWs w;
  hipStream_t st;
  int batch, m, n;
  const float* A;
  int64_t lda, sA;
  int feat_m = 0;  // rows the sketch features report (0: m); the QR path's square core
                   // reports the tall input's, whose spectrum and power sequence it shares
};

// Host synchronisations made by the library (svdp_host_syncs): the
// forward passes read a device count back only for the bounded paths'
// fallback test and the blocked QR step (n > 512).
std::atomic<int64_t> g_host_syncs{0};

svdp_status read_counter(Ctx& c, const int* dev, int* out) {
  HIPCHK(hipMemcpyAsync(c.h->host_word, dev, sizeof(int), hipMemcpyDeviceToHost, c.st), "counter copy");
  HIPCHK(hipStreamSynchronize(c.st), "counter sync");
  g_host_syncs.fetch_add(1);
  *out = *c.h->host_word;
  return SVDP_OK;
}

// One CANS step on buffers (Xc -> Xn): G = Xc^T Xc, Xn = alpha Xc + beta Xc G.
// With ksched, matrix b takes part only if its step kidx has category kcat
// (sched_cat over the per-matrix counts (K, K1)).
// One CANS step on buffers (Xc -> Xn): G = Xc^T Xc, Xn = alpha Xc + beta Xc G.
// With ksched (the bounded schedule), matrix b takes part only if the
// category of its step kidx is in kcatmask, and its output goes to Xn_bf
// (BF16, with its transpose in Xtn) when that category's bit is set in
// obf_catmask, else to Xn.  Xtc: the BF16 transpose of a BF16 Xc (n x m),
// from which the Gram reads both operands contiguous in k.
hipError_t cans_step(Ctx& c, int prec, const void* Xc, void* Xn, int in_bf16, int out_bf16,
                     const float* coef, int64_t coef_bstride, int kidx, const int* active,
                     float* conv, const int* ksched = nullptr, int kcatmask = 0, int obf_catmask = 0,
                     int kbf16 = 0, const void* Xtc = nullptr, void* Xn_bf = nullptr, void* Xtn = nullptr) {
  const int m = c.m, n = c.n, B = c.batch;
  GemmArgs g = gemm_base(n, n, m, B);
  g.C = c.w.G; g.ldc = n; g.sC = (int64_t)n * n;
  g.sym = 1;
  g.active = active;
  g.ksched = ksched; g.kstep = kidx; g.kcatmask = kcatmask; g.kbf16 = kbf16;
  g.in_bf16 = in_bf16;
  g.out_bf16 = prec == PREC_BF16 ? 1 : 0;
  hipError_t e;
  if (in_bf16 && Xtc) {
    // G = (X^T)(X^T)^T: op(A) = X^T stored n x m, op(B) = X stored as X^T
    g.A = Xtc; g.lda = m; g.sA = (int64_t)m * n;
    g.B = Xtc; g.ldb = m; g.sB = (int64_t)m * n;
    e = gemm_launch(g, prec, 0, 1, c.st);
  } else {
    g.A = Xc; g.lda = n; g.sA = (int64_t)m * n;
    g.B = Xc; g.ldb = n; g.sB = (int64_t)m * n;
    e = gemm_launch(g, prec, 1, 0, c.st);
  }
  if (e) return e;
  GemmArgs u = gemm_base(m, n, n, B);
  u.A = Xc; u.lda = n; u.sA = (int64_t)m * n;
  // G is symmetric: read it as B^T (k-contiguous rows) for the BF16 kernel
  u.B = c.w.G; u.ldb = n; u.sB = (int64_t)n * n;
  u.C = Xn; u.ldc = n; u.sC = (int64_t)m * n;
  u.Cin = Xc; u.ldcin = n; u.sCin = (int64_t)m * n; u.cin_bf16 = in_bf16;
  u.coef = coef; u.coef_bstride = coef_bstride; u.coef_idx = kidx;
  u.active = active;
  u.ksched = ksched; u.kstep = kidx; u.kcatmask = kcatmask; u.kbf16 = kbf16;
  u.obf_catmask = obf_catmask; u.C_bf = Xn_bf;
  u.conv = conv;
  u.in_bf16 = in_bf16;
  u.out_bf16 = out_bf16;
  if (Xtn) { u.Ct = Xtn; u.ldct = m; u.sCt = (int64_t)m * n; }
  return gemm_launch(u, prec, 0, prec == PREC_BF16 ? 1 : 0, c.st);
}

// One quintic step (FP32): G = Xc^T Xc, P = c5 G G + c3 G, Xn = c1 Xc + Xc P,
// with the change sums of the stop test from the last product.
hipError_t cans5_step(Ctx& c, const float* Xc, float* Xn, const double* cf, const int* active, float* conv) {
  const int m = c.m, n = c.n, B = c.batch;
  GemmArgs g = gemm_base(n, n, m, B);
  g.A = Xc; g.lda = n; g.sA = (int64_t)m * n;
  g.B = Xc; g.ldb = n; g.sB = (int64_t)m * n;
  g.C = c.w.G; g.ldc = n; g.sC = (int64_t)n * n;
  g.sym = 1;
  g.active = active;
  hipError_t e = gemm_launch(g, PREC_F32, 1, 0, c.st);
  if (e) return e;
  GemmArgs q = gemm_base(n, n, n, B);
  q.A = c.w.G; q.lda = n; q.sA = (int64_t)n * n;
  q.B = c.w.G; q.ldb = n; q.sB = (int64_t)n * n;
  q.C = c.w.P; q.ldc = n; q.sC = (int64_t)n * n;
  q.Cin = c.w.G; q.ldcin = n; q.sCin = (int64_t)n * n;
  q.alpha = (float)cf[2]; q.beta = (float)cf[1];
  q.sym = 1;
  q.active = active;
  if ((e = gemm_launch(q, PREC_F32, 0, 0, c.st))) return e;
  GemmArgs u = gemm_base(m, n, n, B);
  u.A = Xc; u.lda = n; u.sA = (int64_t)m * n;
  u.B = c.w.P; u.ldb = n; u.sB = (int64_t)n * n;
  u.C = Xn; u.ldc = n; u.sC = (int64_t)m * n;
  u.Cin = Xc; u.ldcin = n; u.sCin = (int64_t)m * n;
  u.alpha = 1.f; u.beta = (float)cf[0];
  u.active = active;
  u.conv = conv;
  return gemm_launch(u, PREC_F32, 0, 0, c.st);
}

// Conservative CANS in FP32 with per-matrix stopping (mask: matrices to run,
// null = all): Algorithm 3 scaling, pre_iters preprocessing steps, then the
// interval recursion from [1 - delta, 1 + delta] until the relative change is
// below tol.  Leaves W of matrix b in X0 (where[b] = 0) or X1 (where[b] = 1).
svdp_status conservative_fp32(Ctx& c, const int* mask) {
  const svdp_params* p = c.p;
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  ProfScope phase_bound(PROF_PHASE_BOUND, c.st);
  HIPCHK(norms_launch(c.A, c.lda, c.sA, B, m, n, w.colsum, w.rowmax, w.fro2, w.fpart, w.flags, mask, c.st),
         "norms");
  if (p->poly == SVDP_POLY_PE)
    HIPCHK(fro_scale_launch(w.fro2, B, w.scale, mask, c.st), "scale");
  else
    HIPCHK(ns_scale_launch(w.colsum, w.rowmax, B, n, w.scale, mask, c.st), "scale");
  HIPCHK(scale_copy_launch(c.A, c.lda, c.sA, B, m, n, w.scale, w.X0, 0, mask, c.st), "normalise");
  phase_bound.next(PROF_PHASE_CANS);
  double tab[128], tab3[3 * 64];
  if (p->poly == SVDP_POLY_PE) {
    // a fixed schedule without stop test (the 1.01 damping holds the
    // iterate on a plateau short of convergence until the last step)
    const int T = pe_table(p->pe_lo, p->max_iters, tab3);
    if (T < 0) return fail(SVDP_ERR_INVALID_ARG, "Polar Express schedule longer than max_iters");
    if (mask) HIPCHK(copy_i32(w.active, mask, B, c.st), "active");
    else HIPCHK(fill_i32(w.active, 1, B, c.st), "active");
    for (int k = 0; k < T; ++k) {
      const float* Xc = (k & 1) ? w.X1 : w.X0;
      float* Xn = (k & 1) ? w.X0 : w.X1;
      HIPCHK(cans5_step(c, Xc, Xn, tab3 + 3 * k, w.active, nullptr), "pe step");
    }
    HIPCHK(fill_masked_launch(w.where, T & 1, B, mask, c.st), "where");
    HIPCHK(fill_masked_launch(w.iters, T, B, mask, c.st), "iters");
    return SVDP_OK;
  }
  table_poly(p->poly, p->delta, p->pre_iters, p->max_iters, tab3, nullptr);
  for (int k = 0; k < p->max_iters; ++k) { tab[2 * k] = tab3[3 * k]; tab[2 * k + 1] = tab3[3 * k + 1]; }
  HIPCHK(set_coef_launch(w.coef, tab, p->max_iters, c.st), "coef");
  if (mask) HIPCHK(copy_i32(w.active, mask, B, c.st), "active");
  else HIPCHK(fill_i32(w.active, 1, B, c.st), "active");
  HIPCHK(fill_masked_launch(w.where, 0, B, mask, c.st), "where");
  // The full budget of max_iters steps is enqueued without reading anything
  // back: a matrix leaves the active set on the device at its stop test, and
  // the later steps' workgroups of that matrix exit at once.
  for (int k = 0; k < p->max_iters; ++k) {
    const float* Xc = (k & 1) ? w.X1 : w.X0;
    float* Xn = (k & 1) ? w.X0 : w.X1;
    if (p->poly == SVDP_POLY_CANS5)
      HIPCHK(cans5_step(c, Xc, Xn, tab3 + 3 * k, w.active, w.conv), "cans5 step");
    else
      HIPCHK(cans_step(c, PREC_F32, Xc, Xn, 0, 0, w.coef, 0, k, w.active, w.conv), "cans step");
    HIPCHK(cans_check_launch(B, w.conv, gemm_conv_slots(m, n), (float)p->tol, k, w.active, w.where, w.iters,
                             nullptr, 0, w.flags,
                             w.counter, c.st),
           "cans check");
  }
  // still active after max_iters: not converged
  HIPCHK(or_flags_launch(B, w.flags, SVDP_FLAG_NOT_CONVERGED, w.active, c.st), "flags");
  return SVDP_OK;
}

// Bounded path: learned (sketch features -> MLP) or user bounds give a
// per-matrix scale and interval [lo, 1]; each matrix takes its own number K
// of interval-optimal steps (to the BF16 hand-off error) in `prec`, then FP32
// refinement with the stop test.  Result in X0 / X1 as where[] says.
svdp_status bounded(Ctx& c) {
  const svdp_params* p = c.p;
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  const int kcap = std::min(p->max_iters, 64);
  ProfScope phase(PROF_PHASE_BOUND, c.st);
  if (p->bound == SVDP_BOUND_LEARNED) {
    // features: |A|_F^2 via the row pass, then the alternating power sequence
    HIPCHK(norms_launch(c.A, c.lda, c.sA, B, m, n, w.colsum, w.rowmax, w.fro2, w.fpart, w.flags, nullptr,
                        c.st), "norms");
    HIPCHK(vnorm_launch(p->probe, n, B, n, w.nrm, 0, c.st), "probe norm");
    const float* x = p->probe;
    int64_t sx = n;
    for (int k = 1; k <= 7; ++k) {
      float* y = (k & 1) ? w.y0 : w.y1;
      int trans = (k & 1) ? 0 : 1;
      int len = trans ? n : m;
      HIPCHK(matvec_launch(c.A, c.lda, c.sA, B, m, n, x, sx, y, m, trans, w.fro2, c.st), "matvec");
      HIPCHK(vnorm_launch(y, m, B, len, w.nrm, k, c.st), "vnorm");
      x = y;
      sx = m;
    }
    HIPCHK(features_launch(w.fro2, w.nrm, B, c.feat_m ? c.feat_m : m, n, w.F, w.aux, c.st), "features");
    HIPCHK(mlp_fwd_launch(c.h->model, c.h->model + SVDP_MLP_PARAMS, c.h->model + SVDP_MLP_PARAMS + 8, w.F, B,
                          w.mlpout, nullptr, c.st), "mlp");
    HIPCHK(bounds_launch(B, 0, w.mlpout, w.aux, nullptr, p->margin_max, p->margin_min, p->bf16_handoff,
                         p->bf16_from, kcap, w.scale, w.coef, w.ksteps, nullptr, c.st), "bounds");
  } else {
    HIPCHK(bounds_launch(B, 1, nullptr, nullptr, p->user_bounds, p->margin_max, p->margin_min, p->bf16_handoff,
                         p->bf16_from, kcap, w.scale, w.coef, w.ksteps, nullptr, c.st), "bounds");
  }
  // Every matrix runs its own schedule: K interval-optimal steps, the first
  // K1 in FP32 (while small singular values are still small: BF16 rounding
  // would rotate their singular vectors), the rest in BF16.  Step k runs as
  // one batch-wide launch per category of step (FP32 or BF16 in, FP32 or
  // BF16 out); the GEMMs skip the matrices of other categories.  The
  // iterate after step k lives in X[k % 2] (FP32) or Y[k % 2] (BF16).  The
  // host reads the per-step category counts (one synchronisation).
  // No read-back: the host enqueues a budget of steps that covers every
  // matrix's K -- the number of steps from the smallest interval the bound
  // kernel produces (kLoFloor) to the hand-off -- and each launch skips the
  // matrices whose schedule has no step of its kind at k.
  const int bf16 = p->precision == SVDP_PREC_BF16;
  const int kbudget = std::min(kcap, bounded_budget(p->bf16_handoff));
  HIPCHK(sched_mask_launch(B, w.ksteps, bf16, 0, w.gmask, c.st), "fp32 start");
  HIPCHK(scale_copy_launch(c.A, c.lda, c.sA, B, m, n, w.scale, w.X0, 0, w.gmask, c.st), "normalise");
  if (bf16) {
    HIPCHK(sched_mask_launch(B, w.ksteps, bf16, 1, w.gmask, c.st), "bf16 start");
    HIPCHK(scale_copy_launch(c.A, c.lda, c.sA, B, m, n, w.scale, w.Y0, 1, w.gmask, c.st), "normalise");
    HIPCHK(transpose_bf16_launch(w.Y0, B, m, n, w.Yt0, w.gmask, c.st), "transpose");
  }
  phase.next(PROF_PHASE_CANS);
  // Step k runs as one launch pair for FP32 input (categories 0: FP32 out,
  // 1: BF16 out) and, on the BF16 path, one for BF16 input (2: BF16 out, 3:
  // FP32 out); the iterate after step k is in X[k % 2] (FP32) or Y[k % 2]
  // (BF16, with its transpose in Yt[k % 2]).
  for (int k = 0; k < kbudget; ++k) {
    void* Xn = ((k + 1) & 1) ? w.X1 : w.X0;
    void* Yn = ((k + 1) & 1) ? w.Y1 : w.Y0;
    void* Ytn = bf16 ? (((k + 1) & 1) ? w.Yt1 : w.Yt0) : nullptr;
    HIPCHK(cans_step(c, PREC_F32, (k & 1) ? w.X1 : w.X0, Xn, 0, 0, w.coef, kcap, k, nullptr, nullptr, w.ksteps,
                     (1 << 0) | (1 << 1), 1 << 1, bf16, nullptr, Yn, Ytn), "cans step");
    if (bf16)
      HIPCHK(cans_step(c, PREC_BF16, (k & 1) ? w.Y1 : w.Y0, Xn, 1, 0, w.coef, kcap, k, nullptr, nullptr, w.ksteps,
                       (1 << 2) | (1 << 3), 1 << 2, bf16, (k & 1) ? w.Yt1 : w.Yt0, Yn, Ytn), "cans step");
  }
  // the last iterate of a matrix with K odd is in X1: move it to X0
  HIPCHK(sched_mask_launch(B, w.ksteps, bf16, 2, w.gmask, c.st), "odd mask");
  HIPCHK(copy_masked_launch(w.X1, w.X0, B, (int64_t)m * n, w.gmask, c.st), "to X0");
  HIPCHK(sched_iters_launch(B, w.ksteps, w.iters, c.st), "iters");
  // FP32 refinement of the whole batch from X0: interval-optimal steps from
  // the hand-off interval (tending to the Newton-Schulz cubic), at least
  // refine_steps of them, then per matrix until the relative change is below
  // tol.  A matrix whose predicted interval missed part of its spectrum is
  // still caught here; one that has not converged within refine_steps +
  // kRefineExtra steps is flagged and falls back to conservative CANS.  The
  // whole budget is enqueued; converged matrices are skipped on the device.
  phase.next(PROF_PHASE_REFINE);
  const int R = p->refine_steps;
  const int Rmax = std::min(R + kRefineExtra, 64);
  double rtab[128];
  const double hoff = std::min(std::max(p->bf16_handoff, 1e-8), 0.5);
  table_interval(1.0 - hoff, Rmax, rtab);
  HIPCHK(set_coef_launch(w.rcoef, rtab, Rmax, c.st), "refine coef");
  HIPCHK(fill_i32(w.active, 1, B, c.st), "active");
  HIPCHK(fill_i32(w.where, 0, B, c.st), "where");
  // the reported count adds the refinement steps to each matrix's K (mask
  // is free until the fallback test)
  HIPCHK(copy_i32(w.mask, w.iters, B, c.st), "iteration base");
  for (int r = 0; r < Rmax; ++r) {
    const float* Xc = (r & 1) ? w.X1 : w.X0;
    float* Xn = (r & 1) ? w.X0 : w.X1;
    // the first R - 1 steps are unconditional: no change sums, no check
    float* conv = r + 1 >= R ? w.conv : nullptr;
    HIPCHK(cans_step(c, PREC_F32, Xc, Xn, 0, 0, w.rcoef, 0, r, w.active, conv), "refine step");
    if (!conv) continue;
    HIPCHK(cans_check_launch(B, w.conv, gemm_conv_slots(m, n), (float)p->tol, r, w.active, w.where, w.iters,
                             w.mask, 1, w.flags,
                             w.counter, c.st), "refine check");
  }
  HIPCHK(or_flags_launch(B, w.flags, SVDP_FLAG_NOT_CONVERGED, w.active, c.st), "flags");
  return SVDP_OK;
}

// residual |W^T W - I|_F / sqrt(n) of the final iterate (Gram into G)
svdp_status final_residual(Ctx& c, const int* mask) {
  ProfScope phase(PROF_PHASE_REFINE, c.st);
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  GemmArgs g = gemm_base(n, n, m, B);
  g.A = w.X0; g.A_alt = w.X1; g.a_sel = w.where; g.lda = n; g.sA = (int64_t)m * n;
  g.B = w.X0; g.B_alt = w.X1; g.b_sel = w.where; g.ldb = n; g.sB = (int64_t)m * n;
  g.C = w.G; g.ldc = n; g.sC = (int64_t)n * n;
  g.sym = 1;
  g.active = mask;
  HIPCHK(gemm_launch(g, PREC_F32, 1, 0, c.st), "W^T W");
  HIPCHK(residual_launch(w.G, 0, B, n, w.rpart, w.resid, mask, c.st), "residual");
  return SVDP_OK;
}

// H = W^T A (full; the eigensolver and the polar output symmetrise it) into G
svdp_status form_h(Ctx& c, const int* mask) {
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  GemmArgs g = gemm_base(n, n, m, B);
  g.A = w.X0; g.A_alt = w.X1; g.a_sel = w.where; g.lda = n; g.sA = (int64_t)m * n;
  g.B = c.A; g.ldb = c.lda; g.sB = c.sA;
  g.C = w.G; g.ldc = n; g.sC = (int64_t)n * n;
  g.active = mask;
  HIPCHK(gemm_launch(g, PREC_F32, 1, 0, c.st), "H = W^T A");
  return SVDP_OK;
}

// CANS polar factor of every matrix (Algorithm 1 steps 1-3).
svdp_status polar_core(Ctx& c) {
  const svdp_params* p = c.p;
  FwdWs& w = c.w;
  const int B = c.batch;
  HIPCHK(fill_i32(w.flags, 0, B, c.st), "flags");
  HIPCHK(fill_i32(w.iters, 0, B, c.st), "iters");
  HIPCHK(fill_i32(w.sweeps, 0, B, c.st), "sweeps");
  HIPCHK(fill_f32(w.resid, 0.f, B, c.st), "resid");
  svdp_status s = p->bound == SVDP_BOUND_CONSERVATIVE ? conservative_fp32(c, nullptr) : bounded(c);
  if (s) return s;
  return final_residual(c, nullptr);
}

// Blocked QR of U for the flagged matrices (n > kQrBlockedFrom): columns
// without direction (sigma_j <= eps_qr sigma_1) are replaced by pseudo-random
// unit vectors and other deficient columns perturbed by eps_qr-sized ones;
// then for each
// block of kQrBlock columns, twice C = U[:, :c0]^T U[:, blk] and
// U[:, blk] -= U[:, :c0] C (block Gram-Schmidt), and twice G = U[:, blk]^T
// U[:, blk], U[:, blk] <- U[:, blk] Rinv (CholeskyQR with column scaling).
// The R factor this implies has a positive diagonal.
// The block loop of the blocked QR on the matrices of qmask: for each block
// of kQrBlock columns, twice C = U[:, :c0]^T U[:, blk] and U[:, blk] -=
// U[:, :c0] C (block Gram-Schmidt), and twice G = U[:, blk]^T U[:, blk],
// U[:, blk] <- U[:, blk] Rinv (CholeskyQR with column scaling).  With
// zero_dep, columns dependent on the earlier ones come out as zero columns.
svdp_status qr_blocks(Ctx& c, float* U, int64_t ldu, int64_t sU, const int* qmask, int zero_dep) {
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  for (int c0 = 0; c0 < n; c0 += kQrBlock) {
    const int bc = std::min(kQrBlock, n - c0);
    for (int pass = 0; c0 > 0 && pass < 2; ++pass) {
      GemmArgs g = gemm_base(c0, bc, m, B);  // C = U[:, :c0]^T U[:, c0:c0+bc]
      g.A = U; g.lda = ldu; g.sA = sU;
      g.B = U + c0; g.ldb = ldu; g.sB = sU;
      g.C = w.qrc; g.ldc = bc; g.sC = (int64_t)n * kQrBlock;
      g.active = qmask;
      HIPCHK(gemm_launch(g, PREC_F32, 1, 0, c.st), "qr project");
      GemmArgs u = gemm_base(m, bc, c0, B);  // U[:, blk] = U[:, blk] - U[:, :c0] C
      u.A = U; u.lda = ldu; u.sA = sU;
      u.B = w.qrc; u.ldb = bc; u.sB = (int64_t)n * kQrBlock;
      u.C = U + c0; u.ldc = ldu; u.sC = sU;
      u.Cin = U + c0; u.ldcin = ldu; u.sCin = sU;
      u.alpha = -1.f; u.beta = 1.f;
      u.active = qmask;
      HIPCHK(gemm_launch(u, PREC_F32, 0, 0, c.st), "qr update");
    }
    for (int pass = 0; pass < 2; ++pass) {
      GemmArgs g = gemm_base(bc, bc, m, B);  // G = U[:, blk]^T U[:, blk]
      g.A = U + c0; g.lda = ldu; g.sA = sU;
      g.B = U + c0; g.ldb = ldu; g.sB = sU;
      g.C = w.qrg; g.ldc = bc; g.sC = (int64_t)kQrBlock * kQrBlock;
      g.sym = 1; g.active = qmask;
      HIPCHK(gemm_launch(g, PREC_F32, 1, 0, c.st), "qr gram");
      HIPCHK(qr_chol_launch(w.qrg, w.qrr, B, bc, qmask, zero_dep, c.st), "qr chol");
      // in place: each workgroup reads the rows of U[:, blk] it writes, and
      // K = bc is consumed before its epilogue
      GemmArgs r = gemm_base(m, bc, bc, B);  // U[:, blk] <- U[:, blk] Rinv
      r.A = U + c0; r.lda = ldu; r.sA = sU;
      r.B = w.qrr; r.ldb = bc; r.sB = (int64_t)kQrBlock * kQrBlock;
      r.C = U + c0; r.ldc = ldu; r.sC = sU;
      r.active = qmask;
      HIPCHK(gemm_launch(r, PREC_F32, 0, 0, c.st), "qr scale");
    }
  }
  return SVDP_OK;
}

// Blocked QR of U for the flagged matrices (n > kQrBlockedFrom): columns
// without direction (sigma_j <= eps_qr sigma_1) are replaced by pseudo-random
// unit vectors and other deficient columns perturbed by eps_qr-sized ones;
// then the block loop of qr_blocks.  The R factor this implies has a
// positive diagonal.
svdp_status qr_blocked(Ctx& c, float* U, int64_t ldu, int64_t sU, const float* S, int64_t sS, const int* mask) {
  const svdp_params* p = c.p;
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  HIPCHK(qr_mask_launch(B, w.flags, mask, w.qmask, w.counter, c.st), "qr mask");
  int flagged = 0;
  svdp_status s = read_counter(c, w.counter, &flagged);
  if (s || flagged == 0) return s;
  HIPCHK(qr_perturb_launch(U, ldu, sU, B, m, n, S, sS, w.colsum, (float)p->eps_qr, w.qmask, c.st), "qr perturb");
  return qr_blocks(c, U, ldu, sU, w.qmask, 0);
}

// Algorithm 1's column-norm test on U and its QR step for the flagged
// matrices (one workgroup per matrix up to kQrBlockedFrom columns, blocked
// above).
svdp_status u_qr_step(Ctx& c, float* U, int64_t ldu, int64_t sU, const float* S, int64_t sS, const int* mask) {
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  HIPCHK(colnorm_check_launch(U, ldu, sU, B, m, n, w.colsum, (float)c.p->eps_qr, w.flags, mask, c.st), "colnorm");
  if (n <= kQrBlockedFrom) {
    HIPCHK(qr_complete_launch(U, ldu, sU, B, m, n, (float)c.p->eps_qr, w.flags, w.qr, mask, c.st), "qr");
    return SVDP_OK;
  }
  return qr_blocked(c, U, ldu, sU, S, sS, mask);
}

// H, eigh(H), U = W V with eigenvalue signs, column-norm test (Algorithm 1
// steps 4-7) for every matrix or the masked ones.
svdp_status svd_tail(Ctx& c, float* U, int64_t ldu, int64_t sU, float* S, int64_t sS, float* V,
                     int64_t ldv, int64_t sV, const int* mask) {
  const svdp_params* p = c.p;
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  ProfScope phase(PROF_PHASE_H, c.st);
  svdp_status s = form_h(c, mask);
  if (s) return s;
  phase.next(PROF_PHASE_EIGH);
  if (!mask && B == 1 && dc_route(p)) {
    // one large FP32 matrix: H = V diag(lam) V^T by divide and conquer, then
    // the Jacobi's mode-1 order (|lam| descending, signs kept for U)
    if ((s = svd_eigh_dc(c.h, p, w.dc, w.G, S, V, ldv, w.sweeps, w.flags, c.st))) return s;
    HIPCHK(dc_abs_order_launch(S, V, ldv, n, w.dsgn, w.dperm, eigh_opts(p).neg_tol, w.flags, c.st), "dc order");
    phase.next(PROF_PHASE_U);
    GemmArgs g = gemm_base(m, n, n, B);
    g.A = w.X0; g.A_alt = w.X1; g.a_sel = w.where; g.lda = n; g.sA = (int64_t)m * n;
    g.B = V; g.ldb = ldv; g.sB = sV;
    g.C = U; g.ldc = ldu; g.sC = sU;
    g.colscale = w.dsgn; g.cs_stride = n;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 0, c.st), "U = W V");
    return u_qr_step(c, U, ldu, sU, S, sS, nullptr);
  }
  EighWs e = eigh_ws_carve(w.eigh, B, n, p->max_sweeps);
  HIPCHK(eigh_run(e, w.G, n, (int64_t)n * n, 1, eigh_opts(p), S, sS, V, ldv, sV, w.sweeps, w.flags,
                  mask, &c.h->aux, c.st), "eigh");
  phase.next(PROF_PHASE_U);
  // B operand of U = W V: V, or V Mu after the BF16 correction
  const float* Vb = V;
  int64_t ldvb = ldv, svb = sV;
  if (p->bf16_correct && p->precision == SVDP_PREC_BF16 && !mask) {
    // First-order correction of the BF16-rounded polar factor (the bounded
    // path's first pass; its fallback reruns are FP32).  P = V^T (W^T A) V is
    // the eigensolver's last restart measure T (in Vw, working order, read
    // through perm); polar_fix gives Mu and the corrected singular values;
    // U = W (V Mu) and V <- V (2 I - Mu) = 2 V - V Mu.  Scratch: the
    // eigensolver's other working copies (np >= n), free once it returned.
    const int64_t n2 = (int64_t)n * n, np2 = (int64_t)e.np * e.np;
    // P and then Mu in Hw, P^T in V2, diag(P) in y0 (batch x m >= n)
    HIPCHK(polar_fix_launch(e.Vw, e.np, np2, e.perm, S, sS, e.sgn, 0, B, n, e.Hw, e.V2, w.y0, w.colsum,
                            nullptr, c.st), "polar fix");
    GemmArgs vu = gemm_base(n, n, n, B);  // V Mu
    vu.A = V; vu.lda = ldv; vu.sA = sV;
    vu.B = e.Hw; vu.ldb = n; vu.sB = n2;
    vu.C = e.V2; vu.ldc = n; vu.sC = n2;
    HIPCHK(gemm_launch(vu, PREC_F32, 0, 0, c.st), "V Mu");
    HIPCHK(vcorr_launch(V, ldv, sV, e.V2, B, n, c.st), "V");
    HIPCHK(sigma_store_launch(w.colsum, n, S, sS, B, nullptr, c.st), "sigma");
    Vb = e.V2; ldvb = n; svb = n2;
  }
  GemmArgs g = gemm_base(m, n, n, B);
  g.A = w.X0; g.A_alt = w.X1; g.a_sel = w.where; g.lda = n; g.sA = (int64_t)m * n;
  g.B = Vb; g.ldb = ldvb; g.sB = svb;
  g.C = U; g.ldc = ldu; g.sC = sU;
  g.colscale = e.sgn; g.cs_stride = n;
  g.active = mask;
  HIPCHK(gemm_launch(g, PREC_F32, 0, 0, c.st), "U = W V");
  // Algorithm 1: a column norm off by more than eps_qr (rank deficiency)
  // -> orthogonalise U by QR
  return u_qr_step(c, U, ldu, sU, S, sS, mask);
}

svdp_status check_model(svdp_handle* h, const svdp_params* p) {
  if (p->bound == SVDP_BOUND_LEARNED) {
    if (!h->has_model) return fail(SVDP_ERR_NO_MODEL, "learned bounds need svdp_set_model first");
    if (!p->probe) return fail(SVDP_ERR_INVALID_ARG, "learned bounds need params.probe");
  }
  if (p->bound == SVDP_BOUND_USER && !p->user_bounds)
    return fail(SVDP_ERR_INVALID_ARG, "user bounds need params.user_bounds");
  return SVDP_OK;
}

// Fallback of the bounded paths: matrices with a residual above refine_tol,
// an unconverged refinement, a negative eigenvalue of H or non-finite
// values rerun conservative CANS.
svdp_status fallback_mask(Ctx& c, int* count) {
  FwdWs& w = c.w;
  HIPCHK(fallback_mask_launch(c.batch, w.flags,
                              SVDP_FLAG_NEG_EIGENVALUE | SVDP_FLAG_NONFINITE | SVDP_FLAG_NOT_CONVERGED, w.resid,
                              (float)c.p->refine_tol, w.mask, w.counter, c.st), "fallback mask");
  return read_counter(c, w.counter, count);
}

// Algorithm 1 on the matrices of the context: the polar factor, H, eigh, U,
// and the conservative reruns of the bounded paths.
svdp_status svd_core(Ctx& c, float* U, int64_t ldu, int64_t sU, float* S, int64_t sS, float* V, int64_t ldv,
                     int64_t sV) {
  svdp_status s;
  if ((s = polar_core(c))) return s;
  if ((s = svd_tail(c, U, ldu, sU, S, sS, V, ldv, sV, nullptr))) return s;
  if (c.p->bound != SVDP_BOUND_CONSERVATIVE) {
    int cnt = 0;
    if ((s = fallback_mask(c, &cnt))) return s;
    if (cnt > 0) {
      ProfScope phase(PROF_PHASE_FALLBACK, c.st);
      const int* mk = c.w.mask;
      if ((s = conservative_fp32(c, mk))) return s;
      if ((s = final_residual(c, mk))) return s;
      if ((s = svd_tail(c, U, ldu, sU, S, sS, V, ldv, sV, mk))) return s;
      HIPCHK(or_flags_launch(c.batch, c.w.flags, SVDP_FLAG_FALLBACK_USED, mk, c.st), "flags");
    }
  }
  return SVDP_OK;
}

// ---------------------------------------------------------------- spectral divide and conquer

// The polar step of the split: one n x n matrix, conservative FP32 CANS with
// the caller's CANS settings.
svdp_params dc_polar_params(const svdp_params* p) {
  svdp_params q = *p;
  q.batch = 1;
  q.m = p->n;
  q.bound = SVDP_BOUND_CONSERVATIVE;
  q.precision = SVDP_PREC_FP32;
  q.poly = SVDP_POLY_CANS3;
  q.probe = nullptr;
  q.user_bounds = nullptr;
  q.tall_qr = 0;
  return q;
}

// Pieces of at most kDcLeafMax go to one batched Jacobi solve; larger ones
// are split again, down to kDcDepth levels (so at most kDcLeaves pieces).
constexpr int kDcLeafMax = 1024;
constexpr int kDcDepth = 4;
constexpr int kDcLeaves = 1 << kDcDepth;

struct DcWs {
  void* polar;              // the polar step's forward workspace (for n)
  void* polar2;             // ... and that of the first basis's polar factors
  float *A, *Om, *HQ;       // n x n temporaries of one split
  float *cs, *sigma, *mu;   // mu: each leaf's shift
  double *part, *cpl;
  int *k, *sw, *fl, *map, *sweeps, *flags;
  float* pool;              // Q, T, W of every split piece (bump-allocated)
  size_t pool_floats;
  float *Hl, *Vl, *laml;    // the batched leaf solve: up to leaf_count zero-padded pieces
  int leaf_n;               // their largest size, min(n, kDcLeafMax)
  int leaf_count;           // 2 when n <= kDcLeafMax (only the first split happens), else kDcLeaves
  void* eigh;               // eigensolver workspace for one n x n matrix
  void* eigh_leaf;          // ... for kDcLeaves matrices of leaf_n
};

DcWs carve_dc(void* base, const svdp_params* p, size_t* total) {
  svdp_params q = dc_polar_params(p);
  size_t fw = 0;
  carve_fwd(nullptr, &q, &fw, false);
  Carver c(base);
  DcWs w;
  const size_t n = p->n, nn = n * n;
  const size_t L = std::min<size_t>(n, kDcLeafMax);
  w.polar = c.take_bytes(fw);
  w.polar2 = c.take_bytes(fw);
  w.A = c.take<float>(nn);
  w.Om = c.take<float>(nn);
  w.HQ = c.take<float>(nn);
  w.cs = c.take<float>(n);
  w.sigma = c.take<float>(1);
  w.mu = c.take<float>(kDcLeaves);
  w.part = c.take<double>(2 * n);
  w.cpl = c.take<double>(6);
  w.k = c.take<int>(1);
  w.sw = c.take<int>(kDcLeaves);
  w.fl = c.take<int>(kDcLeaves);
  w.map = c.take<int>(L);
  w.sweeps = c.take<int>(p->batch);
  w.flags = c.take<int>(p->batch);
  // the split pieces at one depth are disjoint, so their sizes s_i add up to
  // at most n and their s_i^2 to at most n^2: 3 n^2 per level, plus alignment
  w.pool_floats = 3 * nn * kDcDepth + 3 * 64 * kDcLeaves;
  w.pool = c.take<float>(w.pool_floats);
  w.leaf_n = (int)L;
  w.leaf_count = n <= (size_t)kDcLeafMax ? 2 : kDcLeaves;
  const size_t LC = w.leaf_count;
  w.Hl = c.take<float>(LC * L * L);
  w.Vl = c.take<float>(LC * L * L);
  w.laml = c.take<float>(LC * L);
  w.eigh = c.take_bytes(eigh_ws_bytes(1, n, p->max_sweeps));
  w.eigh_leaf = c.take_bytes(eigh_ws_bytes(LC, L, p->max_sweeps));
  if (total) *total = c.off;
  return w;
}

size_t dc_ws_bytes(const svdp_params* p) {
  svdp_params q = *p;
  q.batch = 1;
  size_t total = 0;
  carve_dc(nullptr, &q, &total);
  return total;
}

svdp_status read_doubles(svdp_handle* h, hipStream_t st, const double* dev, int count, double* out) {
  HIPCHK(hipMemcpyAsync(h->host_word, dev, count * sizeof(double), hipMemcpyDeviceToHost, st), "read copy");
  HIPCHK(hipStreamSynchronize(st), "read sync");
  g_host_syncs.fetch_add(1);
  std::memcpy(out, h->host_word, count * sizeof(double));
  return SVDP_OK;
}

// One piece of the divide and conquer: the symmetric s x s input M (pitch
// ldm), whose eigenvalues go to lam[off, off + s) and eigenvectors to V
// (s x s, pitch ldv).  A split piece keeps Q (its basis), T = Q^T M Q and W
// (the eigenvectors of T's two diagonal blocks, block-diagonal).
struct DcPiece {
  int off, s, k, depth;
  const float* M;
  int64_t ldm;
  float* V;
  int64_t ldv;
  float *Q, *T, *W;
  bool split;
};

// The split of one piece by the sign of M - sigma I (sigma = trace(M) / s,
// M taken as its symmetric part (M + M^T) / 2), the polar factor W of that
// shifted matrix: P = (I + W) / 2 projects onto the eigenvectors with
// eigenvalues above sigma and has rank k = (s + trace W) / 2.  An
// orthonormal basis Q = [Q1 Q2] of range(P) and its complement comes from
// Y = [P X1, (I - P) X2] twice: first with X = Om (seeded random), its two
// blocks made orthonormal by their polar factors (the second block after
// two projections against the first's); then once more with X = that basis
// (one step of subspace iteration: the first Y can be badly conditioned and
// keeps W's error in its range; the second is nearly orthonormal and squares
// that error -- W is an odd polynomial of the shifted piece, so its error is
// in its eigenvalues, and P's wrong-side eigenvalues enter squared), whose
// first k columns and then the rest, projected twice
// against them, are made orthonormal by three Newton-Schulz steps each.
// Polar factors and Newton-Schulz steps are right multiplications, so each
// block keeps its span.  Then T = Q^T M Q (made
// exactly symmetric: the polar factor of a slightly non-symmetric piece
// misplaces the directions near its sigma), block diagonal up to the
// coupling T[:k, k:], which must stay below 10 tol |T|_F.  *ok = 0 (and Q, T
// unused) when the piece does not split: k = 0 or s, the polar iteration
// unconverged or non-finite, |W|_F^2 off s by more than 1/2, a Newton-Schulz
// block whose last Gram matrix is off I by more than 1e-3 (Frobenius), or
// too large a coupling.
svdp_status dc_split(svdp_handle* h, const svdp_params* p, const DcWs& w, DcPiece& pc, uint32_t seed,
                     hipStream_t st, bool* ok) {
  *ok = false;
  const int s = pc.s;
  const int64_t ss = (int64_t)s * s;
  svdp_params q = dc_polar_params(p);
  q.m = q.n = s;
  HIPCHK(dc_shift_launch(pc.M, pc.ldm, w.A, s, s, w.sigma, st), "dc shift");
  Ctx c{h, &q, carve_fwd(w.polar, &q, nullptr, false), st, 1, s, s, w.A, s, ss};
  svdp_status r = polar_core(c);
  if (r) return r;
  HIPCHK(dc_coupling_launch(c.w.X0, c.w.X1, c.w.where, s, nullptr, w.part, w.cpl, st), "dc |W|_F");
  HIPCHK(dc_rank_launch(c.w.X0, c.w.X1, c.w.where, w.cpl, c.w.flags, s, w.k, st), "dc rank");
  int k = 0;
  if ((r = read_counter(c, w.k, &k))) return r;
  if (k <= 0 || k >= s) return SVDP_OK;
  HIPCHK(dc_random_launch(w.Om, ss, seed, st), "dc random");
  HIPCHK(dc_signs_launch(w.cs, s, w.k, st), "dc signs");
  // Y = (X + W X diag(cs)) / 2, cs = +1 for the first k columns
  auto range = [&](const float* X, float* Y) {
    GemmArgs g = gemm_base(s, s, s, 1);
    g.A = c.w.X0; g.A_alt = c.w.X1; g.a_sel = c.w.where; g.lda = s; g.sA = ss;
    g.B = X; g.ldb = s; g.sB = ss;
    g.C = Y; g.ldc = s; g.sC = ss;
    g.Cin = X; g.ldcin = s; g.sCin = ss;
    g.alpha = 0.5f; g.beta = 0.5f;
    g.colscale = w.cs; g.cs_stride = s;
    return gemm_launch(g, PREC_F32, 0, 0, st);
  };
  HIPCHK(range(w.Om, w.HQ), "dc range 1");
  // Y2 <- Y2 - Q1 (Q1^T Y2) for the s x (s - k) block at Y (pitch s), Q1 the
  // first k columns of pc.Q
  auto project = [&](float* Y2) -> hipError_t {
    GemmArgs g = gemm_base(k, s - k, s, 1);
    g.A = pc.Q; g.lda = s; g.sA = ss;
    g.B = Y2; g.ldb = s; g.sB = ss;
    g.C = w.A; g.ldc = s - k; g.sC = ss;
    hipError_t e = gemm_launch(g, PREC_F32, 1, 0, st);
    if (e) return e;
    GemmArgs u = gemm_base(s, s - k, k, 1);
    u.A = pc.Q; u.lda = s; u.sA = ss;
    u.B = w.A; u.ldb = s - k; u.sB = ss;
    u.C = Y2; u.ldc = s; u.sC = ss;
    u.Cin = Y2; u.ldcin = s; u.sCin = ss;
    u.alpha = -1.f; u.beta = 1.f;
    return gemm_launch(u, PREC_F32, 0, 0, st);
  };
  // the first basis: polar factors (conservative FP32 CANS) of Y1 and of Y2
  // with Y1's span projected out, into pc.Q.  A polar factor spans its
  // input's columns, and CANS converges from a badly conditioned input,
  // where CholeskyQR would not; what it leaves off orthonormal the
  // Newton-Schulz check below catches.
  auto basis = [&](const float* Y, int cols, float* dst) -> svdp_status {
    svdp_params q2 = dc_polar_params(p);
    q2.m = s;
    q2.n = cols;
    Ctx c2{h, &q2, carve_fwd(w.polar2, &q2, nullptr, false), st, 1, s, cols, Y, s, ss};
    svdp_status r2 = polar_core(c2);
    if (r2) return r2;
    HIPCHK(dc_copy_sel_launch(c2.w.X0, c2.w.X1, c2.w.where, cols, dst, s, s, cols, st), "dc basis");
    return SVDP_OK;
  };
  if ((r = basis(w.HQ, k, pc.Q))) return r;
  for (int pass = 0; pass < 2; ++pass) HIPCHK(project(w.HQ + k), "dc project 1");
  if ((r = basis(w.HQ + k, s - k, pc.Q + k))) return r;
  HIPCHK(range(pc.Q, w.Om), "dc range 2");
  // Newton-Schulz on the s x cols block at column c0: Z = Y (3 I - Y^T Y) / 2,
  // from Om to Q, back and to Q again; |G - I|_F^2 of the last G to dev
  auto newton_schulz = [&](int c0, int cols, double* dev) -> hipError_t {
    float* src = w.Om + c0;
    float* dst = pc.Q + c0;
    for (int it = 0; it < 3; ++it) {
      GemmArgs g = gemm_base(cols, cols, s, 1);  // G = Y^T Y
      g.A = src; g.lda = s; g.sA = ss;
      g.B = src; g.ldb = s; g.sB = ss;
      g.C = w.A; g.ldc = cols; g.sC = ss;
      g.sym = 1;
      hipError_t e = gemm_launch(g, PREC_F32, 1, 0, st);
      if (e) return e;
      if (it == 2 && (e = dc_dev_launch(w.A, cols, w.part, dev, st))) return e;
      GemmArgs u = gemm_base(s, cols, cols, 1);  // Z = 1.5 Y - 0.5 Y G
      u.A = src; u.lda = s; u.sA = ss;
      u.B = w.A; u.ldb = cols; u.sB = ss;
      u.C = dst; u.ldc = s; u.sC = ss;
      u.Cin = src; u.ldcin = s; u.sCin = ss;
      u.alpha = -0.5f; u.beta = 1.5f;
      if ((e = gemm_launch(u, PREC_F32, 0, 0, st))) return e;
      std::swap(src, dst);
    }
    return hipSuccess;
  };
  HIPCHK(newton_schulz(0, k, w.cpl + 2), "dc orth Q1");
  for (int pass = 0; pass < 2; ++pass) HIPCHK(project(w.Om + k), "dc project 2");
  HIPCHK(newton_schulz(k, s - k, w.cpl + 4), "dc orth Q2");
  // T = Q^T (M Q) and its coupling block
  GemmArgs g1 = gemm_base(s, s, s, 1);
  g1.A = pc.M; g1.lda = pc.ldm; g1.sA = ss;
  g1.B = pc.Q; g1.ldb = s; g1.sB = ss;
  g1.C = w.Om; g1.ldc = s; g1.sC = ss;
  HIPCHK(gemm_launch(g1, PREC_F32, 0, 0, st), "dc M Q");
  GemmArgs g2 = gemm_base(s, s, s, 1);
  g2.A = pc.Q; g2.lda = s; g2.sA = ss;
  g2.B = w.Om; g2.ldb = s; g2.sB = ss;
  g2.C = pc.T; g2.ldc = s; g2.sC = ss;
  HIPCHK(gemm_launch(g2, PREC_F32, 1, 0, st), "dc Q^T M Q");
  // symmetric in exact arithmetic: the pieces' own polar factors need it to be so
  HIPCHK(dc_sym_launch(pc.T, s, s, st), "dc sym");
  HIPCHK(dc_coupling_launch(pc.T, nullptr, nullptr, s, w.k, w.part, w.cpl, st), "dc coupling");
  double cpl[6];
  if ((r = read_doubles(h, st, w.cpl, 6, cpl))) return r;
  const double tol = 10.0 * p->tol;
  *ok = std::isfinite(cpl[0]) && std::isfinite(cpl[1]) && cpl[0] <= tol * tol * cpl[1] && cpl[2] <= 1e-6 &&
        cpl[4] <= 1e-6;
  pc.k = k;
  return SVDP_OK;
}

// One matrix by polar-based spectral divide and conquer.  The matrix is
// split once; a piece larger than kDcLeafMax is split again (to kDcDepth
// levels).  The pieces of at most kDcLeafMax, zero-padded to the largest of
// them, run through the Jacobi eigensolver as one batch; a larger piece (one
// that did not split, or at the depth limit) runs alone.  Each piece is
// solved shifted by its mean eigenvalue mu = trace / s, added back after:
// the eigenvectors do not change, and the solver's rounding and stop tests,
// which scale with the matrix's norm, then scale with the piece's spread
// rather than its offset from zero.  Then, from the deepest split up,
// V = Q diag(V1, V2).  Eigenvalues come out descending: a split puts the part
// above its sigma first.  A matrix whose first split fails runs the Jacobi
// eigensolver on H itself and gets fb_flag (FALLBACK_USED for svdp_eigh_dc;
// none inside the SVD, where that flag means a bound fallback).
svdp_status eigh_dc_one(svdp_handle* h, const svdp_params* p, const DcWs& w, const float* H, int64_t ldh,
                        float* lam, float* V, int64_t ldv, int* sweeps, int* flags, int b, hipStream_t st,
                        int fb_flag) {
  const int n = (int)p->n;
  const EighOpts eo = eigh_opts(p);
  std::vector<DcPiece> pcs;
  size_t used = 0;
  auto take = [&](size_t count) {
    float* r = w.pool + used;
    used += (count + 63) / 64 * 64;
    return r;
  };
  pcs.push_back({0, n, 0, 0, H, ldh, V, ldv, nullptr, nullptr, nullptr, false});
  std::vector<int> small, large;  // leaves: batched / alone
  svdp_status r;
  for (size_t i = 0; i < pcs.size(); ++i) {
    DcPiece pc = pcs[i];
    bool ok = false;
    if (i == 0 || (pc.s > kDcLeafMax && pc.depth < kDcDepth)) {
      const size_t mark = used, ss = (size_t)pc.s * pc.s;
      pc.Q = take(ss);
      pc.T = take(ss);
      pc.W = take(ss);
      if (used > w.pool_floats) return fail(SVDP_ERR_WORKSPACE, "divide and conquer pool overrun");
      if ((r = dc_split(h, p, w, pc, 0x5EED0000u ^ ((uint32_t)b << 8) ^ (uint32_t)i, st, &ok))) return r;
      if (!ok) used = mark;
    }
    if (ok) {
      pc.split = true;
      pcs[i] = pc;
      const int k = pc.k, s = pc.s;
      const int64_t d = (int64_t)k * s + k;
      pcs.push_back({pc.off, k, 0, pc.depth + 1, pc.T, s, pc.W, s, nullptr, nullptr, nullptr, false});
      pcs.push_back({pc.off + k, s - k, 0, pc.depth + 1, pc.T + d, s, pc.W + d, s, nullptr, nullptr, nullptr,
                     false});
    } else if (i == 0) {
      EighWs e = eigh_ws_carve(w.eigh, 1, n, p->max_sweeps);
      HIPCHK(eigh_run(e, H, ldh, (int64_t)n * n, 0, eo, lam, n, V, ldv, (int64_t)n * n, sweeps, flags, nullptr,
                      &h->aux, st), "dc eigh");
      if (fb_flag) HIPCHK(or_flags_launch(1, flags, fb_flag, nullptr, st), "dc fallback flag");
      return SVDP_OK;
    } else {
      (pc.s <= w.leaf_n ? small : large).push_back((int)i);
    }
  }
  const int nslots = (int)(small.size() + large.size());
  if (nslots > kDcLeaves) return fail(SVDP_ERR_WORKSPACE, "divide and conquer leaf overrun");
  HIPCHK(fill_i32(w.sw, 0, kDcLeaves, st), "dc sweeps");
  HIPCHK(fill_i32(w.fl, 0, kDcLeaves, st), "dc flags");
  if (!small.empty()) {
    int P = 1;
    for (int i : small) P = std::max(P, pcs[i].s);
    const int L = (int)small.size();
    if (L > w.leaf_count) return fail(SVDP_ERR_WORKSPACE, "divide and conquer leaf overrun");
    const int64_t PP = (int64_t)P * P;
    HIPCHK(fill_f32(w.Hl, 0.f, L * PP, st), "dc leaf zero");
    for (int l = 0; l < L; ++l) {
      const DcPiece& pc = pcs[small[l]];
      HIPCHK(dc_shift_launch(pc.M, pc.ldm, w.Hl + l * PP, P, pc.s, w.mu + l, st), "dc leaf shift");
    }
    EighWs e = eigh_ws_carve(w.eigh_leaf, L, P, p->max_sweeps);
    HIPCHK(eigh_run(e, w.Hl, P, PP, 0, eo, w.laml, P, w.Vl, P, PP, w.sw, w.fl, nullptr, &h->aux, st),
           "dc leaf eigh");
    for (int l = 0; l < L; ++l) {
      const DcPiece& pc = pcs[small[l]];
      HIPCHK(dc_leaf_launch(w.Vl + l * PP, w.laml + (int64_t)l * P, w.mu + l, P, pc.s, w.map, lam + pc.off, pc.V,
                            pc.ldv, w.fl + l, st), "dc leaf extract");
    }
  }
  for (size_t j = 0; j < large.size(); ++j) {
    const DcPiece& pc = pcs[large[j]];
    const int slot = (int)(small.size() + j);
    const int64_t ss = (int64_t)pc.s * pc.s;
    EighWs e = eigh_ws_carve(w.eigh, 1, pc.s, p->max_sweeps);
    HIPCHK(dc_shift_launch(pc.M, pc.ldm, w.A, pc.s, pc.s, w.mu + slot, st), "dc piece shift");
    HIPCHK(eigh_run(e, w.A, pc.s, ss, 0, eo, lam + pc.off, pc.s, pc.V, pc.ldv, ss, w.sw + slot, w.fl + slot,
                    nullptr, &h->aux, st), "dc piece eigh");
    HIPCHK(dc_add_launch(lam + pc.off, pc.s, w.mu + slot, st), "dc piece unshift");
  }
  HIPCHK(dc_info_launch(w.sw, w.fl, nslots, sweeps, flags, st), "dc info");
  // V = Q diag(V1, V2), children before their parent
  for (size_t i = pcs.size(); i-- > 0;) {
    const DcPiece& pc = pcs[i];
    if (!pc.split) continue;
    const int k = pc.k, s = pc.s;
    const int64_t ss = (int64_t)s * s, d = (int64_t)k * s + k;
    GemmArgs v1 = gemm_base(s, k, k, 1);
    v1.A = pc.Q; v1.lda = s; v1.sA = ss;
    v1.B = pc.W; v1.ldb = s; v1.sB = ss;
    v1.C = pc.V; v1.ldc = pc.ldv; v1.sC = ss;
    HIPCHK(gemm_launch(v1, PREC_F32, 0, 0, st), "dc V1");
    GemmArgs v2 = gemm_base(s, s - k, s - k, 1);
    v2.A = pc.Q + k; v2.lda = s; v2.sA = ss;
    v2.B = pc.W + d; v2.ldb = s; v2.sB = ss;
    v2.C = pc.V + k; v2.ldc = pc.ldv; v2.sC = ss;
    HIPCHK(gemm_launch(v2, PREC_F32, 0, 0, st), "dc V2");
  }
  return SVDP_OK;
}

svdp_status svd_eigh_dc(svdp_handle* h, const svdp_params* p, void* ws, const float* H, float* lam, float* V,
                        int64_t ldv, int* sweeps, int* flags, hipStream_t st) {
  const DcWs w = carve_dc(ws, p, nullptr);
  return eigh_dc_one(h, p, w, H, p->n, lam, V, ldv, sweeps, flags, 0, st, 0);
}

// QR preprocessing of tall matrices (the paper's rectangular experiments):
// Q, an orthonormal basis of A's columns (block Gram-Schmidt with CholeskyQR
// blocks, dependent columns dropped as zero columns), B = Q^T A (n x n, with
// A = Q B since Q Q^T A = A), the SVD B = U_B S V^T by svd_core on the square
// B, and U = Q U_B.  Zero columns of Q (a rank-deficient A) can leave
// columns of U off unit norm; Algorithm 1's column-norm test and QR step on
// U repair them.
svdp_status svd_tall_qr(Ctx& c, float* U, int64_t ldu, int64_t sU, float* S, int64_t sS, float* V, int64_t ldv,
                        int64_t sV) {
  FwdWs& w = c.w;
  const int B = c.batch, m = c.m, n = c.n;
  const int64_t mn = (int64_t)m * n, nn = (int64_t)n * n;
  {
    ProfScope phase(PROF_PHASE_QR, c.st);
    HIPCHK(copy_launch(c.A, c.lda, c.sA, nullptr, nullptr, w.Qt, n, mn, B, m, n, c.st, nullptr), "Q = A");
    HIPCHK(fill_i32(w.qmask, 1, B, c.st), "qr mask");
    svdp_status s = qr_blocks(c, w.Qt, n, mn, w.qmask, 1);
    if (s) return s;
    GemmArgs g = gemm_base(n, n, m, B);  // B = Q^T A
    g.A = w.Qt; g.lda = n; g.sA = mn;
    g.B = c.A; g.ldb = c.lda; g.sB = c.sA;
    g.C = w.Bq; g.ldc = n; g.sC = nn;
    HIPCHK(gemm_launch(g, PREC_F32, 1, 0, c.st), "Q^T A");
  }
  svdp_params p2 = *c.p;
  p2.m = n;
  Ctx c2 = c;
  c2.p = &p2;
  c2.m = n;
  c2.A = w.Bq;
  c2.lda = n;
  c2.sA = nn;
  c2.feat_m = m;
  svdp_status s = svd_core(c2, w.UBq, n, nn, S, sS, V, ldv, sV);
  if (s) return s;
  ProfScope phase(PROF_PHASE_QR, c.st);
  GemmArgs g = gemm_base(m, n, n, B);  // U = Q U_B
  g.A = w.Qt; g.lda = n; g.sA = mn;
  g.B = w.UBq; g.ldb = n; g.sB = nn;
  g.C = U; g.ldc = ldu; g.sC = sU;
  HIPCHK(gemm_launch(g, PREC_F32, 0, 0, c.st), "Q U_B");
  return u_qr_step(c, U, ldu, sU, S, sS, nullptr);
}

// Scratch of svd_polar_bwd_noalloc, for callers that cannot allocate: a
// file-scope device array, one copy per GPU, held until the process ends.
// In host code its name is only a stand-in: the device address of each GPU's
// copy comes from hipGetSymbolAddress with that GPU current, resolved once
// per device (at svdp_create, or at the entry point's first call on a
// device) and kept in g_scratch_addr.
constexpr size_t kScratchBytes = size_t(128) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

svdp_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(SVDP_ERR_INVALID_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SVDP_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return SVDP_OK;
}

}  // namespace

// =====================================================================
// C ABI
// =====================================================================

extern "C" {

void svdp_default_params(svdp_params* p, int64_t batch, int64_t m, int64_t n) {
  std::memset(p, 0, sizeof(*p));
  p->batch = batch; p->m = m; p->n = n;
  p->precision = SVDP_PREC_FP32;
  p->bound = SVDP_BOUND_CONSERVATIVE;
  p->max_iters = 50;
  p->pre_iters = 2;
  p->refine_steps = 2;
  p->max_sweeps = 16;
  p->inner_sweeps = 1;
  p->fp64_sweeps = 1;
  p->delta = 0.99;
  p->tol = 1e-5;
  p->eps_qr = 1e-5;
  p->bf16_handoff = 1e-2;
  p->refine_tol = 1e-2;
  p->jacobi_tol = 3e-3;
  p->jacobi_abs = 1e-9;
  p->bf16_from = 0.2;
  p->margin_max = 1.1;
  p->margin_min = 1.0;
  p->eigh_off_tol = 6e-6;
  p->eigh_restarts = 2;
  p->jacobi_fro_tol = 3e-4;
  p->poly = SVDP_POLY_CANS3;
  p->bf16_correct = 1;
  p->pe_lo = 1e-3;
  p->tall_qr = 1;
}

const char* svdp_status_string(int32_t s) {
  switch (s) {
    case SVDP_OK: return "ok";
    case SVDP_ERR_INVALID_ARG: return "invalid argument";
    case SVDP_ERR_SHAPE: return "bad shape";
    case SVDP_ERR_WORKSPACE: return "workspace too small";
    case SVDP_ERR_HIP: return "HIP error";
    case SVDP_ERR_NO_MODEL: return "no model loaded";
  }
  return "unknown status";
}

const char* svdp_last_error(void) { return g_last_error.c_str(); }

int64_t svdp_host_syncs(void) { return g_host_syncs.load(); }

svdp_status svdp_create(svdp_handle** out) {
  if (!out) return fail(SVDP_ERR_INVALID_ARG, "null handle pointer");
  svdp_handle* h = new svdp_handle();
  hipError_t e = hipMalloc((void**)&h->model, SVDP_MODEL_FLOATS * sizeof(float));
  if (e == hipSuccess) e = hipHostMalloc((void**)&h->host_word, 4096, hipHostMallocDefault);
  // parts of the batch the eigensolver runs on parallel streams (1 .. 4);
  // SVDP_EIGH_PARTS overrides the default of 2 (more parts measured no
  // faster: the sweeps are then throughput-bound)
  h->aux.parts = 2;
  if (const char* env = std::getenv("SVDP_EIGH_PARTS")) {
    const int v = std::atoi(env);
    if (v >= 1 && v <= kEighParts) h->aux.parts = v;
  }
  for (int i = 0; i < kEighParts - 1 && e == hipSuccess; ++i)
    e = hipStreamCreateWithFlags(&h->aux.st[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->aux.fork, hipEventDisableTiming);
  for (int i = 0; i < kEighParts && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&h->aux.skew[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->aux.join[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    (void)svdp_destroy(h);
    return hip_fail(e, "svdp_create");
  }
  // the allocation-free backward's scratch address on the current device
  void* scr = nullptr;
  svdp_status s = scratch_address(&scr);
  if (s) {
    (void)svdp_destroy(h);
    return s;
  }
  *out = h;
  return SVDP_OK;
}

svdp_status svdp_destroy(svdp_handle* h) {
  if (!h) return SVDP_OK;
  for (int i = 0; i < kEighParts - 1; ++i)
    if (h->aux.st[i]) (void)hipStreamSynchronize(h->aux.st[i]);
  for (int i = 0; i < kEighParts; ++i) {
    if (h->aux.skew[i]) (void)hipEventDestroy(h->aux.skew[i]);
    if (h->aux.join[i]) (void)hipEventDestroy(h->aux.join[i]);
  }
  if (h->aux.fork) (void)hipEventDestroy(h->aux.fork);
  for (int i = 0; i < kEighParts - 1; ++i)
    if (h->aux.st[i]) (void)hipStreamDestroy(h->aux.st[i]);
  if (h->model) (void)hipFree(h->model);
  if (h->host_word) (void)hipHostFree(h->host_word);
  delete h;
  return SVDP_OK;
}

svdp_status svdp_set_model(svdp_handle* h, const float* host_model) {
  if (!h || !host_model) return fail(SVDP_ERR_INVALID_ARG, "null handle or model");
  HIPCHK(hipMemcpy(h->model, host_model, SVDP_MODEL_FLOATS * sizeof(float), hipMemcpyHostToDevice), "set_model");
  h->has_model = true;
  return SVDP_OK;
}

static size_t bwd_bytes(const svdp_params* p, int polar) {
  Carver c(nullptr);
  const size_t b = p->batch, m = p->m, n = p->n;
  c.take<float>(b * n * n);  // X1 (Ahat / V^T dH V)
  c.take<float>(b * n * n);  // X2 (P / (MV)^T dW V)
  c.take<float>(b * n * n);  // Y
  c.take<float>(b * n * n);  // T1
  c.take<float>(b * m * n);  // Z
  c.take<float>(b * n);      // D
  if (polar) {
    c.take<float>(b * m * n);  // MV
    c.take<float>(b * m * n);  // dW V
    c.take<float>(b * n);      // S (own eigh)
    c.take<float>(b * n * n);  // V (own eigh)
    c.take<int>(b);            // sweeps
    c.take<int>(b);            // flags
    c.take_bytes(eigh_ws_bytes(b, n, p->max_sweeps));
  }
  return c.off;
}

svdp_status svdp_workspace_size(const svdp_params* p, int32_t op, size_t* bytes) {
  if (!bytes) return fail(SVDP_ERR_INVALID_ARG, "null bytes");
  svdp_status s = check_common(p);
  if (s) return s;
  size_t total = 0;
  switch (op) {
    case SVDP_OP_SVD_FWD: carve_fwd(nullptr, p, &total); break;
    case SVDP_OP_POLAR_FWD:
    case SVDP_OP_FEATURES: carve_fwd(nullptr, p, &total, false); break;
    case SVDP_OP_SVD_BWD: total = bwd_bytes(p, 0); break;
    case SVDP_OP_EIGH_BWD: {
      Carver c(nullptr);
      c.take<float>((size_t)p->batch * p->n * p->n * 3);
      total = c.off;
      break;
    }
    case SVDP_OP_POLAR_BWD: total = bwd_bytes(p, 1); break;
    case SVDP_OP_EIGH_DC: carve_dc(nullptr, p, &total); break;
    case SVDP_OP_EIGH: {
      Carver c(nullptr);
      c.take<int>(p->batch);
      c.take<int>(p->batch);
      c.take_bytes(eigh_ws_bytes(p->batch, p->n, p->max_sweeps));
      total = c.off;
      break;
    }
    default: return fail(SVDP_ERR_INVALID_ARG, "unknown op");
  }
  *bytes = total;
  return SVDP_OK;
}

#define REQ(ptr) \
  if (!(ptr)) return fail(SVDP_ERR_INVALID_ARG, "null pointer argument: " #ptr)
#define LDCHK(ld, cols, stride, rows) \
  if (bad_ld(ld, cols, stride, rows)) return fail(SVDP_ERR_INVALID_ARG, "leading dimension or stride too small: " #ld)

svdp_status svd_polar_fwd(svdp_handle* h, const svdp_params* p, const float* A, int64_t lda, int64_t sA,
                          float* U, int64_t ldu, int64_t sU, float* S, int64_t sS, float* V, int64_t ldv,
                          int64_t sV, svdp_info* info, void* ws, size_t ws_bytes, void* stream) {
  REQ(h);
  svdp_status s = check_common(p);
  if (s) return s;
  if ((s = check_model(h, p))) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(A); REQ(U); REQ(S); REQ(V);
  LDCHK(lda, p->n, p->batch > 1 ? sA : 0, p->m);
  LDCHK(ldu, p->n, p->batch > 1 ? sU : 0, p->m);
  LDCHK(ldv, p->n, p->batch > 1 ? sV : 0, p->n);
  if (p->batch > 1 && sS < p->n) return fail(SVDP_ERR_INVALID_ARG, "sS < n");
  size_t need = 0;
  carve_fwd(nullptr, p, &need);
  if (!ws || ws_bytes < need) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  Ctx c{h, p, carve_fwd(ws, p, nullptr), (hipStream_t)stream, (int)p->batch, (int)p->m, (int)p->n, A, lda, sA};
  if (use_tall_qr(p)) {
    if ((s = svd_tall_qr(c, U, ldu, sU, S, sS, V, ldv, sV))) return s;
  } else if ((s = svd_core(c, U, ldu, sU, S, sS, V, ldv, sV))) {
    return s;
  }
  if (info) HIPCHK(info_pack_launch(c.batch, c.w.iters, c.w.sweeps, c.w.flags, c.w.resid, info, nullptr, c.st), "info");
  return SVDP_OK;
}

svdp_status polar_fwd(svdp_handle* h, const svdp_params* p, const float* A, int64_t lda, int64_t sA, float* W,
                      int64_t ldw, int64_t sW, float* H, int64_t ldh, int64_t sH, float* S_cache, int64_t sS,
                      float* V_cache, int64_t ldv, int64_t sV, svdp_info* info, void* ws, size_t ws_bytes,
                      void* stream) {
  REQ(h);
  svdp_status s = check_common(p);
  if (s) return s;
  if ((s = check_model(h, p))) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(A); REQ(W); REQ(H);
  if ((S_cache == nullptr) != (V_cache == nullptr))
    return fail(SVDP_ERR_INVALID_ARG, "S_cache and V_cache must both be given or both null");
  LDCHK(lda, p->n, p->batch > 1 ? sA : 0, p->m);
  LDCHK(ldw, p->n, p->batch > 1 ? sW : 0, p->m);
  LDCHK(ldh, p->n, p->batch > 1 ? sH : 0, p->n);
  if (V_cache) LDCHK(ldv, p->n, p->batch > 1 ? sV : 0, p->n);
  size_t need = 0;
  carve_fwd(nullptr, p, &need, false);
  if (!ws || ws_bytes < need) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  Ctx c{h, p, carve_fwd(ws, p, nullptr, false), (hipStream_t)stream, (int)p->batch, (int)p->m, (int)p->n, A, lda,
        sA};
  const int B = c.batch, m = c.m, n = c.n;
  if ((s = polar_core(c))) return s;
  // the BF16 correction (bf16_correct) of W, H and the eigenpairs, when the
  // eigenpairs are requested: W is then written by the first pass, and only
  // the fallback reruns copy their iterate at the end
  const bool correct = V_cache && p->bf16_correct && p->precision == SVDP_PREC_BF16 &&
                       p->bound != SVDP_BOUND_CONSERVATIVE;
  auto tail = [&](const int* mask) -> svdp_status {
    svdp_status s2 = form_h(c, mask);
    if (s2) return s2;
    if (V_cache) {
      EighWs e = eigh_ws_carve(c.w.eigh, B, n, p->max_sweeps);
      HIPCHK(eigh_run(e, c.w.G, n, (int64_t)n * n, 0, eigh_opts(p), S_cache, sS, V_cache, ldv, sV, c.w.sweeps,
                      c.w.flags, mask, &h->aux, c.st), "eigh");
      if (correct && !mask) {
        // as in svd_tail, with signed eigenvalues: Mu in Hw, V Mu in V2,
        // V <- 2 V - V Mu, S corrected; then W <- W (V Mu) V^T (the new V)
        // and G = W^T A for H = sym(G)
        const int64_t n2 = (int64_t)n * n, np2 = (int64_t)e.np * e.np;
        HIPCHK(polar_fix_launch(e.Vw, e.np, np2, e.perm, S_cache, sS, e.sgn, 1, B, n, e.Hw, e.V2, c.w.y0,
                                c.w.colsum, nullptr, c.st), "polar fix");
        GemmArgs vu = gemm_base(n, n, n, B);  // V Mu
        vu.A = V_cache; vu.lda = ldv; vu.sA = sV;
        vu.B = e.Hw; vu.ldb = n; vu.sB = n2;
        vu.C = e.V2; vu.ldc = n; vu.sC = n2;
        HIPCHK(gemm_launch(vu, PREC_F32, 0, 0, c.st), "V Mu");
        HIPCHK(vcorr_launch(V_cache, ldv, sV, e.V2, B, n, c.st), "V");
        HIPCHK(sigma_store_launch(c.w.colsum, n, S_cache, sS, B, nullptr, c.st), "eigenvalues");
        GemmArgs r = gemm_base(n, n, n, B);  // R = (V Mu) V^T
        r.A = e.V2; r.lda = n; r.sA = n2;
        r.B = V_cache; r.ldb = ldv; r.sB = sV;
        r.C = e.Hw; r.ldc = n; r.sC = n2;
        HIPCHK(gemm_launch(r, PREC_F32, 0, 1, c.st), "R");
        GemmArgs wc = gemm_base(m, n, n, B);  // W out = W R
        wc.A = c.w.X0; wc.A_alt = c.w.X1; wc.a_sel = c.w.where; wc.lda = n; wc.sA = (int64_t)m * n;
        wc.B = e.Hw; wc.ldb = n; wc.sB = n2;
        wc.C = W; wc.ldc = ldw; wc.sC = sW;
        HIPCHK(gemm_launch(wc, PREC_F32, 0, 0, c.st), "W R");
        GemmArgs g = gemm_base(n, n, m, B);  // G = W^T A
        g.A = W; g.lda = ldw; g.sA = sW;
        g.B = c.A; g.ldb = c.lda; g.sB = c.sA;
        g.C = c.w.G; g.ldc = n; g.sC = n2;
        HIPCHK(gemm_launch(g, PREC_F32, 1, 0, c.st), "W^T A");
      }
    }
    return SVDP_OK;
  };
  if ((s = tail(nullptr))) return s;
  if (p->bound != SVDP_BOUND_CONSERVATIVE) {
    int cnt = 0;
    if ((s = fallback_mask(c, &cnt))) return s;
    if (cnt > 0) {
      const int* mk = c.w.mask;
      if ((s = conservative_fp32(c, mk))) return s;
      if ((s = final_residual(c, mk))) return s;
      if ((s = tail(mk))) return s;
      HIPCHK(or_flags_launch(B, c.w.flags, SVDP_FLAG_FALLBACK_USED, mk, c.st), "flags");
    }
  }
  HIPCHK(symmetrize_launch(c.w.G, B, n, H, ldh, sH, c.st), "H out");
  HIPCHK(copy_launch(c.w.X0, n, (int64_t)m * n, c.w.where, c.w.X1, W, ldw, sW, B, m, n, c.st,
                     correct ? c.w.mask : nullptr), "W out");
  if (info) HIPCHK(info_pack_launch(B, c.w.iters, c.w.sweeps, c.w.flags, c.w.resid, info, nullptr, c.st), "info");
  return SVDP_OK;
}

svdp_status svdp_eigh_bwd(svdp_handle* h, const svdp_params* p, const float* lam, int64_t slam, const float* V,
                          int64_t ldv, int64_t sV, const float* dlam, int64_t sdlam, const float* dV, int64_t lddv,
                          int64_t sdV, float* dH, int64_t lddh, int64_t sdH, void* ws, size_t ws_bytes, void* stream) {
  REQ(h);
  svdp_params q = *p;
  q.m = q.n;
  svdp_status s = check_common(&q);
  if (s) return s;
  if (q.batch == 0) return SVDP_OK;
  REQ(lam); REQ(V); REQ(dH);
  const int B = (int)q.batch, n = (int)q.n;
  LDCHK(ldv, n, B > 1 ? sV : 0, n);
  LDCHK(lddh, n, B > 1 ? sdH : 0, n);
  if (dV) LDCHK(lddv, n, B > 1 ? sdV : 0, n);
  size_t need = 0;
  svdp_workspace_size(&q, SVDP_OP_EIGH_BWD, &need);
  if (!ws || ws_bytes < need) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  Carver c(ws);
  float* P = c.take<float>((size_t)B * n * n);
  float* C = c.take<float>((size_t)B * n * n);
  float* T = c.take<float>((size_t)B * n * n);
  if (dV) {  // P = V^T dV
    GemmArgs g = gemm_base(n, n, n, B);
    g.A = V; g.lda = ldv; g.sA = sV;
    g.B = dV; g.ldb = lddv; g.sB = sdV;
    g.C = P; g.ldc = n; g.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(g, PREC_F32, 1, 0, st), "V^T dV");
  }
  HIPCHK(sylvester_launch(2, nullptr, dV ? P : nullptr, lam, slam, dlam, sdlam, nullptr, B, n, q.eps_K, 0.0, C, st),
         "eigh bwd scaling");
  {  // T = V C
    GemmArgs g = gemm_base(n, n, n, B);
    g.A = V; g.lda = ldv; g.sA = sV;
    g.B = C; g.ldb = n; g.sB = (int64_t)n * n;
    g.C = T; g.ldc = n; g.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 0, st), "V C");
  }
  {  // dH = T V^T
    GemmArgs g = gemm_base(n, n, n, B);
    g.A = T; g.lda = n; g.sA = (int64_t)n * n;
    g.B = V; g.ldb = ldv; g.sB = sV;
    g.C = dH; g.ldc = lddh; g.sC = sdH;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 1, st), "T V^T");
  }
  return SVDP_OK;
}

}  // extern "C"

namespace {
// Algorithm 4 backward in the eigenbasis on a workspace (checked by the
// caller to hold bwd_bytes(p, 0)).
svdp_status svd_bwd_impl(const svdp_params* p, const float* U, int64_t ldu, int64_t sU, const float* S, int64_t sS,
                         const float* V, int64_t ldv, int64_t sV, const float* dU, int64_t lddu, int64_t sdU,
                         const float* dS, int64_t sdS, const float* dV, int64_t lddv, int64_t sdV, float* dA,
                         int64_t ldda, int64_t sdA, void* ws, hipStream_t st) {
  const int B = (int)p->batch, m = (int)p->m, n = (int)p->n;
  ProfScope phase(PROF_PHASE_BWD, st);
  Carver c(ws);
  float* X1 = c.take<float>((size_t)B * n * n);
  float* X2 = c.take<float>((size_t)B * n * n);
  float* Y = c.take<float>((size_t)B * n * n);
  c.take<float>((size_t)B * n * n);
  float* Z = c.take<float>((size_t)B * m * n);
  float* D = c.take<float>((size_t)B * n);
  if (dU) {  // Ahat = U^T dU
    GemmArgs g = gemm_base(n, n, m, B);
    g.A = U; g.lda = ldu; g.sA = sU;
    g.B = dU; g.ldb = lddu; g.sB = sdU;
    g.C = X1; g.ldc = n; g.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(g, PREC_F32, 1, 0, st), "U^T dU");
  }
  if (dV) {  // P = V^T dV
    GemmArgs g = gemm_base(n, n, n, B);
    g.A = V; g.lda = ldv; g.sA = sV;
    g.B = dV; g.ldb = lddv; g.sB = sdV;
    g.C = X2; g.ldc = n; g.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(g, PREC_F32, 1, 0, st), "V^T dV");
  }
  HIPCHK(dvec_launch(S, sS, B, n, p->eps_R, D, st), "D");
  HIPCHK(sylvester_launch(0, dU ? X1 : nullptr, dV ? X2 : nullptr, S, sS, dS, sdS, D, B, n, p->eps_K, p->eps_T, Y,
                          st), "sylvester");
  {  // Z = 2 U (S Y) + dU diag(D)
    GemmArgs g = gemm_base(m, n, n, B);
    g.A = U; g.lda = ldu; g.sA = sU;
    g.B = Y; g.ldb = n; g.sB = (int64_t)n * n;
    g.C = Z; g.ldc = n; g.sC = (int64_t)m * n;
    g.alpha = 2.f;
    if (dU) {
      g.Cin = dU; g.ldcin = lddu; g.sCin = sdU; g.beta = 1.f;
      g.colscale_in = D; g.csin_stride = n;
    }
    HIPCHK(gemm_launch(g, PREC_F32, 0, 0, st), "Z");
  }
  {  // dA = Z V^T
    GemmArgs g = gemm_base(m, n, n, B);
    g.A = Z; g.lda = n; g.sA = (int64_t)m * n;
    g.B = V; g.ldb = ldv; g.sB = sV;
    g.C = dA; g.ldc = ldda; g.sC = sdA;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 1, st), "Z V^T");
  }
  return SVDP_OK;
}

// Argument checks shared by svd_polar_bwd and svd_polar_bwd_noalloc.
svdp_status svd_bwd_check(const svdp_params* p, const float* U, int64_t ldu, int64_t sU, const float* S,
                          const float* V, int64_t ldv, int64_t sV, const float* dU, int64_t lddu, int64_t sdU,
                          const float* dV, int64_t lddv, int64_t sdV, float* dA, int64_t ldda, int64_t sdA) {
  svdp_status s = check_common(p);
  if (s) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(U); REQ(S); REQ(V); REQ(dA);
  const int B = (int)p->batch, m = (int)p->m, n = (int)p->n;
  LDCHK(ldu, n, B > 1 ? sU : 0, m);
  LDCHK(ldv, n, B > 1 ? sV : 0, n);
  LDCHK(ldda, n, B > 1 ? sdA : 0, m);
  if (dU) LDCHK(lddu, n, B > 1 ? sdU : 0, m);
  if (dV) LDCHK(lddv, n, B > 1 ? sdV : 0, n);
  return SVDP_OK;
}
}  // namespace

extern "C" {

svdp_status svd_polar_bwd(svdp_handle* h, const svdp_params* p, const float* U, int64_t ldu, int64_t sU,
                          const float* S, int64_t sS, const float* V, int64_t ldv, int64_t sV, const float* dU,
                          int64_t lddu, int64_t sdU, const float* dS, int64_t sdS, const float* dV,
                          int64_t lddv, int64_t sdV, float* dA, int64_t ldda, int64_t sdA, void* ws,
                          size_t ws_bytes, void* stream) {
  REQ(h);
  svdp_status s = svd_bwd_check(p, U, ldu, sU, S, V, ldv, sV, dU, lddu, sdU, dV, lddv, sdV, dA, ldda, sdA);
  if (s || p->batch == 0) return s;
  if (!ws || ws_bytes < bwd_bytes(p, 0)) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  return svd_bwd_impl(p, U, ldu, sU, S, sS, V, ldv, sV, dU, lddu, sdU, dS, sdS, dV, lddv, sdV, dA, ldda, sdA, ws,
                      (hipStream_t)stream);
}

svdp_status svd_polar_bwd_noalloc(svdp_handle* h, const svdp_params* p, const float* U, int64_t ldu, int64_t sU,
                                  const float* S, int64_t sS, const float* V, int64_t ldv, int64_t sV,
                                  const float* dU, int64_t lddu, int64_t sdU, const float* dS, int64_t sdS,
                                  const float* dV, int64_t lddv, int64_t sdV, float* dA, int64_t ldda, int64_t sdA,
                                  void* stream) {
  REQ(h);
  svdp_status s = svd_bwd_check(p, U, ldu, sU, S, V, ldv, sV, dU, lddu, sdU, dV, lddv, sdV, dA, ldda, sdA);
  if (s || p->batch == 0) return s;
  const size_t need = bwd_bytes(p, 0);
  if (need > kScratchBytes) {
    char msg[160];
    std::snprintf(msg, sizeof(msg),
                  "svd_polar_bwd_noalloc: this batch needs %zu bytes of scratch, the static scratch holds %zu",
                  need, kScratchBytes);
    return fail(SVDP_ERR_WORKSPACE, msg);
  }
  void* ws = nullptr;
  if ((s = scratch_address(&ws))) return s;
  return svd_bwd_impl(p, U, ldu, sU, S, sS, V, ldv, sV, dU, lddu, sdU, dS, sdS, dV, lddv, sdV, dA, ldda, sdA, ws,
                      (hipStream_t)stream);
}

svdp_status polar_bwd(svdp_handle* h, const svdp_params* p, const float* A, int64_t lda, int64_t sA,
                      const float* H, int64_t ldh, int64_t sH, const float* S_cache, int64_t sS,
                      const float* V_cache, int64_t ldv, int64_t sV, const float* dW, int64_t lddw,
                      int64_t sdW, const float* dH, int64_t lddh, int64_t sdH, float* dA, int64_t ldda,
                      int64_t sdA, void* ws, size_t ws_bytes, void* stream) {
  REQ(h);
  svdp_status s = check_common(p);
  if (s) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(A); REQ(dA);
  if ((S_cache == nullptr) != (V_cache == nullptr))
    return fail(SVDP_ERR_INVALID_ARG, "S_cache and V_cache must both be given or both null");
  if (!V_cache) REQ(H);
  const int B = (int)p->batch, m = (int)p->m, n = (int)p->n;
  LDCHK(lda, n, B > 1 ? sA : 0, m);
  LDCHK(ldda, n, B > 1 ? sdA : 0, m);
  if (H) LDCHK(ldh, n, B > 1 ? sH : 0, n);
  if (V_cache) LDCHK(ldv, n, B > 1 ? sV : 0, n);
  if (dW) LDCHK(lddw, n, B > 1 ? sdW : 0, m);
  if (dH) LDCHK(lddh, n, B > 1 ? sdH : 0, n);
  if (!ws || ws_bytes < bwd_bytes(p, 1)) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  ProfScope phase(PROF_PHASE_BWD, st);
  Carver c(ws);
  float* X1 = c.take<float>((size_t)B * n * n);
  float* X2 = c.take<float>((size_t)B * n * n);
  float* Y = c.take<float>((size_t)B * n * n);
  float* T1 = c.take<float>((size_t)B * n * n);
  float* Z = c.take<float>((size_t)B * m * n);
  float* D = c.take<float>((size_t)B * n);
  float* MV = c.take<float>((size_t)B * m * n);
  float* WV = c.take<float>((size_t)B * m * n);
  float* Sown = c.take<float>((size_t)B * n);
  float* Vown = c.take<float>((size_t)B * n * n);
  int* sweeps = c.take<int>(B);
  int* flags = c.take<int>(B);
  void* ews = c.take_bytes(eigh_ws_bytes(B, n, p->max_sweeps));
  const float* Sx = S_cache;
  const float* Vx = V_cache;
  int64_t sSx = sS, ldvx = ldv, sVx = sV;
  if (!V_cache) {  // Algorithm 2, step 1: EVD of H
    EighWs e = eigh_ws_carve(ews, B, n, p->max_sweeps);
    HIPCHK(fill_i32(flags, 0, B, st), "flags");
    HIPCHK(eigh_run(e, H, ldh, sH, 0, eigh_opts(p), Sown, n, Vown, n, (int64_t)n * n, sweeps, flags,
                    nullptr, &h->aux, st), "eigh");
    Sx = Sown; Vx = Vown; sSx = n; ldvx = n; sVx = (int64_t)n * n;
  }
  {  // MV = A V
    GemmArgs g = gemm_base(m, n, n, B);
    g.A = A; g.lda = lda; g.sA = sA;
    g.B = Vx; g.ldb = ldvx; g.sB = sVx;
    g.C = MV; g.ldc = n; g.sC = (int64_t)m * n;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 0, st), "A V");
  }
  if (dW) {
    GemmArgs g = gemm_base(m, n, n, B);  // dW V
    g.A = dW; g.lda = lddw; g.sA = sdW;
    g.B = Vx; g.ldb = ldvx; g.sB = sVx;
    g.C = WV; g.ldc = n; g.sC = (int64_t)m * n;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 0, st), "dW V");
    GemmArgs q = gemm_base(n, n, m, B);  // (A V)^T (dW V)
    q.A = MV; q.lda = n; q.sA = (int64_t)m * n;
    q.B = WV; q.ldb = n; q.sB = (int64_t)m * n;
    q.C = X2; q.ldc = n; q.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(q, PREC_F32, 1, 0, st), "(AV)^T dW V");
  }
  if (dH) {
    GemmArgs g = gemm_base(n, n, n, B);  // V^T dH
    g.A = Vx; g.lda = ldvx; g.sA = sVx;
    g.B = dH; g.ldb = lddh; g.sB = sdH;
    g.C = T1; g.ldc = n; g.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(g, PREC_F32, 1, 0, st), "V^T dH");
    GemmArgs q = gemm_base(n, n, n, B);  // (V^T dH) V
    q.A = T1; q.lda = n; q.sA = (int64_t)n * n;
    q.B = Vx; q.ldb = ldvx; q.sB = sVx;
    q.C = X1; q.ldc = n; q.sC = (int64_t)n * n;
    HIPCHK(gemm_launch(q, PREC_F32, 0, 0, st), "V^T dH V");
  }
  HIPCHK(dvec_launch(Sx, sSx, B, n, p->eps_R, D, st), "D");
  HIPCHK(sylvester_launch(1, dH ? X1 : nullptr, dW ? X2 : nullptr, Sx, sSx, nullptr, 0, D, B, n, p->eps_K,
                          p->eps_T, Y, st), "sylvester");
  {  // Z = 2 (A V) Xt + (dW V) diag(D)
    GemmArgs g = gemm_base(m, n, n, B);
    g.A = MV; g.lda = n; g.sA = (int64_t)m * n;
    g.B = Y; g.ldb = n; g.sB = (int64_t)n * n;
    g.C = Z; g.ldc = n; g.sC = (int64_t)m * n;
    g.alpha = 2.f;
    if (dW) {
      g.Cin = WV; g.ldcin = n; g.sCin = (int64_t)m * n; g.beta = 1.f;
      g.colscale_in = D; g.csin_stride = n;
    }
    HIPCHK(gemm_launch(g, PREC_F32, 0, 0, st), "Z");
  }
  {  // dA = Z V^T
    GemmArgs g = gemm_base(m, n, n, B);
    g.A = Z; g.lda = n; g.sA = (int64_t)m * n;
    g.B = Vx; g.ldb = ldvx; g.sB = sVx;
    g.C = dA; g.ldc = ldda; g.sC = sdA;
    HIPCHK(gemm_launch(g, PREC_F32, 0, 1, st), "Z V^T");
  }
  return SVDP_OK;
}

svdp_status svdp_eigh(svdp_handle* h, const svdp_params* p, const float* H, int64_t ldh, int64_t sH, float* lam,
                      int64_t slam, float* V, int64_t ldv, int64_t sV, svdp_info* info, void* ws, size_t ws_bytes,
                      void* stream) {
  REQ(h);
  svdp_status s = check_common(p);
  if (s) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(H); REQ(lam); REQ(V);
  const int B = (int)p->batch, n = (int)p->n;
  LDCHK(ldh, n, B > 1 ? sH : 0, n);
  LDCHK(ldv, n, B > 1 ? sV : 0, n);
  if (B > 1 && slam < n) return fail(SVDP_ERR_INVALID_ARG, "slam < n");
  size_t need = 0;
  svdp_workspace_size(p, SVDP_OP_EIGH, &need);
  if (!ws || ws_bytes < need) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  Carver c(ws);
  int* sweeps = c.take<int>(B);
  int* flags = c.take<int>(B);
  void* ews = c.take_bytes(eigh_ws_bytes(B, n, p->max_sweeps));
  EighWs e = eigh_ws_carve(ews, B, n, p->max_sweeps);
  HIPCHK(fill_i32(flags, 0, B, st), "flags");
  HIPCHK(fill_i32(sweeps, 0, B, st), "sweeps");
  HIPCHK(eigh_run(e, H, ldh, sH, 0, eigh_opts(p), lam, slam, V, ldv, sV, sweeps, flags, nullptr,
                  &h->aux, st), "eigh");
  if (info) HIPCHK(info_pack_launch(B, nullptr, sweeps, flags, nullptr, info, nullptr, st), "info");
  return SVDP_OK;
}

svdp_status svdp_eigh_dc(svdp_handle* h, const svdp_params* p, const float* H, int64_t ldh, int64_t sH, float* lam,
                         int64_t slam, float* V, int64_t ldv, int64_t sV, svdp_info* info, void* ws,
                         size_t ws_bytes, void* stream) {
  REQ(h);
  svdp_status s = check_common(p);
  if (s) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(H); REQ(lam); REQ(V);
  const int B = (int)p->batch, n = (int)p->n;
  LDCHK(ldh, n, B > 1 ? sH : 0, n);
  LDCHK(ldv, n, B > 1 ? sV : 0, n);
  if (B > 1 && slam < n) return fail(SVDP_ERR_INVALID_ARG, "slam < n");
  size_t need = 0;
  svdp_workspace_size(p, SVDP_OP_EIGH_DC, &need);
  if (!ws || ws_bytes < need) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  const DcWs w = carve_dc(ws, p, nullptr);
  HIPCHK(fill_i32(w.flags, 0, B, st), "flags");
  HIPCHK(fill_i32(w.sweeps, 0, B, st), "sweeps");
  for (int b = 0; b < B; ++b) {
    if ((s = eigh_dc_one(h, p, w, H + b * sH, ldh, lam + b * slam, V + b * sV, ldv, w.sweeps + b, w.flags + b,
                         b, st, SVDP_FLAG_FALLBACK_USED)))
      return s;
    HIPCHK(dc_neg_launch(lam + b * slam, n, eigh_opts(p).neg_tol, w.flags + b, st), "dc negative eigenvalue");
  }
  if (info) HIPCHK(info_pack_launch(B, nullptr, w.sweeps, w.flags, nullptr, info, nullptr, st), "info");
  return SVDP_OK;
}

svdp_status svdp_bound_features(svdp_handle* h, const svdp_params* p, const float* A, int64_t lda, int64_t sA,
                                const float* probe, float* F, float* aux, void* ws, size_t ws_bytes,
                                void* stream) {
  REQ(h);
  svdp_status s = check_common(p);
  if (s) return s;
  if (p->batch == 0) return SVDP_OK;
  REQ(A); REQ(probe); REQ(F); REQ(aux);
  LDCHK(lda, p->n, p->batch > 1 ? sA : 0, p->m);
  size_t need = 0;
  carve_fwd(nullptr, p, &need, false);
  if (!ws || ws_bytes < need) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  FwdWs w = carve_fwd(ws, p, nullptr, false);
  hipStream_t st = (hipStream_t)stream;
  const int B = (int)p->batch, m = (int)p->m, n = (int)p->n;
  HIPCHK(fill_i32(w.flags, 0, B, st), "flags");
  HIPCHK(norms_launch(A, lda, sA, B, m, n, w.colsum, w.rowmax, w.fro2, w.fpart, w.flags, nullptr, st), "norms");
  HIPCHK(vnorm_launch(probe, n, B, n, w.nrm, 0, st), "probe norm");
  const float* x = probe;
  int64_t sx = n;
  for (int k = 1; k <= 7; ++k) {
    float* y = (k & 1) ? w.y0 : w.y1;
    int trans = (k & 1) ? 0 : 1;
    HIPCHK(matvec_launch(A, lda, sA, B, m, n, x, sx, y, m, trans, w.fro2, st), "matvec");
    HIPCHK(vnorm_launch(y, m, B, trans ? n : m, w.nrm, k, st), "vnorm");
    x = y;
    sx = m;
  }
  HIPCHK(features_launch(w.fro2, w.nrm, B, m, n, F, aux, st), "features");
  return SVDP_OK;
}

svdp_status svdp_spectral_features(const float* sv, const float* z, int64_t rows, int64_t n,
                                   const float* m_over_n, float* F, float* aux, void* stream) {
  if (rows == 0) return SVDP_OK;
  REQ(sv); REQ(z); REQ(m_over_n); REQ(F); REQ(aux);
  if (rows < 0 || n < 1 || rows > (1 << 26)) return fail(SVDP_ERR_SHAPE, "bad rows / n");
  HIPCHK(spectral_features_launch(sv, z, (int)rows, (int)n, m_over_n, F, aux, (hipStream_t)stream), "features");
  return SVDP_OK;
}

svdp_status svdp_training_targets(const float* sv, const float* aux, int64_t rows, int64_t n, float* T,
                                  void* stream) {
  if (rows == 0) return SVDP_OK;
  REQ(sv); REQ(aux); REQ(T);
  if (rows < 0 || n < 1 || rows > (1 << 26)) return fail(SVDP_ERR_SHAPE, "bad rows / n");
  HIPCHK(training_targets_launch(sv, aux, (int)rows, (int)n, T, (hipStream_t)stream), "training targets");
  return SVDP_OK;
}

svdp_status svdp_feature_stats(const float* F, int64_t rows, float* mu, float* sd, void* stream) {
  REQ(F); REQ(mu); REQ(sd);
  if (rows < 1 || rows > (1 << 26)) return fail(SVDP_ERR_SHAPE, "need 1 <= rows <= 2^26");
  HIPCHK(feature_stats_launch(F, (int)rows, mu, sd, (hipStream_t)stream), "feature stats");
  return SVDP_OK;
}

svdp_status svdp_mlp_fwd(const float* params, const float* mu, const float* sd, const float* X, int64_t rows,
                         float* out, float* act, void* stream) {
  if (rows == 0) return SVDP_OK;
  REQ(params); REQ(X); REQ(out);
  if ((mu == nullptr) != (sd == nullptr)) return fail(SVDP_ERR_INVALID_ARG, "mu and sd go together");
  if (rows < 0 || rows > (1 << 26)) return fail(SVDP_ERR_SHAPE, "bad rows");
  HIPCHK(mlp_fwd_launch(params, mu, sd, X, (int)rows, out, act, (hipStream_t)stream), "mlp fwd");
  return SVDP_OK;
}

size_t svdp_mlp_bwd_ws_bytes(int64_t rows) {
  return rows <= 0 ? 256 : mlp_bwd_partial_floats((int)rows) * sizeof(float);
}

svdp_status svdp_mlp_bwd(const float* params, const float* mu, const float* sd, const float* X, const float* act,
                         const float* dout, int64_t rows, float* dparams, void* ws, size_t ws_bytes, void* stream) {
  REQ(params); REQ(dparams);
  if ((mu == nullptr) != (sd == nullptr)) return fail(SVDP_ERR_INVALID_ARG, "mu and sd go together");
  if (rows < 0 || rows > (1 << 26)) return fail(SVDP_ERR_SHAPE, "bad rows");
  hipStream_t st = (hipStream_t)stream;
  if (rows == 0) {
    HIPCHK(fill_f32(dparams, 0.f, SVDP_MLP_PARAMS, st), "zero grad");
    return SVDP_OK;
  }
  REQ(X); REQ(act); REQ(dout);
  if (!ws || ws_bytes < svdp_mlp_bwd_ws_bytes(rows)) return fail(SVDP_ERR_WORKSPACE, "workspace too small");
  HIPCHK(mlp_bwd_launch(params, mu, sd, X, act, dout, (int)rows, (float*)ws, dparams, st), "mlp bwd");
  return SVDP_OK;
}

svdp_status svdp_pinball(const float* out, const float* target, int64_t rows, float tau0, float tau1, float* dout,
                         float* loss, void* stream) {
  if (rows == 0) return SVDP_OK;
  REQ(out); REQ(target); REQ(dout);
  if (rows < 0 || rows > (1 << 26)) return fail(SVDP_ERR_SHAPE, "bad rows");
  if (!(tau0 > 0 && tau0 < 1 && tau1 > 0 && tau1 < 1)) return fail(SVDP_ERR_INVALID_ARG, "tau must be in (0, 1)");
  HIPCHK(pinball_launch(out, target, (int)rows, tau0, tau1, dout, loss, (hipStream_t)stream), "pinball");
  return SVDP_OK;
}

svdp_status svdp_adam_step(float* params, float* m, float* v, const float* grad, int64_t n, float lr, float beta1,
                           float beta2, float eps, int64_t t, void* stream) {
  if (n == 0) return SVDP_OK;
  REQ(params); REQ(m); REQ(v); REQ(grad);
  if (n < 0 || t < 1) return fail(SVDP_ERR_INVALID_ARG, "need n >= 0 and t >= 1");
  HIPCHK(adam_launch(params, m, v, grad, n, lr, beta1, beta2, eps, (int)t, (hipStream_t)stream), "adam");
  return SVDP_OK;
}

svdp_status svdp_cans_table(int32_t kind, double delta, int32_t pre_iters, double lo, int32_t steps, double* table,
                            double* t_out) {
  REQ(table);
  if (steps < 0) return fail(SVDP_ERR_INVALID_ARG, "steps < 0");
  if (kind == 0) {
    if (!(delta > 0 && delta < 1) || pre_iters < 0) return fail(SVDP_ERR_INVALID_ARG, "bad delta / pre_iters");
    table_conservative(delta, pre_iters, steps, table, t_out);
  } else if (kind == 1) {
    if (!(lo > 0 && lo <= 1)) return fail(SVDP_ERR_INVALID_ARG, "lo must be in (0, 1]");
    table_interval(lo, steps, table);
    if (t_out) *t_out = lo;
  } else {
    return fail(SVDP_ERR_INVALID_ARG, "kind must be 0 or 1");
  }
  return SVDP_OK;
}

svdp_status svdp_poly_table(int32_t poly, double delta, int32_t pre_iters, int32_t steps, double* table,
                            double* t_out) {
  if (poly < SVDP_POLY_CANS3 || poly > SVDP_POLY_CANS5)
    return fail(SVDP_ERR_INVALID_ARG, "unknown poly (Polar Express: svdp_pe_table)");
  if (!table || steps < 1 || steps > 64 || pre_iters < 0 || pre_iters > steps || !(delta > 0 && delta < 1))
    return fail(SVDP_ERR_INVALID_ARG, "need table, 1 <= steps <= 64, 0 <= pre_iters <= steps, 0 < delta < 1");
  double t = 0.0;
  table_poly(poly, delta, pre_iters, steps, table, &t);
  if (t_out) *t_out = t;
  return SVDP_OK;
}

svdp_status svdp_pe_table(double lo, int32_t max_steps, double* table, int32_t* steps) {
  REQ(table); REQ(steps);
  if (!(lo > 0 && lo < 1) || max_steps < 1 || max_steps > 64)
    return fail(SVDP_ERR_INVALID_ARG, "need 0 < lo < 1 and 1 <= max_steps <= 64");
  const int t = pe_table(lo, max_steps, table);
  if (t < 0) return fail(SVDP_ERR_INVALID_ARG, "the schedule needs more than max_steps steps");
  *steps = t;
  return SVDP_OK;
}

}  // extern "C"
