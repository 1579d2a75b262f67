// Shared device/host definitions of the gfx950 library (no torch types).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16_t;
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

#define SVDP_DEV __device__ __forceinline__

// One batched GEMM launch: out[b] = epilogue(op(A[b]) * op(B[b])).
// Row-major storage.  op(A) is M x K: A[i*lda + k] (ta = 0) or A[k*lda + i]
// (ta = 1).  op(B) is K x N: B[k*ldb + j] (tb = 0) or B[j*ldb + k] (tb = 1).
// Epilogue (per matrix b, entry (i, j)):
//   out = s_acc * acc * cs[j] + s_in * Cin[i, j] * csin[j]
// where (s_in, s_acc) = coef[b*coef_bstride + coef_idx] when coef is set,
// else (beta, alpha); cs / csin default to 1 when null.
struct GemmArgs {
  int M, N, K, batch;
  const void* A; int64_t lda, sA;
  const void* A_alt;   // matrix b reads A_alt instead of A when a_sel[b] != 0
  const int* a_sel;
  const void* B; int64_t ldb, sB;
  const void* B_alt;   // likewise for B
  const int* b_sel;
  void* C; int64_t ldc, sC;
  const void* Cin; int64_t ldcin, sCin;
  float alpha, beta;
  const float* coef; int64_t coef_bstride; int coef_idx;
  const float* colscale; int64_t cs_stride;
  const float* colscale_in; int64_t csin_stride;
  const int* active;   // matrix b is skipped when active[b] == 0
  const int* ksched;   // bounded CANS schedule: per-matrix (K, K1); when set,
  int kstep, kcatmask; // matrix b runs only if bit sched_cat(ksched, b, kstep,
  int kbf16;           // kbf16) of kcatmask is set, and writes its output in
  int obf_catmask;     // BF16 to C_bf (and Ct) when that bit of obf_catmask is set
  void* C_bf;          // (same leading dimension and stride as C), else to C
  float* conv;         // per matrix and wave sub-tile (gemm_conv_slots slots): sum (out - Cin)^2, sum out^2
  int sym;             // output symmetric: upper tiles computed, mirrored
  int out_bf16, in_bf16, cin_bf16;
  void* Ct; int64_t ldct, sCt;  // out_bf16: also write the output transposed, Ct[j, i] (BF16)
  double* work;        // profiling: += the algorithmic flops of each tile computed
};

enum { PREC_F32 = 0, PREC_BF16 = 1 };

// Launch a batched GEMM.  prec selects FP32 MFMA (inputs FP32) or BF16 MFMA
// (inputs FP32 or BF16 per in_bf16, rounded to BF16, FP32 accumulation).
hipError_t gemm_launch(const GemmArgs& g, int prec, int ta, int tb, hipStream_t st);
// slots per matrix of GemmArgs::conv for an M x N output (one per wave sub-tile)
int gemm_conv_slots(int64_t M, int64_t N);

// Category of step k of matrix b in the bounded CANS schedule, from its step
// counts (K, K1): K steps in all, the first K1 in FP32 (all of them when
// bf16 == 0).  -1: no step; 0: FP32 in, FP32 out; 1: FP32 in, BF16 out (the
// last FP32 step before BF16 ones); 2: BF16 in and out; 3: BF16 in, FP32
// out (the last step).
SVDP_DEV int sched_cat(const int* ks, int b, int k, int bf16) {
  const int K = max(ks[2 * b], 1);
  const int K1 = bf16 ? min(max(ks[2 * b + 1], 0), K) : K;
  if (k >= K) return -1;
  if (k < K1) return (k + 1 >= K1 && k + 1 < K) ? 1 : 0;
  return k + 1 < K ? 2 : 3;
}

SVDP_DEV float bf2f(bf16_t x) { return (float)x; }
SVDP_DEV bf16_t f2bf(float x) { return (bf16_t)x; }

template <typename T>
SVDP_DEV float ldf(const T* p, int64_t i) { return (float)p[i]; }

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
