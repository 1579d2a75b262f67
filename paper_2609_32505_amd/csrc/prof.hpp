// Optional per-kernel-class timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

enum ProfKind {
  PROF_JAC_SOLVE_F32 = 0,
  PROF_JAC_SOLVE_F64 = 1,
  PROF_JAC_APPLY = 2,
  PROF_GEMM_F32 = 3,
  PROF_GEMM_BF16 = 4,
  // phases of a forward / backward call, bracketed on the caller's stream
  PROF_PHASE_BOUND = 5,     // normalisation, sketch features, predictor, schedule
  PROF_PHASE_CANS = 6,      // CANS steps before the FP32 refinement
  PROF_PHASE_REFINE = 7,    // FP32 refinement steps and the final residual
  PROF_PHASE_H = 8,         // H = W^T A
  PROF_PHASE_EIGH = 9,      // eigendecomposition of H
  PROF_PHASE_U = 10,        // BF16 correction, U = W V, column-norm test, QR step
  PROF_PHASE_FALLBACK = 11, // conservative reruns of the bounded paths
  PROF_PHASE_BWD = 12,      // svd_polar_bwd / polar_bwd
  PROF_PHASE_QR = 13,       // QR preprocessing of tall matrices (Q, Q^T A, Q U_B)
  PROF_JAC_VSWEEP = 14,     // Jacobi: once-per-sweep V update from the phases' rotations
  PROF_KINDS = 15
};

// Device-side work counters (one double per kind) while profiling is on,
// null otherwise: a kernel adds the algorithmic flops of each workgroup that
// runs (workgroups of converged or masked matrices exit without adding).
double* prof_work_dev();

// Brackets one launch with events when profiling is on; a no-op otherwise.
// `work` is host-side algorithmic work (flops) added to the class's total
// (kernels that count on the device pass 0).
struct ProfScope {
  ProfScope(int kind, hipStream_t st, double work = 0.0);
  ~ProfScope();
  // end this record here and start one of another kind on the same stream
  void next(int kind);
  int kind;
  hipStream_t st;
  int slot;
  bool phase;
};
