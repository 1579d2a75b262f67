// Optional per-kernel-class timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

enum ProfKind {
  PROF_JAC_SOLVE_F32 = 0,
  PROF_JAC_SOLVE_F64 = 1,
  PROF_JAC_APPLY = 2,
  PROF_GEMM_F32 = 3,
  PROF_GEMM_BF16 = 4,
  PROF_KINDS = 5
};

// Brackets one launch with events when profiling is on; a no-op otherwise.
// `work` is the launch's algorithmic work (flops), summed per class.
struct ProfScope {
  ProfScope(int kind, hipStream_t st, double work = 0.0);
  ~ProfScope();
  int kind;
  hipStream_t st;
  int slot;
};
