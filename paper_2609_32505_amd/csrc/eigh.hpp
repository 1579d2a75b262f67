// Batched block-Jacobi eigh: workspace layout and host entry points.
#pragma once
#include "common.hpp"
#include "svdp.h"

struct EighWs {
  int batch, n, np, nb, max_sweeps;  // np = 16 nb, nb a power of two >= 4
  float* Hw;      // batch x np x np: H as 16 x 16 tiles (those on and above the diagonal)
  float* Vw;      // batch x np x np: accumulated rotations as 16 x 16 tiles
  float* V2;      // batch x np x np re-orthonormalised eigenvectors (row-major)
  float* lamr;    // batch x n Rayleigh-quotient eigenvalues
  float* Qw;      // batch x nph_store x (nb/4) x (64 x 64 group rotation M_G)
  float* hnorm2;  // batch: |H|_F^2
  double* off2;   // batch: |off(sym(V^T H V))|_F^2 of the last restart measure
  float* hn_part;    // batch x (nb/4)^2 x 4: |H|_F^2 per setup workgroup and wave
  double* off_part;  // batch x chunks: the restart measure per workgroup
  float* sgn;     // batch x n: sign of each sorted eigenvalue
  int* perm;      // batch x n: sorted position -> working column
  int* rotcnt;    // batch x (max_sweeps + 2): largest relative entry rotated (float bits)
  float* rotsq;   // batch x (nb/4) x 2: sum of squares of the entries rotated in the
                  // current sweep, per group and wave (added in order, then cleared)
  int* active;    // batch: 1 while not converged
  int* counter;   // device scalar: active matrices after a sweep
  int deferred;   // 1: V row-major, updated once per sweep from every phase's group
                  // rotations (np <= 1024); 0: V tiled, updated by every phase's apply
  int nph_store;  // group-rotation slots per matrix in Qw: the phases of a sweep (deferred), else 1
  double* work;   // profiling: device work counters per kind (null when profiling is off)
};

// Two fused block-Jacobi steps: block B is paired with B ^ sA, then with
// B ^ sB; groups {B, B^sA, B^sB, B^sA^sB} are indexed by the member whose
// bits lo and hi are clear.
struct EighPhase {
  int sA, sB;
  int lo, hi;
  int fullA;  // the first step also runs the intra-block rounds
  int skipB;  // the phase has a single step
  int idx;    // position in the sweep (slot of its group rotations when V is deferred)
};

// Phase p of a sweep over nb blocks: (1, -) with the full inner rounds, then
// (2, 3), (4, 5), ..., (nb - 2, nb - 1) with cross rounds.  The first phase
// has one step; its grouping uses sB = 2 (any other partner works).  lo, hi:
// the pivot bits of span{sA, sB} in echelon form.
__host__ __device__ inline EighPhase eigh_phase(int p) {
  EighPhase ph;
  ph.sA = p == 0 ? 1 : 2 * p;
  ph.sB = p == 0 ? 2 : 2 * p + 1;
  ph.fullA = p == 0;
  ph.skipB = p == 0;
  ph.idx = p;
  const int u = ph.sA;
  int v = ph.sB;
  const int p1 = 31 - __builtin_clz((unsigned)u);
  if ((v >> p1) & 1) v ^= u;
  const int p2 = 31 - __builtin_clz((unsigned)v);
  ph.lo = p1 < p2 ? p1 : p2;
  ph.hi = p1 < p2 ? p2 : p1;
  return ph;
}

struct EighOpts {
  int inner_sweeps;  // repetitions of a step's scalar rounds per pair subproblem (FP32)
  int fp64_sweeps;   // final block sweeps with FP64 pair solves
  int fp64_inner;    // repetitions in those
  float tol;         // converged after a sweep whose largest rotated |h_pq| is
                     // <= tol sqrt(|h_pp h_qq|) (quadratic convergence: the next
                     // sweep, the FP64 one, leaves ~tol^2)
  float abs_tol;     // entries below abs_tol |H|_F do not count
  float fro_tol;     // ... or after a sweep whose rotated entries have a sum of squares
                     // <= fro_tol^2 |H|_F^2 (normwise)
  float neg_tol;     // NEG_EIGENVALUE when lam_min < -neg_tol max|lam| (mode 1)
  float off_tol;     // restarts end once |off(V^T H V)|_F <= off_tol |H|_F
  int restarts;      // cap on restarts (re-formed V^T H V swept again from I)
};

// Extra streams and events: the sweeps run parts of the batch on the
// caller's stream and on up to kEighParts - 1 more streams, each part
// starting one pair solve after the previous one, so that the
// latency-bound pair solves of some parts overlap the block rotations of
// the others.
constexpr int kEighParts = 4;
struct EighAux {
  int parts;                         // 1 .. kEighParts
  hipStream_t st[kEighParts - 1];    // streams of parts 1 .. parts - 1
  hipEvent_t fork;
  hipEvent_t skew[kEighParts];
  hipEvent_t join[kEighParts];
};

int eigh_blocks(int64_t n);
int eigh_par_sweeps(int64_t n);
size_t eigh_ws_bytes(int64_t batch, int64_t n, int max_sweeps);
EighWs eigh_ws_carve(void* ws, int64_t batch, int64_t n, int max_sweeps);
hipError_t eigh_run(EighWs e, const float* H, int64_t ldh, int64_t sH, int mode,
                    const EighOpts& o, float* lam, int64_t slam, float* Vout, int64_t ldv,
                    int64_t sV, int* sweeps_out, int* flags, const int* mask,
                    const EighAux* aux, hipStream_t st);
hipError_t copy_i32(int* dst, const int* src, int64_t n, hipStream_t st);
hipError_t fill_i32(int* p, int v, int64_t n, hipStream_t st);
hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t st);
