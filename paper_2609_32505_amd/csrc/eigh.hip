// Batched symmetric eigendecomposition H = V diag(lam) V^T by block Jacobi
// (the EVD step of the SVD-via-polar algorithm, Algorithm 1).
//
// The (padded) index range is cut into 16-wide blocks; a parallel step pairs
// the blocks round-robin, and each pair (P, Q) owns the 32 x 32 subproblem
// H[P u Q, P u Q].
//   * k_jac_solve: one WAVEFRONT per pair runs a cyclic scalar Jacobi sweep on
//     the subproblem held in its own slice of LDS (16 disjoint rotations per
//     inner step; each 2 x 2 block of the subproblem is updated independently),
//     accumulates the 32 x 32 orthogonal J in FP64, writes the rotated
//     diagonal block back into H and J to a per-pair buffer.  The wave works
//     alone on its data, so its inner steps need no workgroup barrier: LDS
//     operations of one wave complete in program order.  FP32 subproblem
//     arithmetic, or FP64 for the final sweep.
//   * k_jac_apply: every off-diagonal pair block H[P, R] <- J_P^T H[P, R] J_R
//     (upper triangle, mirrored) and every 32-row slab V[:, P] <- V[:, P] J_P,
//     one wavefront per 32 x 32 x 32 product on FP32 MFMA (32x32x2).
// A sweep is nb - 1 steps.  Convergence is tested per matrix on the largest
// relative off-diagonal entry rotated during a sweep; converged matrices are
// skipped by later launches.
#include <algorithm>
#include <cstring>
#include "common.hpp"
#include "eigh.hpp"
#include "prof.hpp"

namespace {

constexpr int BS = 16;       // block width
constexpr int PB = 2 * BS;   // pair subproblem size (32)
constexpr int NPP = PB / 2;  // disjoint rotations per inner step (16)
constexpr int LP = PB + 1;   // LDS row pitch

// Round-robin (circle method) pairing of `players` (even) in `round`:
// position 0 is fixed, the others rotate; pair k joins positions k and
// players - 1 - k.
SVDP_DEV int rr_player(int pos, int round, int players) {
  return pos == 0 ? 0 : 1 + (pos - 1 + round) % (players - 1);
}
SVDP_DEV void rr_pair(int k, int round, int players, int& x, int& y) {
  int a = rr_player(k, round, players), c = rr_player(players - 1 - k, round, players);
  x = a < c ? a : c;
  y = a < c ? c : a;
}

// local index (0..31) of a pair subproblem -> global index
SVDP_DEV int gidx(int a, int p, int q) { return a < BS ? p * BS + a : q * BS + (a - BS); }

// orders the wave's own LDS traffic: no instruction is moved across it, and
// LDS operations of one wave complete in issue order
SVDP_DEV void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename R>
SVDP_DEV void rotation(R app, R aqq, R apq, R& c, R& s) {
  R tau = (aqq - app) / (R(2) * apq);
  R t;
  if (fabs(tau) > R(1e10)) t = R(0.5) / tau;
  else t = (tau >= R(0) ? R(1) : R(-1)) / (fabs(tau) + sqrt(R(1) + tau * tau));
  c = R(1) / sqrt(R(1) + t * t);
  s = t * c;
}

template <typename R>
__global__ __launch_bounds__(256) void k_jac_solve(EighWs e, int step, int inner_sweeps,
                                                   float abs_tol, int* rotmax) {
  __shared__ R Sall[4][PB][LP];
  __shared__ double Jall[4][PB][LP];
  __shared__ R csall[4][2][NPP];
  __shared__ unsigned char ptab[PB - 1][NPP][2];
  const int t = threadIdx.x;
  for (int i = t; i < (PB - 1) * NPP; i += 256) {
    int x, y;
    rr_pair(i % NPP, i / NPP, PB, x, y);
    ptab[i / NPP][i % NPP][0] = (unsigned char)x;
    ptab[i / NPP][i % NPP][1] = (unsigned char)y;
  }
  __syncthreads();
  const int wave = t >> 6, lane = t & 63;
  const int npairs = e.nb / 2;
  const int task = blockIdx.x * 4 + wave;
  const int b = task / npairs, k = task - b * npairs;
  if (b >= e.batch) return;
  if (e.active && !e.active[b]) return;
  R (*S)[LP] = Sall[wave];
  double (*J)[LP] = Jall[wave];
  R* cs_c = csall[wave][0];
  R* cs_s = csall[wave][1];
  int p, q;
  rr_pair(k, step, e.nb, p, q);
  float* H = e.Hw + (int64_t)b * e.np * e.np;
  for (int idx = lane; idx < PB * PB; idx += 64) {
    int a = idx / PB, c = idx % PB;
    S[a][c] = (R)H[(int64_t)gidx(a, p, q) * e.np + gidx(c, p, q)];
    J[a][c] = a == c ? 1.0 : 0.0;
  }
  const R floor_abs = (R)abs_tol * (R)sqrtf(e.hnorm2[b]);
  float mrel = 0.f;
  wave_sync();
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    int any = 0;
    for (int s = 0; s < PB - 1; ++s) {
      if (lane < NPP) {
        const int x = ptab[s][lane][0], y = ptab[s][lane][1];
        R app = S[x][x], aqq = S[y][y], apq = S[y][x] * R(0.5) + S[x][y] * R(0.5);
        R c = 1, sn = 0;
        if (apq != R(0) && isfinite((float)apq)) {
          rotation(app, aqq, apq, c, sn);
          any = 1;
          if (fabs(apq) > floor_abs) {
            R den = sqrt(fabs(app * aqq));
            mrel = fmaxf(mrel, den > R(0) ? (float)(fabs(apq) / den) : 1e30f);
          }
        }
        cs_c[lane] = c;
        cs_s[lane] = sn;
      }
      wave_sync();
      // 16 x 16 blocks of 2 x 2, four per lane
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int blk = lane + 64 * u;
        const int kx = blk >> 4, ky = blk & 15;
        const int x1 = ptab[s][kx][0], y1 = ptab[s][kx][1];
        const int x2 = ptab[s][ky][0], y2 = ptab[s][ky][1];
        const R c1 = cs_c[kx], s1 = cs_s[kx], c2 = cs_c[ky], s2 = cs_s[ky];
        const R a = S[x1][x2], bq = S[x1][y2], cq = S[y1][x2], d = S[y1][y2];
        const R t00 = c1 * a - s1 * cq, t01 = c1 * bq - s1 * d;
        const R t10 = s1 * a + c1 * cq, t11 = s1 * bq + c1 * d;
        R y00 = c2 * t00 - s2 * t01, y01 = s2 * t00 + c2 * t01;
        R y10 = c2 * t10 - s2 * t11, y11 = s2 * t10 + c2 * t11;
        if (kx == ky && s1 != R(0)) { y01 = 0; y10 = 0; }
        S[x1][x2] = y00; S[x1][y2] = y01; S[y1][x2] = y10; S[y1][y2] = y11;
      }
      // rotation accumulation: 32 rows x 16 pairs, eight per lane
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int it = lane + 64 * u;
        const int r = it >> 4, kk = it & 15;
        const int x = ptab[s][kk][0], y = ptab[s][kk][1];
        const double c = cs_c[kk], sn = cs_s[kk];
        const double jx = J[r][x], jy = J[r][y];
        J[r][x] = c * jx - sn * jy;
        J[r][y] = sn * jx + c * jy;
      }
      wave_sync();
    }
    // every lane of the wave takes the same exit
    if (!__any(any)) break;
  }
  for (int idx = lane; idx < PB * PB; idx += 64) {
    int a = idx / PB, c = idx % PB;
    H[(int64_t)gidx(a, p, q) * e.np + gidx(c, p, q)] = (float)S[a][c];
    e.Qw[((int64_t)b * npairs + k) * (PB * PB) + idx] = (float)J[a][c];
  }
  // largest relative off-diagonal entry rotated by this wave (float bits)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mrel = fmaxf(mrel, __shfl_xor(mrel, off));
  if (lane == 0 && rotmax) atomicMax(rotmax + b, __float_as_int(mrel));
}

// 32 x 32 x 32 product on one wavefront: A read as A[i][k] (or A[k][i] when
// a_trans), B as B[k][j]; returns the 32 x 32 MFMA accumulator (lane l,
// slot 4g + r -> row 8g + 4(l / 32) + r, column l % 32).
SVDP_DEV f16v mm32(const float (*A)[LP], bool a_trans, const float (*Bm)[LP], int lane) {
  f16v acc;
#pragma unroll
  for (int e2 = 0; e2 < 16; ++e2) acc[e2] = 0.f;
  const int kh = lane >> 5, ic = lane & 31;
#pragma unroll
  for (int kk = 0; kk < PB; kk += 2) {
    float av = a_trans ? A[kk + kh][ic] : A[ic][kk + kh];
    float bv = Bm[kk + kh][ic];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

__global__ __launch_bounds__(256) void k_jac_apply(EighWs e, int step) {
  __shared__ float Xall[4][PB][LP];
  __shared__ float JLall[4][PB][LP];
  __shared__ float JRall[4][PB][LP];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int npairs = e.nb / 2;
  const int nh = npairs * (npairs - 1) / 2;
  const int nrs = e.np / PB;
  const int ntask = nh + nrs * npairs;
  const int gt = blockIdx.x * 4 + wave;
  const int b = gt / ntask, task = gt - b * ntask;
  if (b >= e.batch) return;
  if (e.active && !e.active[b]) return;
  float (*X)[LP] = Xall[wave];
  float (*JL)[LP] = JLall[wave];
  float (*JR)[LP] = JRall[wave];
  float* H = e.Hw + (int64_t)b * e.np * e.np;
  float* V = e.Vw + (int64_t)b * e.np * e.np;
  const float* Q = e.Qw + (int64_t)b * npairs * (PB * PB);
  const int jc = lane & 31;
  if (task < nh) {
    // upper-triangular pair index (kp < kr)
    int tt = task, kp = 0;
    while (tt >= npairs - 1 - kp) { tt -= npairs - 1 - kp; ++kp; }
    const int kr = kp + 1 + tt;
    int p1, q1, p2, q2;
    rr_pair(kp, step, e.nb, p1, q1);
    rr_pair(kr, step, e.nb, p2, q2);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = lane + 64 * u;  // 32 rows x 8 float4
      const int a = idx >> 3, c = (idx & 7) * 4;
      const f4v v = *(const f4v*)&H[(int64_t)gidx(a, p1, q1) * e.np + gidx(c, p2, q2)];
      const f4v jl = *(const f4v*)&Q[(int64_t)kp * (PB * PB) + a * PB + c];
      const f4v jr = *(const f4v*)&Q[(int64_t)kr * (PB * PB) + a * PB + c];
#pragma unroll
      for (int w2 = 0; w2 < 4; ++w2) { X[a][c + w2] = v[w2]; JL[a][c + w2] = jl[w2]; JR[a][c + w2] = jr[w2]; }
    }
    wave_sync();
    const f16v T = mm32(JL, true, X, lane);  // J_P^T X
    wave_sync();
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) X[8 * g + 4 * (lane >> 5) + r][jc] = T[4 * g + r];
    wave_sync();
    const f16v Y = mm32(X, false, JR, lane);  // (J_P^T X) J_R
    const int gj = gidx(jc, p2, q2);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int i0 = 8 * g + 4 * (lane >> 5);
      f4v col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        H[(int64_t)gidx(i0 + r, p1, q1) * e.np + gj] = Y[4 * g + r];
        col[r] = Y[4 * g + r];
      }
      // mirror: row gj, columns gidx(i0 .. i0+3) are contiguous (one 16-block)
      *(f4v*)&H[(int64_t)gj * e.np + gidx(i0, p1, q1)] = col;
    }
  } else {
    const int v = task - nh, rs = v / npairs, kp = v - rs * npairs;
    int p1, q1;
    rr_pair(kp, step, e.nb, p1, q1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = lane + 64 * u;
      const int a = idx >> 3, c = (idx & 7) * 4;
      const f4v x = *(const f4v*)&V[(int64_t)(rs * PB + a) * e.np + gidx(c, p1, q1)];
      const f4v jl = *(const f4v*)&Q[(int64_t)kp * (PB * PB) + a * PB + c];
#pragma unroll
      for (int w2 = 0; w2 < 4; ++w2) { X[a][c + w2] = x[w2]; JL[a][c + w2] = jl[w2]; }
    }
    wave_sync();
    const f16v Y = mm32(X, false, JL, lane);
    const int gj = gidx(jc, p1, q1);
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        V[(int64_t)(rs * PB + 8 * g + 4 * (lane >> 5) + r) * e.np + gj] = Y[4 * g + r];
  }
}

// Copy (and symmetrise) H into the padded work matrix, V = I, |H|_F^2.
// One 32 x 32 tile per workgroup; the transposed partner tile goes through
// LDS so that every global access is row-contiguous.
__global__ void k_eigh_setup(EighWs e, const float* Hin, int64_t ldh, int64_t sH, const int* mask) {
  const int b = blockIdx.z;
  if (mask && !mask[b]) return;
  __shared__ float tt[32][33];
  const int I0 = blockIdx.y * 32, J0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const float* Hb = Hin + b * sH;
  for (int r = ty; r < 32; r += 8) {
    int i = J0 + r, j = I0 + tx;  // partner tile (J, I)
    tt[r][tx] = (i < e.n && j < e.n) ? Hb[(int64_t)i * ldh + j] : 0.f;
  }
  __syncthreads();
  float* Hw = e.Hw + (int64_t)b * e.np * e.np;
  float* Vw = e.Vw + (int64_t)b * e.np * e.np;
  float acc = 0.f;
  for (int r = ty; r < 32; r += 8) {
    int i = I0 + r, j = J0 + tx;
    float v = 0.f;
    if (i < e.n && j < e.n) v = 0.5f * (Hb[(int64_t)i * ldh + j] + tt[tx][r]);
    Hw[(int64_t)i * e.np + j] = v;
    Vw[(int64_t)i * e.np + j] = i == j ? 1.f : 0.f;
    acc += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(e.hnorm2 + b, acc);
}

// Mark matrices whose sweep made no significant rotation as converged and
// count the ones still active (single workgroup).
__global__ void k_eigh_check(EighWs e, const int* rotcnt, float tol, int sweep, int* sweeps_out,
                             int* n_active) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int b = threadIdx.x; b < e.batch; b += blockDim.x) {
    if (e.active[b]) {
      if (__int_as_float(rotcnt[b]) <= tol) {
        e.active[b] = 0;
        sweeps_out[b] = sweep + 1;
      } else {
        sweeps_out[b] = sweep + 1;
        ++mine;
      }
    }
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *n_active = cnt;
}

// Sort the diagonal (eigenvalues) descending -- by value (mode 0) or by
// magnitude (mode 1, singular values of H = W^T A with sign kept apart) --
// with a bitonic sort in LDS; write lam, the permutation and the signs, and
// raise flags for non-finite values and for eigenvalues below
// -neg_tol * max |lam| (mode 1).
__global__ __launch_bounds__(1024) void k_eigh_sort(EighWs e, int mode, float neg_tol, float* lam,
                                                    int64_t slam, int* perm, float* sgn, int* flags,
                                                    const int* mask) {
  extern __shared__ unsigned char smem[];
  const int b = blockIdx.x;
  if (mask && !mask[b]) return;
  int P2 = 1;
  while (P2 < e.np) P2 <<= 1;
  float* key = (float*)smem;
  int* idx = (int*)(key + P2);
  const float* lr = e.lamr + (int64_t)b * e.n;
  __shared__ float vmax, vmin;
  __shared__ int bad;
  if (threadIdx.x == 0) { vmax = 0.f; vmin = 0.f; bad = 0; }
  __syncthreads();
  for (int i = threadIdx.x; i < P2; i += blockDim.x) {
    float d = i < e.n ? lr[i] : 0.f;
    if (i < e.n && !isfinite(d)) { bad = 1; d = 0.f; }
    key[i] = i < e.n ? (mode ? fabsf(d) : d) : -INFINITY;
    idx[i] = i;
    if (i < e.n) {
      atomicMax((int*)&vmax, __float_as_int(fabsf(d)));  // |d| >= 0: int order = float order
      if (d < 0.f) atomicMax((int*)&vmin, __float_as_int(-d));
    }
  }
  __syncthreads();
  // bitonic sort, descending by key, ties by ascending index
  for (int size = 2; size <= P2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P2; i += blockDim.x) {
        int j = i ^ stride;
        if (j > i) {
          bool desc = (i & size) == 0;
          float ki = key[i], kj = key[j];
          int ii = idx[i], ij = idx[j];
          bool i_first = ki > kj || (ki == kj && ii < ij);
          if (desc != i_first) {
            key[i] = kj; key[j] = ki;
            idx[i] = ij; idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  for (int c = threadIdx.x; c < e.n; c += blockDim.x) {
    int src = idx[c];
    float d = lr[src];
    if (!isfinite(d)) d = 0.f;
    lam[b * slam + c] = mode ? fabsf(d) : d;
    perm[(int64_t)b * e.n + c] = src;
    sgn[(int64_t)b * e.n + c] = d < 0.f ? -1.f : 1.f;
  }
  if (threadIdx.x == 0 && flags) {
    int f = 0;
    if (bad) f |= SVDP_FLAG_NONFINITE;
    if (vmin > neg_tol * vmax) f |= SVDP_FLAG_NEG_EIGENVALUE;
    if (f) atomicOr(flags + b, f);
  }
}

// V_out[:, c] = V_work[:n, perm[c]]
__global__ void k_eigh_permute(EighWs e, const int* perm, float* Vout, int64_t ldv, int64_t sV,
                               const int* mask) {
  const int b = blockIdx.y, i = blockIdx.x;
  if (mask && !mask[b]) return;
  const float* Vw = e.V2 + (int64_t)b * e.np * e.np + (int64_t)i * e.np;
  const int* pb = perm + (int64_t)b * e.n;
  float* out = Vout + b * sV + (int64_t)i * ldv;
  for (int c = threadIdx.x; c < e.n; c += blockDim.x) out[c] = Vw[pb[c]];
}

// lamr[b, i] = v_i^T (H0 v_i) with T = H0 V in Hw (FP64 accumulation)
__global__ void k_rayleigh(EighWs e, const int* mask) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= e.n) return;
  const float* V = e.V2 + (int64_t)b * e.np * e.np;
  const float* T = e.Hw + (int64_t)b * e.np * e.np;
  double s = 0.0;
  for (int j = 0; j < e.n; ++j) s += (double)V[(int64_t)j * e.np + i] * (double)T[(int64_t)j * e.np + i];
  e.lamr[(int64_t)b * e.n + i] = (float)s;
}

__global__ void k_flag_active(const int* active, int batch, int* flags, int f) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch && active[b]) atomicOr(flags + b, f);
}

__global__ void k_copy_i32(int* dst, const int* src, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void k_fill_i32(int* p, int v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t fill_i32(int* p, int v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(n, 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}
hipError_t copy_i32(int* dst, const int* src, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i32, dim3(cdiv(n, 256)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}
hipError_t fill_f32(float* p, float v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(cdiv(n, 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

size_t eigh_ws_bytes(int64_t batch, int64_t n, int max_sweeps) {
  int64_t np = (n + 31) / 32 * 32;
  int64_t npairs = np / 32;
  size_t f = 0;
  f += 3 * batch * np * np;          // Hw, Vw, V2
  f += batch * n;                    // lamr
  f += batch * npairs * 1024;        // Qw
  f += batch;                        // hnorm2
  f += 2 * batch * n;                // sign, (perm as int)
  size_t i = batch * (size_t)(max_sweeps + 2) + batch + 16;  // rotcnt, active, counters
  return (f + i) * 4 + 8 * 256;
}

EighWs eigh_ws_carve(void* ws, int64_t batch, int64_t n, int max_sweeps) {
  EighWs e;
  e.batch = (int)batch;
  e.n = (int)n;
  e.np = (int)((n + 31) / 32 * 32);
  e.nb = e.np / 16;
  int64_t np = e.np, npairs = np / 32;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) { char* r = p; p += (bytes + 255) / 256 * 256; return (void*)r; };
  e.Hw = (float*)take(batch * np * np * 4);
  e.Vw = (float*)take(batch * np * np * 4);
  e.V2 = (float*)take(batch * np * np * 4);
  e.lamr = (float*)take(batch * n * 4);
  e.Qw = (float*)take(batch * npairs * 1024 * 4);
  e.hnorm2 = (float*)take(batch * 4);
  e.sgn = (float*)take(batch * n * 4);
  e.perm = (int*)take(batch * n * 4);
  e.rotcnt = (int*)take(batch * (size_t)(max_sweeps + 2) * 4);
  e.active = (int*)take(batch * 4);
  e.counter = (int*)take(64);
  e.max_sweeps = max_sweeps;
  return e;
}

// Full eigendecomposition of a batch of symmetric n x n matrices.
hipError_t eigh_run(EighWs e, const float* H, int64_t ldh, int64_t sH, int mode,
                    const EighOpts& o, float* lam, int64_t slam, float* Vout, int64_t ldv,
                    int64_t sV, int* sweeps_out, int* flags, int* host_counter, const int* mask,
                    hipStream_t st) {
  hipError_t err;
  const int batch = e.batch;
  if ((err = fill_f32(e.hnorm2, 0.f, batch, st))) return err;
  if ((err = fill_i32(e.rotcnt, 0, (int64_t)batch * (e.max_sweeps + 2), st))) return err;
  if (mask) { if ((err = copy_i32(e.active, mask, batch, st))) return err; }
  else if ((err = fill_i32(e.active, 1, batch, st))) return err;
  {
    const int tiles = e.np / 32;
    hipLaunchKernelGGL(k_eigh_setup, dim3(tiles, tiles, batch), dim3(256), 0, st, e, H, ldh, sH, mask);
    if ((err = hipGetLastError())) return err;
  }
  const int npairs = e.nb / 2;
  const int nh = npairs * (npairs - 1) / 2;
  const int ntask = nh + (e.np / 32) * npairs;
  const int steps = e.nb - 1;
  const unsigned solve_blocks = (unsigned)cdiv((int64_t)batch * npairs, 4);
  const unsigned apply_blocks = (unsigned)cdiv((int64_t)batch * ntask, 4);
  // algorithmic flops per matrix and step: pair solves (2 x 2 block updates,
  // 24 flops each, and rotation accumulation, 6 per entry pair) and the
  // block rotations (two 32^3 products per off-diagonal pair block, one per
  // 32-row slab of V)
  const double solve_work = (double)npairs * 31.0 * (256.0 * 24.0 + 512.0 * 6.0);
  const double apply_work = (double)nh * 4.0 * 32768.0 + (double)(e.np / 32) * npairs * 2.0 * 32768.0;
  int n_active = batch;
  if (mask) {  // active count of a masked run is only needed for the work tally
    n_active = batch;
  }
  int sweep = 0;
  for (; sweep < e.max_sweeps; ++sweep) {
    int* rc = e.rotcnt + (int64_t)batch * sweep;
    for (int s = 0; s < steps; ++s) {
      {
        ProfScope ps(PROF_JAC_SOLVE_F32, st, solve_work * o.inner_sweeps * n_active);
        hipLaunchKernelGGL(k_jac_solve<float>, dim3(solve_blocks), dim3(256), 0, st, e, s,
                           o.inner_sweeps, o.abs_tol, rc);
      }
      if ((err = hipGetLastError())) return err;
      if (ntask > 0) {
        ProfScope ps(PROF_JAC_APPLY, st, apply_work * n_active);
        hipLaunchKernelGGL(k_jac_apply, dim3(apply_blocks), dim3(256), 0, st, e, s);
        if ((err = hipGetLastError())) return err;
      }
    }
    hipLaunchKernelGGL(k_eigh_check, dim3(1), dim3(1024), 0, st, e, rc, o.tol, sweep, sweeps_out, e.counter);
    if ((err = hipGetLastError())) return err;
    if ((err = hipMemcpyAsync(host_counter, e.counter, sizeof(int), hipMemcpyDeviceToHost, st))) return err;
    if ((err = hipStreamSynchronize(st))) return err;
    n_active = *host_counter;
    if (*host_counter == 0) break;
  }
  // matrices still active after max_sweeps did not converge
  if (sweep == e.max_sweeps) {
    // flag them: active[b] == 1
    hipLaunchKernelGGL(k_flag_active, dim3(cdiv(batch, 256)), dim3(256), 0, st, e.active, batch,
                       flags, (int)SVDP_FLAG_EIGH_NOT_CONVERGED);
    if ((err = hipGetLastError())) return err;
  }
  // final sweep(s) with FP64 pair solves on every matrix
  if (o.fp64_sweeps > 0) {
    if (mask) { if ((err = copy_i32(e.active, mask, batch, st))) return err; }
    else if ((err = fill_i32(e.active, 1, batch, st))) return err;
    for (int f = 0; f < o.fp64_sweeps; ++f)
      for (int s = 0; s < steps; ++s) {
        {
          ProfScope ps(PROF_JAC_SOLVE_F64, st, solve_work * o.fp64_inner * batch);
          hipLaunchKernelGGL(k_jac_solve<double>, dim3(solve_blocks), dim3(256), 0, st, e, s,
                             o.fp64_inner, o.abs_tol, (int*)nullptr);
        }
        if ((err = hipGetLastError())) return err;
        if (ntask > 0) {
          ProfScope ps(PROF_JAC_APPLY, st, apply_work * batch);
          hipLaunchKernelGGL(k_jac_apply, dim3(apply_blocks), dim3(256), 0, st, e, s);
          if ((err = hipGetLastError())) return err;
        }
      }
  }
  // One Newton-Schulz step re-orthonormalises the accumulated rotations,
  // V2 = V (3 I - V^T V) / 2, then the eigenvalues are the Rayleigh
  // quotients v_i^T H v_i against the input matrix.
  {
    const int np = e.np;
    GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.M = np; g.N = np; g.K = np; g.batch = batch;
    g.A = e.Vw; g.lda = np; g.sA = (int64_t)np * np;
    g.B = e.Vw; g.ldb = np; g.sB = (int64_t)np * np;
    g.C = e.Hw; g.ldc = np; g.sC = (int64_t)np * np;
    g.alpha = 1.f; g.sym = 1; g.active = mask;
    if ((err = gemm_launch(g, PREC_F32, 1, 0, st))) return err;
    GemmArgs u;
    memset(&u, 0, sizeof(u));
    u.M = np; u.N = np; u.K = np; u.batch = batch;
    u.A = e.Vw; u.lda = np; u.sA = (int64_t)np * np;
    u.B = e.Hw; u.ldb = np; u.sB = (int64_t)np * np;
    u.C = e.V2; u.ldc = np; u.sC = (int64_t)np * np;
    u.Cin = e.Vw; u.ldcin = np; u.sCin = (int64_t)np * np;
    u.alpha = -0.5f; u.beta = 1.5f; u.active = mask;
    if ((err = gemm_launch(u, PREC_F32, 0, 0, st))) return err;
    GemmArgs r;
    memset(&r, 0, sizeof(r));
    r.M = e.n; r.N = e.n; r.K = e.n; r.batch = batch;
    r.A = H; r.lda = ldh; r.sA = sH;
    r.B = e.V2; r.ldb = np; r.sB = (int64_t)np * np;
    r.C = e.Hw; r.ldc = np; r.sC = (int64_t)np * np;
    r.alpha = 1.f; r.active = mask;
    if ((err = gemm_launch(r, PREC_F32, 0, 0, st))) return err;
    hipLaunchKernelGGL(k_rayleigh, dim3(cdiv(e.n, 256), batch), dim3(256), 0, st, e, mask);
    if ((err = hipGetLastError())) return err;
  }
  {
    int P2 = 1;
    while (P2 < e.np) P2 <<= 1;
    size_t sh = (size_t)P2 * 8;
    hipLaunchKernelGGL(k_eigh_sort, dim3(batch), dim3(1024), sh, st, e, mode, o.neg_tol, lam, slam,
                       e.perm, e.sgn, flags, mask);
    if ((err = hipGetLastError())) return err;
  }
  if (Vout) {
    hipLaunchKernelGGL(k_eigh_permute, dim3(e.n, batch), dim3(256), 0, st, e, e.perm, Vout, ldv, sV, mask);
    if ((err = hipGetLastError())) return err;
  }
  return hipSuccess;
}
