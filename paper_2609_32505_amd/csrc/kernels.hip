// Element-wise, reduction and small-network kernels of the SVD path:
// normalisation (Algorithm 3), CANS bookkeeping, the rank-deficiency test on
// U, the eigenbasis Sylvester scaling of the backward (Algorithms 2 and 4),
// the sketch features, and the interval-predictor MLP (forward, backward,
// pinball loss, Adam) with the bound -> coefficient-table step.
#include <algorithm>
#include "common.hpp"
#include "kernels.hpp"
#include "eigh.hpp"

namespace {

SVDP_DEV float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
SVDP_DEV float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}
// non-negative float max through its int bit pattern
SVDP_DEV void atomic_max_pos(float* p, float v) { atomicMax((int*)p, __float_as_int(v)); }

SVDP_DEV bool skip(const int* mask, int b) { return mask && !mask[b]; }

// ------------------------------------------------------------ normalisation

// Row sums of |A| (their maximum, the infinity norm) and the non-finite
// flag: a workgroup reduces rows_per rows (a wave per row at a time), then
// takes one atomic maximum and one atomic or (both order-independent).
__global__ void k_rownorms(const float* A, int64_t lda, int64_t sA, int m, int n, int rows_per, float* rowmax,
                           int* flags, const int* mask) {
  const int b = blockIdx.y;
  if (skip(mask, b)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r0 = blockIdx.x * rows_per, r1 = min(m, r0 + rows_per);
  float mx = 0.f;
  bool bad = false;
  for (int i = r0 + w; i < r1; i += 4) {
    const float* r = A + b * sA + (int64_t)i * lda;
    float s = 0.f;
    for (int j = lane; j < n; j += 64) {
      const float v = r[j];
      bad |= !isfinite(v);
      s += fabsf(v);
    }
    s = wave_sum(s);
    mx = fmaxf(mx, isfinite(s) ? s : 0.f);
  }
  const int anybad = __ballot(bad) != 0ull;
  __shared__ float smx[4];
  __shared__ int sbad[4];
  if (lane == 0) { smx[w] = mx; sbad[w] = anybad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    const float m4 = fmaxf(fmaxf(smx[0], smx[1]), fmaxf(smx[2], smx[3]));
    atomic_max_pos(rowmax + b, m4);
    if (sbad[0] | sbad[1] | sbad[2] | sbad[3]) atomicOr(flags + b, SVDP_FLAG_NONFINITE);
  }
}

// Column pass, one workgroup of 16 waves per 64 columns of one matrix:
// colsum[j] = sum_i |a_ij| and part[blk] = the block's sum of squares.  Wave
// w takes rows w, w + 16, ...; the 16 partial columns are added in wave order
// and the squares by a fixed shuffle tree, so the results do not depend on
// scheduling (no atomics).
__global__ __launch_bounds__(1024) void k_colnorms(const float* A, int64_t lda, int64_t sA, int m, int n,
                                                   float* colsum, float* part, int nblk, const int* mask) {
  const int b = blockIdx.y;
  if (skip(mask, b)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 64 + lane;
  float s = 0.f, q = 0.f;
  if (j < n) {
    const float* p = A + b * sA + j;
#pragma unroll 4
    for (int i = w; i < m; i += 16) {
      const float v = p[(int64_t)i * lda];
      s += fabsf(v);
      q += v * v;
    }
  }
  __shared__ float ls[16][64], lq[16][64];
  ls[w][lane] = s;
  lq[w][lane] = q;
  __syncthreads();
  if (w == 0) {
    float cs = 0.f, cq = 0.f;
    for (int k = 0; k < 16; ++k) {
      cs += ls[k][lane];
      cq += lq[k][lane];
    }
    if (j < n) colsum[(int64_t)b * n + j] = cs;
    cq = wave_sum(cq);
    if (lane == 0) part[(int64_t)b * nblk + blockIdx.x] = cq;
  }
}

// |A[b]|_F^2 = the column blocks' sums of squares added in block order
__global__ void k_fro_finalize(const float* part, int nblk, int batch, float* fro2, const int* mask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || skip(mask, b)) return;
  float t = 0.f;
  for (int k = 0; k < nblk; ++k) t += part[(int64_t)b * nblk + k];
  fro2[b] = t;
}

__global__ void k_ns_scale(const float* colsum, const float* rowmax, int batch, int n, float* scale,
                           const int* mask) {
  const int b = blockIdx.x;
  if (b >= batch || skip(mask, b)) return;
  float mx = 0.f;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    float c = colsum[(int64_t)b * n + j];
    mx = fmaxf(mx, isfinite(c) ? c : 0.f);
  }
  mx = wave_max(mx);
  __shared__ float part[16];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    float v = 0.f;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v = fmaxf(v, part[w]);
    double s = sqrt((double)v * (double)rowmax[b]);
    scale[b] = s > 0.0 ? (float)s : 1.f;
  }
}

// scale[b] = |A[b]|_F from the row pass's sum of squares (Polar Express
// normalisation), 1 for a zero matrix
__global__ void k_fro_scale(const float* fro2, int batch, float* scale, const int* mask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || skip(mask, b)) return;
  const float f = sqrtf(fro2[b]);
  scale[b] = f > 0.f && isfinite(f) ? f : 1.f;
}

__global__ void k_scale_copy(const float* A, int64_t lda, int64_t sA, int m, int n, const float* scale,
                             void* X, int out_bf16, const int* mask) {
  const int b = blockIdx.y;
  if (skip(mask, b)) return;
  const float inv = 1.f / scale[b];
  const int64_t total = (int64_t)m * n;
  // rows over workgroups, columns over threads (no per-element division)
  for (int i = blockIdx.x; i < m; i += gridDim.x) {
    const float* a = A + b * sA + (int64_t)i * lda;
    const int64_t o = b * total + (int64_t)i * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const float v = a[j] * inv;
      if (out_bf16) ((bf16_t*)X)[o + j] = f2bf(v);
      else ((float*)X)[o + j] = v;
    }
  }
}

// ------------------------------------------------------------ CANS bookkeeping

struct CoefTab { float v[128]; };
__global__ void k_set_coef(float* coef, CoefTab t, int steps) {
  int i = threadIdx.x;
  if (i < 2 * steps) coef[i] = t.v[i];
}

// conv holds, per matrix, `slots` pairs (change, output) of sums of squares,
// one per output sub-tile of the update GEMM (gemm_conv_slots), added here in
// slot order so that the decision does not depend on scheduling
__global__ void k_cans_check(int batch, const float* conv, int slots, float tol, int k, int* active, int* where,
                             int* iters, const int* iter_base, int base_stride, int* flags, int* counter) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    if (!active[b]) continue;
    float d2 = 0.f, o2 = 0.f;
    const float* cb = conv + (int64_t)b * slots * 2;
    for (int q = 0; q < slots; ++q) {
      d2 += cb[2 * q];
      o2 += cb[2 * q + 1];
    }
    iters[b] = (iter_base ? iter_base[(int64_t)b * base_stride] : 0) + k + 1;
    where[b] = (k + 1) & 1;
    if (!isfinite(d2) || !isfinite(o2)) {
      active[b] = 0;
      atomicOr(flags + b, SVDP_FLAG_NONFINITE);
    } else if (d2 <= tol * tol * o2) {
      active[b] = 0;
    } else {
      ++mine;
    }
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *counter = cnt;
}

// |G - I|_F^2 per matrix: workgroup x of matrix b writes its four waves'
// partial sums to part[b][4 x + w] (kResidBlocks workgroups per matrix)
constexpr int kResidBlocks = 64;
__global__ void k_residual(const void* G, int gbf16, int n, float* part, const int* mask) {
  const int b = blockIdx.y;
  if (skip(mask, b)) return;
  const int64_t total = (int64_t)n * n;
  float s = 0.f;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int64_t o = b * total + (int64_t)i * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const float g = gbf16 ? bf2f(((const bf16_t*)G)[o + j]) : ((const float*)G)[o + j];
      const float d = g - (i == j ? 1.f : 0.f);
      s += d * d;
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[((int64_t)b * kResidBlocks + blockIdx.x) * 4 + (threadIdx.x >> 6)] = s;
}

// resid = sqrt(|G - I|_F^2 / n), the partials added in order (workgroups
// beyond n rows wrote nothing and are skipped)
__global__ void k_residual_finish(int batch, int n, const float* part, float* resid, const int* mask) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || skip(mask, b)) return;
  const int nb = min(n, kResidBlocks);
  float t = 0.f;
  for (int q = 0; q < nb * 4; ++q) t += part[(int64_t)b * kResidBlocks * 4 + q];
  resid[b] = sqrtf(t / (float)n);
}

// ------------------------------------------------------------ U column norms

// squared column norms of U: one 16-wave workgroup per 64 columns, wave w over
// rows w, w + 16, ..., the 16 partial sums added in wave order
__global__ __launch_bounds__(1024) void k_colnorm(const float* U, int64_t ldu, int64_t sU, int m, int n,
                                                  float* cn2, const int* mask) {
  const int b = blockIdx.y;
  if (skip(mask, b)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (j < n) {
    const float* p = U + b * sU + j;
#pragma unroll 4
    for (int i = w; i < m; i += 16) {
      const float v = p[(int64_t)i * ldu];
      s += v * v;
    }
  }
  __shared__ float ls[16][64];
  ls[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += ls[k][lane];
    cn2[(int64_t)b * n + j] = t;
  }
}

__global__ void k_colnorm_flag(const float* cn2, int n, float eps_qr, int* flags, const int* mask) {
  const int b = blockIdx.x;
  if (skip(mask, b)) return;
  int bad = 0, nonfin = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    float c = cn2[(int64_t)b * n + j];
    if (!isfinite(c)) nonfin = 1;
    else if (fabsf(sqrtf(c) - 1.f) > eps_qr) bad = 1;
  }
  if (__any(bad)) if ((threadIdx.x & 63) == 0) atomicOr(flags + b, SVDP_FLAG_RANK_DEFICIENT);
  if (__any(nonfin)) if ((threadIdx.x & 63) == 0) atomicOr(flags + b, SVDP_FLAG_NONFINITE);
}

// Algorithm 1's orthogonalisation of U, for the matrices flagged
// RANK_DEFICIENT: U <- Q of U = QR with R_ii >= 0, by classical Gram-Schmidt
// applied twice per column, left to right, against the finished columns
// (R_ii is the residual norm).  A column whose residual is below eps_qr (a
// zero singular value: CANS leaves that column of W V near zero) is replaced
// by the unit vector of the coordinate the finished columns cover least --
// its residual is at least sqrt(1 - i / m) > 0 -- and orthogonalised the
// same way.  One workgroup per matrix; scratch holds v (m) and the coverage
// (m) per matrix; LDS holds the n projection coefficients.
SVDP_DEV float block_sum256(float x, float* red) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(256) void k_qr_complete(float* U, int64_t ldu, int64_t sU, int m, int n, float eps_qr,
                                                     const int* flags, float* scratch, const int* mask) {
  const int b = blockIdx.x;
  if (skip(mask, b) || !(flags[b] & SVDP_FLAG_RANK_DEFICIENT)) return;
  extern __shared__ float rco[];  // n projection coefficients
  __shared__ float red[4];
  __shared__ float redv[4];
  __shared__ int redk[4];
  float* Ub = U + b * sU;
  float* v = scratch + (int64_t)b * 2 * m;
  float* cov = v + m;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  for (int k = t; k < m; k += 256) cov[k] = 0.f;
  for (int i = 0; i < n; ++i) {
    for (int k = t; k < m; k += 256) v[k] = Ub[(int64_t)k * ldu + i];
    __syncthreads();
    float nrm = 0.f;
    for (int attempt = 0; attempt < 2; ++attempt) {
      for (int pass = 0; pass < 2; ++pass) {
        // coefficients against the finished columns j < i (rows read coalesced)
        for (int j = t; j < i; j += 256) {
          float s2 = 0.f;
          for (int k = 0; k < m; ++k) s2 += Ub[(int64_t)k * ldu + j] * v[k];
          rco[j] = s2;
        }
        __syncthreads();
        // v -= sum_j rco_j U_j: one wave per row
        for (int k = w; k < m; k += 4) {
          float s2 = 0.f;
          for (int j = lane; j < i; j += 64) s2 += rco[j] * Ub[(int64_t)k * ldu + j];
          for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
          if (lane == 0) v[k] -= s2;
        }
        __syncthreads();
      }
      float s2 = 0.f;
      for (int k = t; k < m; k += 256) s2 += v[k] * v[k];
      nrm = sqrtf(block_sum256(s2, red));
      if (nrm >= eps_qr || attempt == 1) break;
      // zero column: start again from the least covered coordinate
      float best = INFINITY;
      int bk = 0;
      for (int k = t; k < m; k += 256)
        if (cov[k] < best) { best = cov[k]; bk = k; }
      for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off);
        const int ok = __shfl_xor(bk, off);
        if (ob < best || (ob == best && ok < bk)) { best = ob; bk = ok; }
      }
      if (lane == 0) { redv[w] = best; redk[w] = bk; }
      __syncthreads();
      int kstar = redk[0];
      float vbest = redv[0];
      for (int q = 1; q < 4; ++q)
        if (redv[q] < vbest || (redv[q] == vbest && redk[q] < kstar)) { vbest = redv[q]; kstar = redk[q]; }
      for (int k = t; k < m; k += 256) v[k] = k == kstar ? 1.f : 0.f;
      __syncthreads();
    }
    const float inv = nrm > 0.f ? 1.f / nrm : 0.f;
    for (int k = t; k < m; k += 256) {
      const float qv = v[k] * inv;
      Ub[(int64_t)k * ldu + i] = qv;
      cov[k] += qv * qv;
    }
    __syncthreads();
  }
}

// Blocked QR of flagged matrices.  With g a deterministic pseudo-random
// vector of unit-variance entries (a hash of matrix, row and column): a
// column whose singular value is <= eps_qr sigma_1 carries no direction
// (the polar iteration leaves it at zero or at rounding noise) and is
// replaced by g / sqrt(m); any other column whose norm is off from 1 by
// more than eps_qr gains gamma g with gamma = eps_qr / sqrt(m), keeping its
// direction to O(eps_qr).  Every column then keeps a component outside the
// span of the others, so the Gram-Schmidt passes need no completion step.
SVDP_DEV float hash_unit(uint32_t a, uint32_t b, uint32_t c) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u ^ (c + 0x2545F491u) * 0xC2B2AE3Du;
  h ^= h >> 16; h *= 0x7FEB352Du; h ^= h >> 15; h *= 0x846CA68Bu; h ^= h >> 16;
  return ((float)(h >> 8) * (1.f / 16777216.f) - 0.5f) * 3.4641016f;  // uniform, variance 1
}

__global__ void k_qr_perturb(float* U, int64_t ldu, int64_t sU, int m, int n, int rows_per, const float* S,
                             int64_t sS, const float* colnorm2, float eps_qr, const int* qmask) {
  const int b = blockIdx.z;
  if (!qmask[b]) return;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const bool nodir = !(S[b * sS + j] > eps_qr * S[b * sS]);
  if (!nodir && fabsf(sqrtf(colnorm2[(int64_t)b * n + j]) - 1.f) <= eps_qr) return;
  const float gamma = (nodir ? 1.f : eps_qr) * rsqrtf((float)m);
  float* Ub = U + b * sU;
  const int r0 = blockIdx.y * rows_per, r1 = min(m, r0 + rows_per);
  for (int k = r0; k < r1; ++k) {
    const float g = gamma * hash_unit((uint32_t)b, (uint32_t)k, (uint32_t)j);
    float* u = Ub + (int64_t)k * ldu + j;
    *u = nodir ? g : *u + g;
  }
}

// qmask[b] = 1 for the matrices (of mask) flagged RANK_DEFICIENT; *counter
// gains their number
__global__ void k_qr_mask(int batch, const int* flags, const int* mask, int* qmask, int* counter) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int q = !skip(mask, b) && (flags[b] & SVDP_FLAG_RANK_DEFICIENT);
  qmask[b] = q;
  if (q) atomicAdd(counter, 1);
}

// CholeskyQR step of one block of bc <= 64 columns Z (flagged matrices):
// G = Z^T Z (bc x bc, row-major with leading dimension bc, matrices 64 * 64
// floats apart) -> Rinv (same layout) with
// Z Rinv orthonormal.  With D = diag(G)^(1/2) and G' = D^-1 G D^-1 = R'^T R'
// (Cholesky, upper R', FP64 in LDS), Z = Q R' D, so Rinv = D^-1 R'^-1, upper
// triangular with a positive diagonal (R_ii > 0).  Column scales are kept
// >= 1e-15 of the largest and pivots (of the unit-diagonal G') >= 1e-12, so
// a (numerically) dependent block gives large but finite factors.  With
// zero_dep, a column whose pivot is <= 1e-13 (its angle to the block's
// earlier columns below 3e-7: dependent to FP32 resolution) is dropped
// instead: its row of R' is taken as e_k (no trailing update) and its column
// of Rinv as zero, so Z Rinv has a zero column there and the other columns
// stay orthonormal and independent of it.
// Layout: the Cholesky's trailing updates give thread t the 4 x 4 block of
// rows 4 (t / 16).. and columns 4 (t % 16).., one barrier per step: every
// thread takes step k's pivot itself, and the rows are scaled only after the
// last step (the update uses A[k][i] A[k][j] / r_k^2), so row k is never
// written while step k reads it.  The inverse runs up the rows, four
// adjacent lanes per column of R'^-1 summing interleaved terms.
__global__ __launch_bounds__(256) void k_qr_chol(const float* G, float* Rinv, int bc, const int* qmask,
                                                 int zero_dep) {
  const int b = blockIdx.x;
  if (!qmask[b]) return;
  __shared__ double A[64][65];  // G', then R' (upper, scaled at the end)
  __shared__ double X[64][65];  // R'^-1
  __shared__ double d[64], rd[64];
  __shared__ int dep[64];
  __shared__ double gmax;
  const int t = threadIdx.x;
  // per-matrix stride 64 x 64 whatever bc (the layout of the block GEMMs)
  const float* Gb = G + (int64_t)b * 64 * 64;
  if (t == 0) {
    double mx = 0.0;
    for (int j = 0; j < bc; ++j) mx = fmax(mx, (double)Gb[(int64_t)j * bc + j]);
    gmax = mx > 0.0 ? mx : 1.0;
  }
  __syncthreads();
  for (int j = t; j < bc; j += 256) d[j] = sqrt(fmax((double)Gb[(int64_t)j * bc + j], 1e-30 * gmax));
  __syncthreads();
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    A[i][j] = (i < bc && j < bc) ? (double)Gb[i * bc + j] / (d[i] * d[j]) : 0.0;
  }
  __syncthreads();
  const int i0 = (t >> 4) * 4, j0 = (t & 15) * 4;
  for (int k = 0; k < bc; ++k) {
    const double piv = A[k][k];
    const bool dk = zero_dep && !(piv > 1e-13);
    const double r = dk ? 1.0 : (piv > 1e-12 ? sqrt(piv) : 1e-6);
    if (t == 0) {
      dep[k] = dk;
      rd[k] = r;
    }
    if (!dk && j0 + 3 > k && i0 <= j0 + 3) {
      const double inv = 1.0 / (r * r);
      double ai[4], aj[4];
      for (int q = 0; q < 4; ++q) {
        ai[q] = A[k][i0 + q];
        aj[q] = A[k][j0 + q] * inv;
      }
      for (int p = 0; p < 4; ++p) {
        const int i = i0 + p;
        if (i <= k || i >= bc) continue;
        for (int q = 0; q < 4; ++q) {
          const int j = j0 + q;
          if (j >= i && j < bc) A[i][j] -= ai[p] * aj[q];
        }
      }
    }
    __syncthreads();
  }
  // R' row k = A[k][k..] / r_k (a dropped column: e_k)
  for (int idx = t; idx < 64 * 64; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    if (i < bc && j < bc && j >= i) A[i][j] = j == i ? rd[i] : (dep[i] ? 0.0 : A[i][j] / rd[i]);
  }
  __syncthreads();
  // X = R'^-1: row i from the rows below it
  const int jc = t >> 2, part = t & 3;
  for (int i = bc - 1; i >= 0; --i) {
    double acc = 0.0;
    if (jc < bc && jc > i)
      for (int k = i + 1 + part; k <= jc; k += 4) acc += A[i][k] * X[k][jc];
    acc += __shfl_xor(acc, 1);
    acc += __shfl_xor(acc, 2);
    if (part == 0 && jc < bc) X[i][jc] = jc < i ? 0.0 : ((jc == i ? 1.0 : 0.0) - acc) / A[i][i];
    __syncthreads();
  }
  float* Rb = Rinv + (int64_t)b * 64 * 64;
  for (int idx = t; idx < bc * bc; idx += 256) {
    const int i = idx / bc, j = idx - i * bc;
    Rb[idx] = (j >= i && !dep[j]) ? (float)(X[i][j] / d[i]) : 0.f;
  }
}

// ------------------------------------------------------------ backward

__global__ void k_dvec(const float* S, int64_t sS, int n, double eR, float* D) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = S[b * sS + j];
  double den = s * s + eR;
  D[(int64_t)b * n + j] = den == 0.0 ? 0.f : (float)(s / den);
}

SVDP_DEV double reg_ratio(double x, double e) {
  double d = x * x + e;
  return d == 0.0 ? 0.0 : x / d;
}

// 32 x 32 output tile per workgroup (256 threads, 4 entries each); the tile
// at (I, J) and its transpose partner (J, I) of both inputs go through LDS so
// all global reads are row-contiguous.
// mode 0: SVD (Algorithm 4 in the eigenbasis); mode 1: polar (Algorithm 2);
// mode 2: symmetric EVD (the EVD pseudo-gradient theorem, regularised K),
// S = sigma (the eigenvalues), dS = their incoming gradient.
__global__ void k_sylvester(int mode, const float* X1, const float* X2, const float* S, int64_t sS,
                            const float* dS, int64_t sdS, const float* D, int n, double eK,
                            double eT, float* out) {
  __shared__ float a_ij[32][33], a_ji[32][33], p_ij[32][33], p_ji[32][33];
  const int b = blockIdx.z;
  const int I0 = blockIdx.y * 32, J0 = blockIdx.x * 32;
  const int64_t base = (int64_t)b * n * n;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    int i = I0 + r, j = J0 + tx;     // (i, j) row-contiguous in j
    int i2 = J0 + r, j2 = I0 + tx;   // transposed partner tile
    bool in1 = i < n && j < n, in2 = i2 < n && j2 < n;
    a_ij[r][tx] = (X1 && in1) ? X1[base + (int64_t)i * n + j] : 0.f;
    p_ij[r][tx] = (X2 && in1) ? X2[base + (int64_t)i * n + j] : 0.f;
    a_ji[r][tx] = (X1 && in2) ? X1[base + (int64_t)i2 * n + j2] : 0.f;
    p_ji[r][tx] = (X2 && in2) ? X2[base + (int64_t)i2 * n + j2] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = I0 + r, j = J0 + tx;
    if (i >= n || j >= n) continue;
    const double si = S[b * sS + i], sj = S[b * sS + j];
    const double Di = D ? D[(int64_t)b * n + i] : 0.0, Dj = D ? D[(int64_t)b * n + j] : 0.0;  // null in mode 2
    // element (i, j) of input X is *_ij[r][tx]; element (j, i) is *_ji[tx][r]
    const double x1ij = a_ij[r][tx], x1ji = a_ji[tx][r];
    const double x2ij = p_ij[r][tx], x2ji = p_ji[tx][r];
    double c;
    if (mode == 0) {
      // X1 = U^T dU (Ahat), X2 = V^T dV (P)
      double bs = 0.5 * (x2ij + x1ij - x2ji - x1ji);          // skew(P + Ahat)_ij
      double kji = reg_ratio(sj - si, eK);                     // (K^T)_ij
      c = kji * bs - 0.5 * Di * Dj * (si * x1ij + sj * x1ji);  // sym(.. - diag(D s) Ahat diag(D))
      if (i == j && dS) c += dS[b * sdS + i];
      double t = reg_ratio(si + sj, eT);
      out[base + (int64_t)i * n + j] = (float)(si * t * c);
    } else if (mode == 1) {
      // X1 = V^T dH V, X2 = (M V)^T (dW V)
      c = 0.5 * (x1ij + x1ji) - 0.5 * Di * Dj * (x2ij + x2ji);
      double t = reg_ratio(si + sj, eT);
      out[base + (int64_t)i * n + j] = (float)(t * c);
    } else {
      // EVD: X2 = V^T dV; S = K^T o (P - P^T) / 2 + diag(dlam)
      c = 0.5 * reg_ratio(sj - si, eK) * (x2ij - x2ji);
      if (i == j && dS) c += dS[b * sdS + i];
      out[base + (int64_t)i * n + j] = (float)c;
    }
  }
}

__global__ void k_symmetrize(const float* in, int n, float* out, int64_t ldo, int64_t so) {
  const int b = blockIdx.y;
  const int64_t total = (int64_t)n * n;
  for (int i = blockIdx.x; i < n; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x)
      out[b * so + (int64_t)i * ldo + j] =
          0.5f * (in[b * total + (int64_t)i * n + j] + in[b * total + (int64_t)j * n + i]);
}

__global__ void k_copy(const float* src, int64_t lds, int64_t ss, const int* sel, const float* src_alt,
                       float* dst, int64_t ldd, int64_t sd, int m, int n, const int* mask) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const float* s = (sel && sel[b]) ? src_alt : src;
  for (int i = blockIdx.x; i < m; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x)
      dst[b * sd + (int64_t)i * ldd + j] = s[b * ss + (int64_t)i * lds + j];
}

// ------------------------------------------------------------ polar factor correction

// First-order correction of a polar factor W = W_t (I + S) (S skew, small:
// the rounding of a BF16 iterate) from P = V^T (W^T A) V, with (lam, V) the
// eigenpairs of sym(W^T A) (lam_i = sgn_i s_i).  P is the eigensolver's last
// T = V_w^T (W^T A) V_w (working column order) in sorted order:
// P_ij = T[perm_i, perm_j].  In that basis S~ = V^T S V solves
// S~ L + L S~ = -(P - P^T), so S~_ij = -2 skew(P)_ij t_ij with
// t_ij = 1 / (lam_i + lam_j), regularised as s / (s^2 + (2^-10 lam_max)^2),
// s = lam_i + lam_j: the FP32 rounding of W^T A and P (about 1e-7 lam_max)
// over a smaller s would swamp the signal, and a noisy S~ changes column
// norms at second order.  U = W V carries U_t (I + S~/2) and V carries
// V_t (I - S~/2), hence Mu = I - S~/2 and Mv = I + S~/2 = 2 I - Mu (only Mu
// is written).  The singular value of the corrected pair is
// diag((I + S~/2) P (I + S~/2)) = P_ii + 2 sum_j skew(P)_ij^2 t_ij
// - 1/4 sum_j S~_ij^2 lam_j + O(S^3) (P ~ L in the last term).  The
// symmetric off-diagonal part e = sym(P)_ij that the eigensolver's stop
// test left adds, pair by pair, the exact 2 x 2 eigenvalue shift
// sign(d) e^2 / (sqrt(d^2/4 + e^2) + |d|/2), d = P_ii - P_jj (e^2 / d for a
// wide gap, at most |e| for a close pair).  The result goes to snew as a
// magnitude.
// Three passes, all row-contiguous: k_polar_gather stages row perm_i of T
// in LDS and writes row i of P (and its diagonal entry), k_transpose32
// forms P^T, and k_polar_fix reads rows i of P and P^T.

// P[i, :] = T[perm_i, perm[:]] and dP[i] = P_ii; one workgroup per row, the
// row of T (n floats) in dynamic LDS
__global__ void k_polar_gather(const float* T, int ldt, int64_t sT, const int* perm, int n, float* P, float* dP,
                               const int* mask) {
  extern __shared__ float trow[];
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const float* Tb = T + b * sT;
  const int* pb = perm + (int64_t)b * n;
  float* Pb = P + (int64_t)b * n * n;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const float* tr = Tb + (int64_t)pb[i] * ldt;
    for (int j = threadIdx.x; j < n; j += blockDim.x) trow[j] = tr[j];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) Pb[(int64_t)i * n + j] = trow[pb[j]];
    if (threadIdx.x == 0) dP[(int64_t)b * n + i] = trow[pb[i]];
    __syncthreads();
  }
}

// Xt = X^T per matrix (X m x n BF16 contiguous, Xt n x m), 32 x 32 tiles
// through LDS; matrices outside mask are skipped
__global__ void k_transpose_bf16(const bf16_t* X, int m, int n, bf16_t* Xt, const int* mask) {
  __shared__ bf16_t tile[32][34];
  const int b = blockIdx.z;
  if (mask && !mask[b]) return;
  const int64_t off = (int64_t)b * m * n;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int i = i0 + r, j = j0 + threadIdx.x;
    if (i < m && j < n) tile[r][threadIdx.x] = X[off + (int64_t)i * n + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int j = j0 + r, i = i0 + threadIdx.x;  // Xt[j][i] = X[i][j]
    if (i < m && j < n) Xt[off + (int64_t)j * m + i] = tile[threadIdx.x][r];
  }
}

// Pt = P^T per matrix (n x n contiguous), 32 x 32 tiles through LDS
__global__ void k_transpose32(const float* P, int n, float* Pt, const int* mask) {
  __shared__ float tile[32][33];
  const int b = blockIdx.z;
  if (mask && !mask[b]) return;
  const int64_t off = (int64_t)b * n * n;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int i = i0 + r, j = j0 + threadIdx.x;
    if (i < n && j < n) tile[r][threadIdx.x] = P[off + (int64_t)i * n + j];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += blockDim.y) {
    const int i = j0 + r, j = i0 + threadIdx.x;  // Pt[i][j] = P[j][i]
    if (i < n && j < n) Pt[off + (int64_t)i * n + j] = tile[threadIdx.x][r];
  }
}

// Mu and snew from P, Pt = P^T and dP = diag(P); one workgroup per row, FP32
// arithmetic on values scaled by 1 / lam_max (so that e^2 and the
// regularisation stay far from the FP32 range limits at any scale of A).
// Every term is formed from differences and products of FP32 inputs whose
// rounding (about 2^-24 lam_max) is already below what the correction
// resolves; the row sums only add second-order terms to P_ii.  Mu may be P
// itself: each element is read before the same thread overwrites it, and no
// other row reads it.  S holds magnitudes with their signs in sgn (lam =
// sgn S, snew a magnitude), or with signed_lam the signed eigenvalues
// themselves (lam = S, snew signed).  An exactly tied pair (d = 0) takes the
// 2 x 2 eigenvalues a + |e| and a - |e| in index order, the smaller index
// the larger value, as the descending sort would.
__global__ void k_polar_fix(const float* P, const float* Pt, const float* dP, const float* S, int64_t sS,
                            const float* sgn, int signed_lam, int n, float* Mu, float* snew, const int* mask) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const int64_t off = (int64_t)b * n * n;
  const float* sb = S + b * sS;
  const float* gb = sgn + (int64_t)b * n;
  const float* db = dP + (int64_t)b * n;
  const float lmax = signed_lam ? fmaxf(fabsf(sb[0]), fabsf(sb[n - 1])) : fabsf(sb[0]);
  // all-zero spectrum: nothing to correct (t = 0, e = 0)
  const float inv = lmax > 0.f ? 1.f / lmax : 0.f;
  auto lam = [&](int i) -> float { return (signed_lam ? sb[i] : gb[i] * sb[i]) * inv; };
  const float reg = 0x1p-20f;  // (2^-10 lam_max)^2 in units of lam_max
  __shared__ float red[2][4];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const float li = lam(i);
    const float pii = db[i] * inv;
    float a1 = 0.f, a2 = 0.f;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const float lj = lam(j);
      const float s = li + lj;
      const float t = s / (s * s + reg);
      const float pij = P[off + (int64_t)i * n + j] * inv, pji = Pt[off + (int64_t)i * n + j] * inv;
      const float sk = 0.5f * (pij - pji);
      const float st = -2.f * sk * t;
      a1 += 2.f * sk * sk * t;
      a2 += st * st * lj;
      if (j != i) {
        const float e = 0.5f * (pij + pji);
        const float dd = pii - db[j] * inv;
        const float hh = sqrtf(0.25f * dd * dd + e * e) + 0.5f * fabsf(dd);
        const float sgn_d = dd > 0.f ? 1.f : (dd < 0.f ? -1.f : (i < j ? 1.f : -1.f));
        if (hh > 0.f) a1 += sgn_d * e * e / hh;
      }
      Mu[off + (int64_t)i * n + j] = (i == j ? 1.f : 0.f) - 0.5f * st;
    }
    for (int o = 32; o > 0; o >>= 1) {
      a1 += __shfl_xor(a1, o);
      a2 += __shfl_xor(a2, o);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = a1;
      red[1][threadIdx.x >> 6] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float s1 = 0.f, s2 = 0.f;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { s1 += red[0][w]; s2 += red[1][w]; }
      const float v = (pii + (s1 - 0.25f * s2)) * lmax;
      snew[(int64_t)b * n + i] = signed_lam ? v : fabsf(v);
    }
    __syncthreads();
  }
}

// V <- 2 V - Vu (V Mv from V Mu, Mv = 2 I - Mu); Vu contiguous n x n
__global__ void k_vcorr(float* V, int64_t ldv, int64_t sV, const float* Vu, int n) {
  const int b = blockIdx.y;
  for (int i = blockIdx.x; i < n; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      float* v = V + b * sV + (int64_t)i * ldv + j;
      *v = 2.f * *v - Vu[((int64_t)b * n + i) * n + j];
    }
}

// S[b] = snew[b] made non-increasing (a corrected value may cross its
// neighbour by its correction only, where the two are already equal to that
// accuracy); one thread per matrix
__global__ void k_sigma_store(const float* snew, int n, float* S, int64_t sS, int batch, const int* mask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || (mask && !mask[b])) return;
  float prev = snew[(int64_t)b * n];
  S[b * sS] = prev;
  for (int i = 1; i < n; ++i) {
    prev = fminf(prev, snew[(int64_t)b * n + i]);
    S[b * sS + i] = prev;
  }
}

// ------------------------------------------------------------ features

// 1 / |A[b]|_F when fro2 is given (the power sequence runs on A / |A|_F, so
// its norms stay below |x| whatever the scale of A), else 1
SVDP_DEV float matvec_scale(const float* fro2, int b) {
  return (fro2 && fro2[b] > 0.f) ? 1.f / sqrtf(fro2[b]) : 1.f;
}
// y = A x: one wave per row
__global__ void k_matvec_n(const float* A, int64_t lda, int64_t sA, int m, int n, const float* x,
                           int64_t sx, float* y, int64_t sy, const float* fro2) {
  const int b = blockIdx.y;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + w;
  if (i >= m) return;
  const float* r = A + b * sA + (int64_t)i * lda;
  const float* xb = x + b * sx;
  float s = 0.f;
  for (int j = lane; j < n; j += 64) s += r[j] * xb[j];
  s = wave_sum(s);
  if (lane == 0) y[b * sy + i] = s * matvec_scale(fro2, b);
}
// y = A^T x: one workgroup of 16 waves per 64 columns, wave w over rows w,
// w + 16, ...; the 16 partial sums are added in wave order (deterministic)
__global__ __launch_bounds__(1024) void k_matvec_t(const float* A, int64_t lda, int64_t sA, int m, int n,
                                                   const float* x, int64_t sx, float* y, int64_t sy,
                                                   const float* fro2) {
  const int b = blockIdx.y;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = blockIdx.x * 64 + lane;
  float s = 0.f;
  if (j < n) {
    const float* p = A + b * sA + j;
    const float* xb = x + b * sx;
#pragma unroll 4
    for (int i = w; i < m; i += 16) s += p[(int64_t)i * lda] * xb[i];
  }
  __shared__ float ls[16][64];
  ls[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += ls[k][lane];
    y[b * sy + j] = t * matvec_scale(fro2, b);
  }
}

// sum of squares in FP64: no overflow before the square root
__global__ void k_vnorm(const float* v, int64_t sv, int len, float* nrm, int slot) {
  const int b = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < len; j += blockDim.x) {
    const double x = v[b * sv + j];
    s += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  __shared__ double part[16];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
    nrm[b * 8 + slot] = (float)sqrt(t);
  }
}

SVDP_DEV void features_from(double F, const double* nr, double n, double m_over_n, float* f,
                            float* aux) {
  double r[7];
  for (int k = 0; k < 7; ++k) r[k] = nr[k + 1] / nr[k];
  f[0] = (float)log(F / r[6]);
  for (int k = 1; k < 6; ++k) f[k] = (float)log(r[k] / r[k + 1]);
  f[6] = (float)log(n);
  f[7] = (float)log(m_over_n);
  aux[0] = (float)r[6];
  aux[1] = (float)F;
}

__global__ void k_features(const float* fro2, const float* nrm, int batch, int m, int n, float* F,
                           float* aux) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  // nrm holds the norms of the sequence on A / |A|_F: its ratios are those of
  // A divided by |A|_F, so the features see |A|_F = 1 and the sigma_max
  // estimate aux[0] is scaled back
  double nr[8];
  for (int k = 0; k < 8; ++k) nr[k] = nrm[b * 8 + k];
  const double fro = sqrt((double)fro2[b]);
  features_from(1.0, nr, (double)n, (double)m / (double)n, F + b * 8, aux + b * 2);
  aux[b * 2] = (float)((double)aux[b * 2] * fro);
  aux[b * 2 + 1] = (float)fro;
}

// one wave per row: |s^k z| for k = 0..7 and |s|
__global__ void k_spectral_features(const float* s, const float* z, int rows, int n,
                                    const float* m_over_n, float* F, float* aux) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  if (row >= rows) return;
  const float* sr = s + (int64_t)row * n;
  const float* zr = z + (int64_t)row * n;
  double acc[9];
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int j = lane; j < n; j += 64) {
    double sv = sr[j], p = zr[j];
    acc[8] += sv * sv;
    for (int k = 0; k < 8; ++k) {
      acc[k] += p * p;
      p *= sv;
    }
  }
  for (int k = 0; k < 9; ++k)
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off);
  if (lane == 0) {
    double nr[8];
    for (int k = 0; k < 8; ++k) nr[k] = sqrt(acc[k]);
    features_from(sqrt(acc[8]), nr, (double)n, (double)m_over_n[row], F + (int64_t)row * 8, aux + (int64_t)row * 2);
  }
}

// Training targets of the interval predictor, one wave per row: with
// smax, smin the largest and smallest entry of the row's spectrum s and
// r7 = aux[row][0] its power-sequence estimate, T = (log(smax / r7),
// log(smax / smin)) (smin clamped at 1e-30).
__global__ void k_training_targets(const float* s, const float* aux, int rows, int n, float* T) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + w;
  if (row >= rows) return;
  const float* sr = s + (int64_t)row * n;
  float mx = 0.f, mn = INFINITY;
  for (int j = lane; j < n; j += 64) {
    mx = fmaxf(mx, sr[j]);
    mn = fminf(mn, sr[j]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off));
    mn = fminf(mn, __shfl_xor(mn, off));
  }
  if (lane == 0) {
    const double smax = mx, smin = fmax((double)mn, 1e-30), r7 = aux[2 * (int64_t)row];
    T[2 * (int64_t)row] = (float)log(smax / r7);
    T[2 * (int64_t)row + 1] = (float)log(smax / smin);
  }
}

// Feature standardisation of a training set, one workgroup: mu = mean of
// each of the 8 columns of F (rows x 8), sd = its sample standard deviation
// (divisor rows - 1), clamped at 1e-3; FP64 sums in a fixed order (each
// thread a fixed set of rows, then a tree in LDS), so the result does not
// depend on scheduling.
__global__ __launch_bounds__(256) void k_feature_stats(const float* F, int rows, float* mu, float* sd) {
  __shared__ double red[2][8][256];
  const int t = threadIdx.x;
  double a[8], q[8];
  for (int f = 0; f < 8; ++f) a[f] = q[f] = 0.0;
  for (int r = t; r < rows; r += 256)
    for (int f = 0; f < 8; ++f) {
      const double v = F[(int64_t)r * 8 + f];
      a[f] += v;
    }
  for (int f = 0; f < 8; ++f) red[0][f][t] = a[f];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st)
      for (int f = 0; f < 8; ++f) red[0][f][t] += red[0][f][t + st];
    __syncthreads();
  }
  double mean[8];
  for (int f = 0; f < 8; ++f) mean[f] = red[0][f][0] / fmax((double)rows, 1.0);
  // second pass on the centred values
  for (int r = t; r < rows; r += 256)
    for (int f = 0; f < 8; ++f) {
      const double v = F[(int64_t)r * 8 + f] - mean[f];
      q[f] += v * v;
    }
  for (int f = 0; f < 8; ++f) red[1][f][t] = q[f];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (t < st)
      for (int f = 0; f < 8; ++f) red[1][f][t] += red[1][f][t + st];
    __syncthreads();
  }
  if (t < 8) {
    mu[t] = (float)mean[t];
    sd[t] = (float)fmax(sqrt(red[1][t][0] / fmax((double)rows - 1.0, 1.0)), 1e-3);
  }
}

// ------------------------------------------------------------ MLP

constexpr int NF = 8, HID = 64, NO = 2;
constexpr int OW1 = 0, OB1 = OW1 + HID * NF, OW2 = OB1 + HID, OB2 = OW2 + HID * HID,
              OW3 = OB2 + HID, OB3 = OW3 + NO * HID, NPAR = OB3 + NO;
static_assert(NPAR == SVDP_MLP_PARAMS, "parameter count");

SVDP_DEV void load_params(float* sp, const float* P) {
  for (int i = threadIdx.x; i < NPAR; i += blockDim.x) sp[i] = P[i];
}
SVDP_DEV void std_input(const float* X, int row, const float* mu, const float* sd, float* x) {
  for (int f = 0; f < NF; ++f) {
    float v = X[(int64_t)row * NF + f];
    x[f] = (mu && sd) ? (v - mu[f]) / sd[f] : v;
  }
}

// one thread per row, parameters staged in LDS
__global__ __launch_bounds__(256) void k_mlp_fwd(const float* P, const float* mu, const float* sd,
                                                 const float* X, int rows, float* out, float* act) {
  __shared__ float sp[NPAR];
  load_params(sp, P);
  __syncthreads();
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  float x[NF], h1[HID];
  std_input(X, row, mu, sd, x);
  for (int o = 0; o < HID; ++o) {
    float a = sp[OB1 + o];
    for (int f = 0; f < NF; ++f) a += sp[OW1 + o * NF + f] * x[f];
    h1[o] = tanhf(a);
    if (act) act[(int64_t)row * 2 * HID + o] = h1[o];
  }
  float o0 = sp[OB3], o1 = sp[OB3 + 1];
  for (int o = 0; o < HID; ++o) {
    float a = sp[OB2 + o];
    for (int i = 0; i < HID; ++i) a += sp[OW2 + o * HID + i] * h1[i];
    float h2 = tanhf(a);
    if (act) act[(int64_t)row * 2 * HID + HID + o] = h2;
    o0 += sp[OW3 + o] * h2;
    o1 += sp[OW3 + HID + o] * h2;
  }
  out[(int64_t)row * NO] = o0;
  out[(int64_t)row * NO + 1] = o1;
}

// Backward over a chunk of 64 rows per workgroup: per-row deltas by one
// thread each, then the weight gradients of the chunk as small outer-product
// sums; partial[chunk] holds them, a second kernel adds the chunks in order.
constexpr int RCH = 32;
__global__ __launch_bounds__(256) void k_mlp_bwd(const float* P, const float* mu, const float* sd,
                                                 const float* X, const float* act, const float* dout,
                                                 int rows, float* partial) {
  __shared__ float sW2[HID * HID];
  __shared__ float sW3[NO * HID];
  __shared__ float xs[RCH][NF + 1];
  __shared__ float h1s[RCH][HID + 1];
  __shared__ float h2s[RCH][HID + 1];
  __shared__ float d1s[RCH][HID + 1];
  __shared__ float d2s[RCH][HID + 1];
  __shared__ float dos[RCH][NO];
  for (int i = threadIdx.x; i < HID * HID; i += blockDim.x) sW2[i] = P[OW2 + i];
  for (int i = threadIdx.x; i < NO * HID; i += blockDim.x) sW3[i] = P[OW3 + i];
  const int r0 = blockIdx.x * RCH;
  for (int idx = threadIdx.x; idx < RCH * HID; idx += blockDim.x) {
    int r = idx / HID, o = idx % HID, row = r0 + r;
    bool in = row < rows;
    h1s[r][o] = in ? act[(int64_t)row * 2 * HID + o] : 0.f;
    h2s[r][o] = in ? act[(int64_t)row * 2 * HID + HID + o] : 0.f;
  }
  for (int idx = threadIdx.x; idx < RCH * NO; idx += blockDim.x) {
    int r = idx / NO, o = idx % NO, row = r0 + r;
    dos[r][o] = row < rows ? dout[(int64_t)row * NO + o] : 0.f;
  }
  if (threadIdx.x < RCH) {
    int row = r0 + threadIdx.x;
    float x[NF];
    if (row < rows) std_input(X, row, mu, sd, x);
    else for (int f = 0; f < NF; ++f) x[f] = 0.f;
    for (int f = 0; f < NF; ++f) xs[threadIdx.x][f] = x[f];
  }
  __syncthreads();
  // d2 = (W3^T dout) * (1 - h2^2): entry (r, o) per thread
  for (int idx = threadIdx.x; idx < RCH * HID; idx += blockDim.x) {
    int r = idx / HID, o = idx % HID;
    float g = sW3[o] * dos[r][0] + sW3[HID + o] * dos[r][1];
    float h = h2s[r][o];
    d2s[r][o] = g * (1.f - h * h);
  }
  __syncthreads();
  // d1 = (W2^T d2) * (1 - h1^2)
  for (int idx = threadIdx.x; idx < RCH * HID; idx += blockDim.x) {
    int r = idx / HID, i = idx % HID;
    float g = 0.f;
    for (int o = 0; o < HID; ++o) g += sW2[o * HID + i] * d2s[r][o];
    float h = h1s[r][i];
    d1s[r][i] = g * (1.f - h * h);
  }
  __syncthreads();
  float* part = partial + (int64_t)blockIdx.x * NPAR;
  // dW2[o][i] = sum_r d2[r][o] h1[r][i]
  for (int idx = threadIdx.x; idx < HID * HID; idx += blockDim.x) {
    int o = idx / HID, i = idx % HID;
    float s = 0.f;
    for (int r = 0; r < RCH; ++r) s += d2s[r][o] * h1s[r][i];
    part[OW2 + idx] = s;
  }
  for (int idx = threadIdx.x; idx < HID * NF; idx += blockDim.x) {
    int o = idx / NF, f = idx % NF;
    float s = 0.f;
    for (int r = 0; r < RCH; ++r) s += d1s[r][o] * xs[r][f];
    part[OW1 + idx] = s;
  }
  for (int idx = threadIdx.x; idx < NO * HID; idx += blockDim.x) {
    int c = idx / HID, o = idx % HID;
    float s = 0.f;
    for (int r = 0; r < RCH; ++r) s += dos[r][c] * h2s[r][o];
    part[OW3 + idx] = s;
  }
  for (int o = threadIdx.x; o < HID; o += blockDim.x) {
    float s1 = 0.f, s2 = 0.f;
    for (int r = 0; r < RCH; ++r) { s1 += d1s[r][o]; s2 += d2s[r][o]; }
    part[OB1 + o] = s1;
    part[OB2 + o] = s2;
  }
  if (threadIdx.x < NO) {
    float s = 0.f;
    for (int r = 0; r < RCH; ++r) s += dos[r][threadIdx.x];
    part[OB3 + threadIdx.x] = s;
  }
}

__global__ void k_sum_chunks(const float* partial, int chunks, float* dP) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPAR) return;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * NPAR + i];
  dP[i] = s;
}

__global__ void k_pinball(const float* out, const float* target, int rows, float tau0, float tau1,
                          float* dout, float* loss) {
  int row = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (row < rows) {
    for (int j = 0; j < 2; ++j) {
      float tau = j ? tau1 : tau0;
      float u = target[(int64_t)row * 2 + j] - out[(int64_t)row * 2 + j];
      l += fmaxf(tau * u, (tau - 1.f) * u);
      dout[(int64_t)row * 2 + j] = (u < 0.f ? 1.f - tau : -tau) / (float)rows;
    }
  }
  l = wave_sum(l);
  if ((threadIdx.x & 63) == 0 && loss) atomicAdd(loss, l / (float)rows);
}

__global__ void k_adam(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ------------------------------------------------------------ bounds

// degree-3 interval-optimal polynomial on [a, b] (equioscillation at a, x*, b)
SVDP_DEV void cans_poly_dev(double a, double b, double& al, double& be, double& lo, double& hi) {
  double s = a * a + a * b + b * b;
  double xs = sqrt(s / 3.0);
  be = -2.0 / (a * b * (a + b) + 2.0 * xs * xs * xs);
  al = -be * s;
  lo = al * a + be * a * a * a;
  hi = al * xs + be * xs * xs * xs;
}

// mode 0: learned (mlp_out = (log(smax / r7), log(smax / smin)), aux = (r7, |A|_F))
// mode 1: user bounds (sigma_min, sigma_max)
__global__ void k_bounds(int batch, int mode, const float* mlp_out, const float* aux,
                         const float* user_bounds, double margin_max, double margin_min,
                         double handoff, double bf16_from, int kcap, float* scale, float* coef,
                         int* ksteps, const int* mask) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || skip(mask, b)) return;
  double smax, smin;
  if (mode == 0) {
    double r7 = aux[2 * b];
    double o1 = fmax((double)mlp_out[2 * b], 0.0);      // r7 <= sigma_max
    double o2 = fmax((double)mlp_out[2 * b + 1], 0.0);  // kappa >= 1
    smax = r7 * exp(o1);
    smin = smax * exp(-o2);
  } else {
    smin = user_bounds[2 * b];
    smax = user_bounds[2 * b + 1];
  }
  // widen the interval: BF16 rounding of the iterate moves its singular
  // values, and a value pushed past the cubic's positive root changes sign
  smax *= margin_max;
  smin *= margin_min;
  if (!(smax > 0.0) || !isfinite(smax)) smax = 1.0;
  double lo = smin / smax;
  // the host's step budget counts the steps from this floor (kLoFloor)
  if (!(lo > 1e-9)) lo = 1e-9;
  if (lo > 1.0) lo = 1.0;
  scale[b] = (float)smax;
  double a = lo, hb = 1.0;
  int K = kcap, K1 = a >= bf16_from ? 0 : kcap;
  for (int k = 0; k < kcap; ++k) {
    double al, be, l2, h2;
    cans_poly_dev(a, hb, al, be, l2, h2);
    coef[((int64_t)b * kcap + k) * 2] = (float)al;
    coef[((int64_t)b * kcap + k) * 2 + 1] = (float)be;
    a = l2;
    hb = h2;
    if (K == kcap && fmax(1.0 - a, hb - 1.0) <= handoff) K = k + 1;
    if (K1 == kcap && a >= bf16_from) K1 = k + 1;
  }
  ksteps[2 * b] = K;
  ksteps[2 * b + 1] = K1;
}

// ------------------------------------------------------------ info

__global__ void k_info(int batch, const int* iters, const int* sweeps, const int* flags,
                       const float* resid, svdp_info* info, const int* mask) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch || skip(mask, b)) return;
  svdp_info r;
  r.iters = iters ? iters[b] : 0;
  r.sweeps = sweeps ? sweeps[b] : 0;
  r.flags = flags ? flags[b] : 0;
  r.residual = resid ? resid[b] : 0.f;
  info[b] = r;
}

__global__ void k_fallback_mask(int batch, int* flags, int bits, const float* resid, float rtol,
                                int* mask, int* counter) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) {
    int f = (flags[b] & bits) != 0 || !(resid[b] <= rtol);
    mask[b] = f;
    if (f) flags[b] = 0;  // the rerun reports its own flags
    mine += f;
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *counter = cnt;
}

__global__ void k_fill_masked(int* p, int v, int n, const int* mask) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < n && !skip(mask, b)) p[b] = v;
}

__global__ void k_or_flags(int batch, int* flags, int bits, const int* mask) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch && !skip(mask, b)) flags[b] |= bits;
}

inline int grid1(int64_t total, int cap = 2048) { return (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(total, 256), cap)); }

}  // namespace

#define LAUNCH_CHECK() return hipGetLastError()

hipError_t norms_launch(const float* A, int64_t lda, int64_t sA, int batch, int m, int n,
                        float* colsum, float* rowmax, float* fro2, float* part, int* flags, const int* mask,
                        hipStream_t st) {
  hipError_t e;
  if ((e = fill_f32(rowmax, 0.f, batch, st))) return e;
  const int rows_wg = 64;
  hipLaunchKernelGGL(k_rownorms, dim3(cdiv(m, rows_wg), batch), dim3(256), 0, st, A, lda, sA, m, n, rows_wg,
                     rowmax, flags, mask);
  if ((e = hipGetLastError())) return e;
  const int nblk = norms_blocks(n);
  hipLaunchKernelGGL(k_colnorms, dim3(nblk, batch), dim3(1024), 0, st, A, lda, sA, m, n, colsum, part, nblk,
                     mask);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_fro_finalize, dim3(cdiv(batch, 256)), dim3(256), 0, st, part, nblk, batch, fro2, mask);
  LAUNCH_CHECK();
}

hipError_t transpose_bf16_launch(const void* X, int batch, int m, int n, void* Xt, const int* mask,
                                 hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_bf16, dim3(cdiv(n, 32), cdiv(m, 32), batch), dim3(32, 8), 0, st,
                     (const bf16_t*)X, m, n, (bf16_t*)Xt, mask);
  return hipGetLastError();
}

hipError_t training_targets_launch(const float* s, const float* aux, int rows, int n, float* T, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_training_targets, dim3(cdiv(rows, 4)), dim3(256), 0, st, s, aux, rows, n, T);
  return hipGetLastError();
}

hipError_t feature_stats_launch(const float* F, int rows, float* mu, float* sd, hipStream_t st) {
  hipLaunchKernelGGL(k_feature_stats, dim3(1), dim3(256), 0, st, F, rows, mu, sd);
  return hipGetLastError();
}

hipError_t fro_scale_launch(const float* fro2, int batch, float* scale, const int* mask, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fro_scale, dim3(cdiv(batch, 256)), dim3(256), 0, st, fro2, batch, scale, mask);
  return hipGetLastError();
}

hipError_t ns_scale_launch(const float* colsum, const float* rowmax, int batch, int n, float* scale,
                           const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_ns_scale, dim3(batch), dim3(256), 0, st, colsum, rowmax, batch, n, scale, mask);
  LAUNCH_CHECK();
}

hipError_t scale_copy_launch(const float* A, int64_t lda, int64_t sA, int batch, int m, int n,
                             const float* scale, void* X, int out_bf16, const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3(std::min(m, 512), batch), dim3(256), 0, st, A, lda, sA, m,
                     n, scale, X, out_bf16, mask);
  LAUNCH_CHECK();
}

hipError_t set_coef_launch(float* coef, const double* tab, int steps, hipStream_t st) {
  CoefTab t;
  if (steps > 64) steps = 64;
  for (int i = 0; i < 2 * steps; ++i) t.v[i] = (float)tab[i];
  hipLaunchKernelGGL(k_set_coef, dim3(1), dim3(128), 0, st, coef, t, steps);
  LAUNCH_CHECK();
}

hipError_t cans_check_launch(int batch, const float* conv, int slots, float tol, int k, int* active, int* where,
                             int* iters, const int* iter_base, int base_stride, int* flags,
                             int* counter, hipStream_t st) {
  hipLaunchKernelGGL(k_cans_check, dim3(1), dim3(1024), 0, st, batch, conv, slots, tol, k, active, where,
                     iters, iter_base, base_stride, flags, counter);
  LAUNCH_CHECK();
}

size_t residual_part_floats(int64_t batch) { return (size_t)batch * kResidBlocks * 4; }

hipError_t residual_launch(const void* G, int gbf16, int batch, int n, float* part, float* resid,
                           const int* mask, hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_residual, dim3(std::min(n, kResidBlocks), batch), dim3(256), 0, st, G, gbf16, n,
                     part, mask);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_residual_finish, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch, n, part, resid,
                     mask);
  LAUNCH_CHECK();
}

hipError_t colnorm_check_launch(const float* U, int64_t ldu, int64_t sU, int batch, int m, int n,
                                float* colnorm2, float eps_qr, int* flags, const int* mask,
                                hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_colnorm, dim3(cdiv(n, 64), batch), dim3(1024), 0, st, U, ldu, sU, m, n, colnorm2, mask);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_colnorm_flag, dim3(batch), dim3(256), 0, st, colnorm2, n, eps_qr, flags, mask);
  LAUNCH_CHECK();
}

hipError_t qr_complete_launch(float* U, int64_t ldu, int64_t sU, int batch, int m, int n, float eps_qr,
                              const int* flags, float* scratch, const int* mask, hipStream_t st) {
  if (batch <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qr_complete, dim3(batch), dim3(256), (size_t)n * sizeof(float), st, U, ldu, sU, m, n, eps_qr,
                     flags, scratch, mask);
  LAUNCH_CHECK();
}

hipError_t qr_chol_launch(const float* G, float* Rinv, int batch, int bc, const int* qmask, int zero_dep,
                          hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  if (bc < 1 || bc > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_qr_chol, dim3(batch), dim3(256), 0, st, G, Rinv, bc, qmask, zero_dep);
  LAUNCH_CHECK();
}

hipError_t qr_perturb_launch(float* U, int64_t ldu, int64_t sU, int batch, int m, int n, const float* S,
                             int64_t sS, const float* colnorm2, float eps_qr, const int* qmask, hipStream_t st) {
  if (batch <= 0 || n <= 0) return hipSuccess;
  const int rows_per = 256;
  hipLaunchKernelGGL(k_qr_perturb, dim3(cdiv(n, 256), cdiv(m, rows_per), batch), dim3(256), 0, st, U, ldu, sU, m,
                     n, rows_per, S, sS, colnorm2, eps_qr, qmask);
  LAUNCH_CHECK();
}

hipError_t qr_mask_launch(int batch, const int* flags, const int* mask, int* qmask, int* counter, hipStream_t st) {
  hipError_t e;
  if ((e = fill_i32(counter, 0, 1, st))) return e;
  hipLaunchKernelGGL(k_qr_mask, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch, flags, mask, qmask, counter);
  LAUNCH_CHECK();
}

hipError_t dvec_launch(const float* S, int64_t sS, int batch, int n, double eR, float* D, hipStream_t st) {
  hipLaunchKernelGGL(k_dvec, dim3(cdiv(n, 256), batch), dim3(256), 0, st, S, sS, n, eR, D);
  LAUNCH_CHECK();
}

hipError_t sylvester_launch(int mode, const float* X1, const float* X2, const float* S, int64_t sS,
                            const float* dS, int64_t sdS, const float* D, int batch, int n, double eK,
                            double eT, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sylvester, dim3(cdiv(n, 32), cdiv(n, 32), batch), dim3(256), 0, st, mode, X1, X2,
                     S, sS, dS, sdS, D, n, eK, eT, out);
  LAUNCH_CHECK();
}

hipError_t symmetrize_launch(const float* in, int batch, int n, float* out, int64_t ldo, int64_t so,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(std::min(n, 512), batch), dim3(256), 0, st, in, n, out, ldo,
                     so);
  LAUNCH_CHECK();
}

hipError_t polar_fix_launch(const float* T, int ldt, int64_t sT, const int* perm, const float* S, int64_t sS,
                            const float* sgn, int signed_lam, int batch, int n, float* P, float* Pt, float* dP,
                            float* snew, const int* mask, hipStream_t st) {
  hipError_t e;
  hipLaunchKernelGGL(k_polar_gather, dim3(std::min(n, 1024), batch), dim3(256), (size_t)n * sizeof(float), st, T,
                     ldt, sT, perm, n, P, dP, mask);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_transpose32, dim3(cdiv(n, 32), cdiv(n, 32), batch), dim3(32, 8), 0, st, P, n, Pt, mask);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_polar_fix, dim3(std::min(n, 1024), batch), dim3(256), 0, st, P, Pt, dP, S, sS, sgn,
                     signed_lam, n, P, snew, mask);
  LAUNCH_CHECK();
}

hipError_t vcorr_launch(float* V, int64_t ldv, int64_t sV, const float* Vu, int batch, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_vcorr, dim3(std::min(n, 512), batch), dim3(256), 0, st, V, ldv, sV, Vu, n);
  LAUNCH_CHECK();
}

hipError_t sigma_store_launch(const float* snew, int n, float* S, int64_t sS, int batch, const int* mask,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_sigma_store, dim3(cdiv(batch, 64)), dim3(64), 0, st, snew, n, S, sS, batch, mask);
  LAUNCH_CHECK();
}

hipError_t copy_launch(const float* src, int64_t lds, int64_t ss, const int* sel, const float* src_alt,
                       float* dst, int64_t ldd, int64_t sd, int batch, int m, int n, hipStream_t st,
                       const int* mask) {
  hipLaunchKernelGGL(k_copy, dim3(std::min(m, 512), batch), dim3(256), 0, st, src, lds, ss, sel,
                     src_alt, dst, ldd, sd, m, n, mask);
  LAUNCH_CHECK();
}

hipError_t matvec_launch(const float* A, int64_t lda, int64_t sA, int batch, int m, int n, const float* x,
                         int64_t sx, float* y, int64_t sy, int trans, const float* fro2, hipStream_t st) {
  if (!trans) {
    hipLaunchKernelGGL(k_matvec_n, dim3(cdiv(m, 4), batch), dim3(256), 0, st, A, lda, sA, m, n, x, sx, y,
                       sy, fro2);
    LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_matvec_t, dim3(cdiv(n, 64), batch), dim3(1024), 0, st, A, lda, sA, m, n, x, sx, y, sy,
                     fro2);
  LAUNCH_CHECK();
}

hipError_t vnorm_launch(const float* v, int64_t sv, int batch, int len, float* nrm, int slot,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_vnorm, dim3(batch), dim3(256), 0, st, v, sv, len, nrm, slot);
  LAUNCH_CHECK();
}

hipError_t features_launch(const float* fro2, const float* nrm, int batch, int m, int n, float* F,
                           float* aux, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(cdiv(batch, 64)), dim3(64), 0, st, fro2, nrm, batch, m, n, F, aux);
  LAUNCH_CHECK();
}

hipError_t spectral_features_launch(const float* s, const float* z, int rows, int n, const float* m_over_n,
                                    float* F, float* aux, hipStream_t st) {
  hipLaunchKernelGGL(k_spectral_features, dim3(cdiv(rows, 4)), dim3(256), 0, st, s, z, rows, n, m_over_n,
                     F, aux);
  LAUNCH_CHECK();
}

hipError_t mlp_fwd_launch(const float* P, const float* mu, const float* sd, const float* X, int rows,
                          float* out, float* act, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_fwd, dim3(cdiv(rows, 256)), dim3(256), 0, st, P, mu, sd, X, rows, out, act);
  LAUNCH_CHECK();
}

size_t mlp_bwd_partial_floats(int rows) { return (size_t)cdiv(rows, RCH) * NPAR; }

hipError_t mlp_bwd_launch(const float* P, const float* mu, const float* sd, const float* X,
                          const float* act, const float* dout, int rows, float* partial, float* dP,
                          hipStream_t st) {
  int chunks = cdiv(rows, RCH);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(chunks), dim3(256), 0, st, P, mu, sd, X, act, dout, rows, partial);
  hipError_t e;
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(k_sum_chunks, dim3(cdiv(NPAR, 256)), dim3(256), 0, st, partial, chunks, dP);
  LAUNCH_CHECK();
}

hipError_t pinball_launch(const float* out, const float* target, int rows, float tau0, float tau1,
                          float* dout, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_pinball, dim3(cdiv(rows, 256)), dim3(256), 0, st, out, target, rows, tau0, tau1,
                     dout, loss);
  LAUNCH_CHECK();
}

hipError_t adam_launch(float* p, float* m, float* v, const float* g, int64_t n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t st) {
  float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(cdiv(n, 256)), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2, eps, c1, c2);
  LAUNCH_CHECK();
}

hipError_t bounds_launch(int batch, int mode, const float* mlp_out, const float* aux,
                         const float* user_bounds, double margin_max, double margin_min, double handoff,
                         double bf16_from, int kcap, float* scale, float* coef, int* ksteps,
                         const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_bounds, dim3(cdiv(batch, 64)), dim3(64), 0, st, batch, mode, mlp_out, aux,
                     user_bounds, margin_max, margin_min, handoff, bf16_from, kcap, scale, coef, ksteps,
                     mask);
  LAUNCH_CHECK();
}

hipError_t info_pack_launch(int batch, const int* iters, const int* sweeps, const int* flags,
                            const float* resid, svdp_info* info, const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_info, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch, iters, sweeps, flags, resid,
                     info, mask);
  LAUNCH_CHECK();
}

hipError_t fallback_mask_launch(int batch, int* flags, int bits, const float* resid, float rtol,
                                int* mask, int* counter, hipStream_t st) {
  hipLaunchKernelGGL(k_fallback_mask, dim3(1), dim3(1024), 0, st, batch, flags, bits, resid, rtol, mask,
                     counter);
  LAUNCH_CHECK();
}

hipError_t or_flags_launch(int batch, int* flags, int bits, const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_or_flags, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch, flags, bits, mask);
  LAUNCH_CHECK();
}

hipError_t fill_masked_launch(int* p, int v, int n, const int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_masked, dim3(cdiv(n, 256)), dim3(256), 0, st, p, v, n, mask);
  LAUNCH_CHECK();
}

namespace {
__global__ void k_count_mask(int batch, const int* mask, int* counter) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int b = threadIdx.x; b < batch; b += blockDim.x) mine += mask[b] != 0;
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *counter = cnt;
}
}  // namespace

hipError_t count_mask_launch(int batch, const int* mask, int* counter, hipStream_t st) {
  hipLaunchKernelGGL(k_count_mask, dim3(1), dim3(1024), 0, st, batch, mask, counter);
  LAUNCH_CHECK();
}

namespace {
// what = 0: the schedule starts in FP32; 1: it starts in BF16; 2: the last
// iterate is in the odd buffer (K odd)
__global__ void k_sched_mask(int batch, const int* ksteps, int bf16, int what, int* mask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int start_bf = sched_cat(ksteps, b, 0, bf16) >= 2;
  const int K = max(ksteps[2 * b], 1);
  mask[b] = what == 0 ? !start_bf : what == 1 ? start_bf : (K & 1);
}
__global__ void k_sched_iters(int batch, const int* ksteps, int* iters) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < batch) iters[b] = max(ksteps[2 * b], 1);
}
// dst[b] = src[b] (per_matrix floats, a multiple of 4) for the masked matrices
__global__ void k_copy_masked(const float* src, float* dst, int64_t per_matrix, const int* mask) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const f4v* s4 = (const f4v*)(src + b * per_matrix);
  f4v* d4 = (f4v*)(dst + b * per_matrix);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_matrix / 4;
       i += (int64_t)gridDim.x * blockDim.x)
    d4[i] = s4[i];
}
// the same for a per-matrix size that is not a multiple of 4 (no vector
// alignment across matrices)
__global__ void k_copy_masked1(const float* src, float* dst, int64_t per_matrix, const int* mask) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_matrix;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[b * per_matrix + i] = src[b * per_matrix + i];
}
}  // namespace

hipError_t sched_mask_launch(int batch, const int* ksteps, int bf16, int what, int* mask, hipStream_t st) {
  hipLaunchKernelGGL(k_sched_mask, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch, ksteps, bf16, what, mask);
  LAUNCH_CHECK();
}
hipError_t sched_iters_launch(int batch, const int* ksteps, int* iters, hipStream_t st) {
  hipLaunchKernelGGL(k_sched_iters, dim3(cdiv(batch, 256)), dim3(256), 0, st, batch, ksteps, iters);
  LAUNCH_CHECK();
}
hipError_t copy_masked_launch(const float* src, float* dst, int batch, int64_t per_matrix, const int* mask,
                              hipStream_t st) {
  if (per_matrix <= 0 || batch <= 0) return hipSuccess;
  if (per_matrix % 4)
    hipLaunchKernelGGL(k_copy_masked1, dim3(grid1(per_matrix, 256), batch), dim3(256), 0, st, src, dst,
                       per_matrix, mask);
  else
    hipLaunchKernelGGL(k_copy_masked, dim3(grid1(per_matrix / 4, 256), batch), dim3(256), 0, st, src, dst,
                       per_matrix, mask);
  LAUNCH_CHECK();
}

// ---- spectral divide and conquer -------------------------------------------
namespace {

// fixed-order sum of one value per thread over a 1024-thread block
SVDP_DEV double block_sum_1024(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// sigma = trace(H) / n (one block)
__global__ __launch_bounds__(1024) void k_dc_sigma(const float* H, int64_t ldh, int n, float* sigma) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += H[(int64_t)i * ldh + i];
  const double mu = block_sum_1024(s, red) / n;
  if (threadIdx.x == 0) *sigma = (float)mu;
}

// dst = (src + src^T) / 2 - sigma I (s x s; sigma null: 0), exactly
// symmetric.  One 32 x 32 tile pair (I, J), (J, I) with I <= J per block,
// both read into LDS before either is written, so dst may be src.
__global__ __launch_bounds__(256) void k_dc_sym(const float* src, int64_t lds, float* dst, int64_t ldd, int s,
                                               const float* sigma) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (I > J) return;
  __shared__ float a[32][33], b[32][33];  // tile (I, J) and tile (J, I)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const float mu = sigma ? *sigma : 0.f;
  for (int r = ty; r < 32; r += 8) {
    const int i = I * 32 + r, j = J * 32 + tx;
    a[r][tx] = (i < s && j < s) ? src[(int64_t)i * lds + j] : 0.f;
    const int i2 = J * 32 + r, j2 = I * 32 + tx;
    b[r][tx] = (i2 < s && j2 < s) ? src[(int64_t)i2 * lds + j2] : 0.f;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = I * 32 + r, j = J * 32 + tx;
    if (i < s && j < s) dst[(int64_t)i * ldd + j] = 0.5f * (a[r][tx] + b[tx][r]) - (i == j ? mu : 0.f);
    const int i2 = J * 32 + r, j2 = I * 32 + tx;
    if (I != J && i2 < s && j2 < s) dst[(int64_t)i2 * ldd + j2] = 0.5f * (b[r][tx] + a[tx][r]);
  }
}

// k = round((n + trace W) / 2), the rank of the projector (I + W) / 2, W =
// sel[0] ? X1 : X0.  k = 0 (no split) when the polar iteration did not
// converge or met non-finite values (flags[0]), or when |W|_F^2 (wn2[1])
// differs from n by more than 1/2: W is then not orthogonal, as for a shifted
// matrix with a zero direction, whose polar factor loses that direction
__global__ __launch_bounds__(1024) void k_dc_rank(const float* X0, const float* X1, const int* sel,
                                                 const double* wn2, const int* flags, int n, int* k) {
  __shared__ double red[1024];
  const float* W = sel[0] ? X1 : X0;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += W[(int64_t)i * n + i];
  const double tr = block_sum_1024(s, red);
  if (threadIdx.x == 0) {
    const long r = lrint(0.5 * (n + tr));
    const bool bad = (flags[0] & (SVDP_FLAG_NOT_CONVERGED | SVDP_FLAG_NONFINITE)) != 0 || !isfinite(tr) ||
                     !(fabs(wn2[1] - n) <= 0.5);
    *k = bad ? 0 : (int)(r < 0 ? 0 : (r > n ? n : r));
  }
}

// the pieces' sweep counts and flags -> the matrix's (max, or).  The pieces
// are solved shifted by their mean eigenvalue, so their NEG_EIGENVALUE says
// nothing about the matrix and is dropped.
__global__ void k_dc_info(const int* sw, const int* fl, int count, int* sweeps, int* flags) {
  if (threadIdx.x == 0) {
    int m = 0, f = 0;
    for (int i = 0; i < count; ++i) {
      m = sw[i] > m ? sw[i] : m;
      f |= fl[i];
    }
    *sweeps = m;
    *flags |= f & ~SVDP_FLAG_NEG_EIGENVALUE;
  }
}

// *flags |= NEG_EIGENVALUE when some lam[i] < -neg_tol max |lam| (one block)
__global__ __launch_bounds__(1024) void k_dc_neg(const float* lam, int n, float neg_tol, int* flags) {
  __shared__ float vmax, vneg;
  if (threadIdx.x == 0) { vmax = 0.f; vneg = 0.f; }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = lam[i];
    if (!isfinite(d)) continue;
    atomicMax((int*)&vmax, __float_as_int(fabsf(d)));  // |d| >= 0: int order = float order
    if (d < 0.f) atomicMax((int*)&vneg, __float_as_int(-d));
  }
  __syncthreads();
  if (threadIdx.x == 0 && vneg > neg_tol * vmax) *flags |= SVDP_FLAG_NEG_EIGENVALUE;
}

// The SVD's order of an eigendecomposition of H = W^T A (one matrix, lam
// descending by value): lam <- |lam| descending (ties by index), sgn = the
// signs, perm = the source positions, flags as the Jacobi solver raises them
// for H (NONFINITE; NEG_EIGENVALUE below -neg_tol max |lam|).  One block of
// 1024 threads, dynamic LDS 8 P2 bytes (P2 = next power of two >= n); the
// signs are read from lam before a barrier, the sorted values written after.
__global__ __launch_bounds__(1024) void k_dc_abs_sort(float* lam, int n, float* sgn, int* perm, float neg_tol,
                                                     int* flags) {
  extern __shared__ unsigned char smem[];
  int P2 = 1;
  while (P2 < n) P2 <<= 1;
  float* key = (float*)smem;
  int* idx = (int*)(key + P2);
  __shared__ float vmax, vneg;
  __shared__ int bad;
  if (threadIdx.x == 0) { vmax = 0.f; vneg = 0.f; bad = 0; }
  __syncthreads();
  for (int i = threadIdx.x; i < P2; i += blockDim.x) {
    float d = i < n ? lam[i] : 0.f;
    if (i < n && !isfinite(d)) { bad = 1; d = 0.f; }
    key[i] = i < n ? fabsf(d) : -INFINITY;
    idx[i] = i;
    if (i < n) {
      atomicMax((int*)&vmax, __float_as_int(fabsf(d)));  // |d| >= 0: int order = float order
      if (d < 0.f) atomicMax((int*)&vneg, __float_as_int(-d));
    }
  }
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < P2; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool desc = (i & size) == 0;
          const float ki = key[i], kj = key[j];
          const int ii = idx[i], ij = idx[j];
          const bool i_first = ki > kj || (ki == kj && ii < ij);
          if (desc != i_first) {
            key[i] = kj; key[j] = ki;
            idx[i] = ij; idx[j] = ii;
          }
        }
      }
      __syncthreads();
    }
  for (int c = threadIdx.x; c < n; c += blockDim.x) sgn[c] = lam[idx[c]] < 0.f ? -1.f : 1.f;
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    lam[c] = key[c];
    perm[c] = idx[c];
  }
  if (threadIdx.x == 0) {
    int f = 0;
    if (bad) f |= SVDP_FLAG_NONFINITE;
    if (vneg > neg_tol * vmax) f |= SVDP_FLAG_NEG_EIGENVALUE;
    if (f) *flags |= f;
  }
}

// V[i, c] <- V[i, perm[c]] (n x n, pitch ldv), one row per block through LDS
__global__ void k_dc_permute_cols(float* V, int64_t ldv, int n, const int* perm) {
  extern __shared__ float row[];
  float* v = V + (int64_t)blockIdx.x * ldv;
  for (int c = threadIdx.x; c < n; c += blockDim.x) row[c] = v[c];
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) v[c] = row[perm[c]];
}

// dst (rows x cols, pitch ldd) <- sel[0] ? X1 : X0 (pitch lds), one row per block
__global__ void k_dc_copy_sel(const float* X0, const float* X1, const int* sel, int64_t lds, float* dst,
                              int64_t ldd, int cols) {
  const float* src = sel[0] ? X1 : X0;
  const int64_t i = blockIdx.x;
  for (int j = threadIdx.x; j < cols; j += blockDim.x) dst[i * ldd + j] = src[i * lds + j];
}

// x[i] += *mu
__global__ void k_dc_add(float* x, int n, const float* mu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += *mu;
}

// A piece of size s solved inside a zero-padded P x P matrix: its padding
// rows and columns are zero, never rotated, so the padding eigenpairs are
// (0, e_j) for j >= s and the piece's eigenvectors are zero in rows >= s.
// Column c of V (P x P, row-major, columns the eigenvectors) is padding when
// its squared norm over rows s.. exceeds 1/2.  map[c] = the position of c
// among the piece's columns in order (-1 for padding); EIGH_NOT_CONVERGED
// when the count is not s.  One block of 1024 threads, P <= 1024.
__global__ __launch_bounds__(1024) void k_dc_leaf_map(const float* V, int P, int s, int* map, int* flags) {
  __shared__ int scan[1024];
  const int c = threadIdx.x;
  int real = 0;
  if (c < P) {
    float pad = 0.f;
    for (int i = s; i < P; ++i) {
      const float v = V[(int64_t)i * P + c];
      pad += v * v;
    }
    real = pad <= 0.5f ? 1 : 0;
  }
  scan[c] = real;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
    const int add = c >= d ? scan[c - d] : 0;
    __syncthreads();
    scan[c] += add;
    __syncthreads();
  }
  if (c < P) map[c] = real ? scan[c] - 1 : -1;
  if (c == 0 && scan[1023] != s) *flags |= SVDP_FLAG_EIGH_NOT_CONVERGED;
}

// The piece's eigenpairs in order: lam_out[map[c]] = lam[c] + mu, and row i < s
// of V_out (pitch ldo) from row i of V (P x P); one row per block.  Positions
// beyond s (a miscount, already flagged) are not written.
__global__ void k_dc_leaf_extract(const float* V, const float* lam, const float* mu, int P, int s, const int* map,
                                  float* lam_out, float* V_out, int64_t ldo) {
  const int64_t i = blockIdx.x;
  for (int c = threadIdx.x; c < P; c += blockDim.x) {
    const int d = map[c];
    if (d < 0 || d >= s) continue;
    V_out[i * ldo + d] = V[i * P + c];
    if (i == 0) lam_out[d] = lam[c] + *mu;
  }
}

// seeded uniform values in [-1, 1): a 32-bit integer hash of (seed, index)
// (the finaliser of MurmurHash3) mapped to 24-bit fractions
__global__ void k_dc_random(float* out, int64_t count, uint32_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    uint32_t h = seed ^ (uint32_t)(i * 0x9E3779B9u) ^ (uint32_t)(i >> 32);
    h ^= h >> 16; h *= 0x85EBCA6Bu; h ^= h >> 13; h *= 0xC2B2AE35u; h ^= h >> 16;
    out[i] = (float)(h >> 8) * (1.f / 8388608.f) - 1.f;
  }
}

// cs[j] = +1 for the first k columns, -1 after
__global__ void k_dc_signs(float* cs, int n, const int* k) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) cs[j] = j < *k ? 1.f : -1.f;
}

// part[2 r], part[2 r + 1] = row r's sums of T[r, j]^2 over j >= k (rows
// r < k) and over all j (T = sel && sel[0] ? T1 : T0, n x n row-major; no k:
// k = 0), one row per block
__global__ void k_dc_coupling_rows(const float* T0, const float* T1, const int* sel, int n, const int* k,
                                   double* part) {
  __shared__ double red[2][256];
  const int r = blockIdx.x, kk = k ? *k : 0;
  const float* T = sel && sel[0] ? T1 : T0;
  double e = 0.0, a = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double v = T[(int64_t)r * n + j];
    a += v * v;
    if (r < kk && j >= kk) e += v * v;
  }
  red[0][threadIdx.x] = e;
  red[1][threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * r] = red[0][0];
    part[2 * r + 1] = red[1][0];
  }
}

// part[2 r] = row r's sum of (G[r, j] - delta_rj)^2, part[2 r + 1] = 0 (G
// n x n row-major), one row per block
__global__ void k_dc_dev_rows(const float* G, int n, double* part) {
  __shared__ double red[256];
  const int r = blockIdx.x;
  double e = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double v = (double)G[(int64_t)r * n + j] - (r == j ? 1.0 : 0.0);
    e += v * v;
  }
  red[threadIdx.x] = e;
  __syncthreads();
  for (int t = 128; t > 0; t >>= 1) {
    if (threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * r] = red[0];
    part[2 * r + 1] = 0.0;
  }
}

// out[0] = |T[:k, k:]|_F^2, out[1] = |T|_F^2: the row sums added in row order
__global__ __launch_bounds__(1024) void k_dc_coupling_sum(const double* part, int n, double* out) {
  __shared__ double red[1024];
  double e = 0.0, a = 0.0;
  for (int r = threadIdx.x; r < n; r += 1024) {
    e += part[2 * r];
    a += part[2 * r + 1];
  }
  const double se = block_sum_1024(e, red);
  const double sa = block_sum_1024(a, red);
  if (threadIdx.x == 0) {
    out[0] = se;
    out[1] = sa;
  }
}

}  // namespace

hipError_t dc_shift_launch(const float* H, int64_t ldh, float* A, int64_t lda, int n, float* sigma,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_dc_sigma, dim3(1), dim3(1024), 0, st, H, ldh, n, sigma);
  hipError_t e = hipGetLastError();
  if (e) return e;
  const unsigned nt = (unsigned)cdiv(n, 32);
  hipLaunchKernelGGL(k_dc_sym, dim3(nt, nt), dim3(256), 0, st, H, ldh, A, lda, n, sigma);
  LAUNCH_CHECK();
}
hipError_t dc_abs_order_launch(float* lam, float* V, int64_t ldv, int n, float* sgn, int* perm, float neg_tol,
                               int* flags, hipStream_t st) {
  if (n < 1 || n > 8192) return hipErrorInvalidValue;
  int P2 = 1;
  while (P2 < n) P2 <<= 1;
  hipLaunchKernelGGL(k_dc_abs_sort, dim3(1), dim3(1024), (size_t)8 * P2, st, lam, n, sgn, perm, neg_tol, flags);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_dc_permute_cols, dim3(n), dim3(256), (size_t)4 * n, st, V, ldv, n, perm);
  LAUNCH_CHECK();
}
hipError_t dc_neg_launch(const float* lam, int n, float neg_tol, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_neg, dim3(1), dim3(1024), 0, st, lam, n, neg_tol, flags);
  LAUNCH_CHECK();
}
hipError_t dc_copy_sel_launch(const float* X0, const float* X1, const int* sel, int64_t lds, float* dst,
                              int64_t ldd, int rows, int cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dc_copy_sel, dim3(rows), dim3(256), 0, st, X0, X1, sel, lds, dst, ldd, cols);
  LAUNCH_CHECK();
}
hipError_t dc_add_launch(float* x, int n, const float* mu, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_add, dim3(cdiv(n, 256)), dim3(256), 0, st, x, n, mu);
  LAUNCH_CHECK();
}
hipError_t dc_sym_launch(float* T, int64_t ldt, int n, hipStream_t st) {
  const unsigned nt = (unsigned)cdiv(n, 32);
  hipLaunchKernelGGL(k_dc_sym, dim3(nt, nt), dim3(256), 0, st, T, ldt, T, ldt, n, nullptr);
  LAUNCH_CHECK();
}
hipError_t dc_rank_launch(const float* X0, const float* X1, const int* sel, const double* wn2, const int* flags,
                          int n, int* k, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_rank, dim3(1), dim3(1024), 0, st, X0, X1, sel, wn2, flags, n, k);
  LAUNCH_CHECK();
}
hipError_t dc_info_launch(const int* sw, const int* fl, int count, int* sweeps, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_info, dim3(1), dim3(64), 0, st, sw, fl, count, sweeps, flags);
  LAUNCH_CHECK();
}
hipError_t dc_leaf_launch(const float* V, const float* lam, const float* mu, int P, int s, int* map, float* lam_out,
                          float* V_out, int64_t ldo, int* flags, hipStream_t st) {
  if (P < 1 || P > 1024 || s < 1 || s > P) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dc_leaf_map, dim3(1), dim3(1024), 0, st, V, P, s, map, flags);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_dc_leaf_extract, dim3(s), dim3(256), 0, st, V, lam, mu, P, s, map, lam_out, V_out, ldo);
  LAUNCH_CHECK();
}
hipError_t dc_random_launch(float* out, int64_t count, uint32_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_random, dim3(512), dim3(256), 0, st, out, count, seed);
  LAUNCH_CHECK();
}
hipError_t dc_signs_launch(float* cs, int n, const int* k, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_signs, dim3(cdiv(n, 256)), dim3(256), 0, st, cs, n, k);
  LAUNCH_CHECK();
}
hipError_t dc_dev_launch(const float* G, int n, double* part, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_dev_rows, dim3(n), dim3(256), 0, st, G, n, part);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_dc_coupling_sum, dim3(1), dim3(1024), 0, st, part, n, out);
  LAUNCH_CHECK();
}
hipError_t dc_coupling_launch(const float* T0, const float* T1, const int* sel, int n, const int* k, double* part,
                              double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_dc_coupling_rows, dim3(n), dim3(256), 0, st, T0, T1, sel, n, k, part);
  hipError_t e = hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_dc_coupling_sum, dim3(1), dim3(1024), 0, st, part, n, out);
  LAUNCH_CHECK();
}
