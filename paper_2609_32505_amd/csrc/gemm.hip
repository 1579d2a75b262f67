// Batched strided GEMM on gfx950 matrix cores (MFMA), with the fused
// epilogues the SVD path needs (CANS update alpha X + beta X G, symmetric
// Gram output, column scaling, per-matrix skip and convergence sums).
//
// Two kernels: FP32 inputs on v_mfma_f32_32x32x2f32, and BF16 operands (from
// FP32 or BF16 storage) on v_mfma_f32_32x32x16_bf16, both accumulating in
// FP32.  A 256-thread workgroup owns a BM x BN output tile (4 waves, each a
// (BM/2) x (BN/2) sub-tile of 32x32 MFMA blocks); K is walked in BK slices
// staged through double-buffered LDS.  Operands stored with the contraction
// index strided are transposed on their way into LDS, so the MFMA operand
// reads are always contiguous.
#include "common.hpp"
#include "prof.hpp"

namespace {

thread_local int g_prof_kind = PROF_GEMM_F32;

// Linear block id -> (matrix, tile).  Workgroups are dealt to the 8 XCDs
// round-robin by linear id; with remap every tile of matrix b runs on XCD
// b % 8, so the panels of one matrix are fetched into one L2 only.
SVDP_DEV bool map_block(int ntiles, int batch, int remap, int& b, int& tile) {
  int L = blockIdx.x;
  if (!remap) {
    b = L / ntiles;
    tile = L - b * ntiles;
    return b < batch;
  }
  int x = L & 7, q = L >> 3;
  int grp = q / ntiles;
  tile = q - grp * ntiles;
  b = grp * 8 + x;
  return b < batch;
}

// upper-triangular tile enumeration (tm <= tn), row by row
SVDP_DEV void sym_tile(int t, int T, int& tm, int& tn) {
  int r = 0;
  while (t >= T - r) { t -= T - r; ++r; }
  tm = r;
  tn = r + t;
}

// Profiling: the tile's algorithmic flops, 2 r c K (r x c the tile inside the
// output), half of it on the diagonal of a symmetric output (its triangle)
SVDP_DEV void count_tile(const GemmArgs& g, int m0, int n0, int BM, int BN, int tm, int tn) {
  if (!g.work || threadIdx.x != 0) return;
  const double r = min(BM, g.M - m0), c = min(BN, g.N - n0);
  atomicAdd(g.work, (g.sym && tm == tn ? 1.0 : 2.0) * r * c * (double)g.K);
}

// Shared epilogue over one wave's accumulators.  acc[f] holds a 32x32 block
// in the MFMA output layout: lane l, slot 4g + r -> row 8g + 4(l/32) + r,
// column l % 32.
template <int FM, int FN>
SVDP_DEV void epilogue(const GemmArgs& g, int b, int rowbase, int colbase, int tm, int tn,
                       f16v (&acc)[FM][FN]) {
  const int lane = threadIdx.x & 63;
  float s_acc = g.alpha, s_in = g.beta;
  if (g.coef) {
    const float* c = g.coef + (b * g.coef_bstride + g.coef_idx) * 2;
    s_in = c[0];
    s_acc = c[1];
  }
  const float* cs = g.colscale ? g.colscale + b * g.cs_stride : nullptr;
  const float* csi = g.colscale_in ? g.colscale_in + b * g.csin_stride : nullptr;
  const char* cin = g.Cin ? (const char*)g.Cin + b * g.sCin * (g.cin_bf16 ? 2 : 4) : nullptr;
  // output format: per matrix from its schedule category when a BF16
  // destination is given (the workgroup ran, so the category is >= 0), else
  // out_bf16
  const bool percat = g.ksched && g.C_bf;
  const int obf = percat ? (g.obf_catmask >> sched_cat(g.ksched, b, g.kstep, g.kbf16)) & 1 : g.out_bf16;
  char* out = (char*)(percat && obf ? g.C_bf : g.C) + b * g.sC * (obf ? 2 : 4);
  bf16_t* outt = (g.Ct && obf) ? (bf16_t*)g.Ct + b * g.sCt : nullptr;
  float d2 = 0.f, o2 = 0.f;
  const bool mirror = g.sym && tm != tn;
#pragma unroll
  for (int mi = 0; mi < FM; ++mi)
#pragma unroll
    for (int ni = 0; ni < FN; ++ni) {
      const int j = colbase + ni * 32 + (lane & 31);
      if (j >= g.N) continue;
      const float csj = cs ? cs[j] : 1.f;
      const float csij = csi ? csi[j] : 1.f;
      // the block's 16 Cin values, all loaded before its first store: the
      // compiler cannot tell that the output does not alias Cin, so a load
      // placed after a store would be waited for on its own
      float cv[16];
      if (cin) {
        const int ib = rowbase + mi * 32 + 4 * (lane >> 5);
        if (g.cin_bf16) {
          bf16_t raw[16];
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int i = ib + 8 * (e >> 2) + (e & 3);
            raw[e] = ((const bf16_t*)cin)[i < g.M ? (int64_t)i * g.ldcin + j : 0];
          }
#pragma unroll
          for (int e = 0; e < 16; ++e) cv[e] = (float)raw[e];
        } else {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const int i = ib + 8 * (e >> 2) + (e & 3);
            cv[e] = ((const float*)cin)[i < g.M ? (int64_t)i * g.ldcin + j : 0];
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i0 = rowbase + mi * 32 + 8 * q + 4 * (lane >> 5);
        bf16_t tv[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r;
          tv[r] = f2bf(0.f);
          if (i >= g.M) continue;
          float v = s_acc * acc[mi][ni][4 * q + r] * csj;
          if (cin) {
            const float c = cv[4 * q + r];
            v += s_in * c * csij;
            d2 += (v - c) * (v - c);
          }
          o2 += v * v;
          if (obf) {
            const bf16_t h = f2bf(v);
            tv[r] = h;
            ((bf16_t*)out)[(int64_t)i * g.ldc + j] = h;
            if (mirror) ((bf16_t*)out)[(int64_t)j * g.ldc + i] = h;
          } else {
            ((float*)out)[(int64_t)i * g.ldc + j] = v;
            if (mirror) ((float*)out)[(int64_t)j * g.ldc + i] = v;
          }
        }
        // the transposed copy: rows i0 .. i0 + 3 of column j are consecutive
        // in row j of Ct, one 8-byte store when all four are inside
        if (outt) {
          bf16_t* dst = outt + (int64_t)j * g.ldct + i0;
          if (i0 + 3 < g.M && (g.ldct & 3) == 0) {
            typedef __bf16 bf4v __attribute__((ext_vector_type(4)));
            bf4v pk = {tv[0], tv[1], tv[2], tv[3]};
            *(bf4v*)dst = pk;
          } else {
            for (int r = 0; r < 4 && i0 + r < g.M; ++r) dst[r] = tv[r];
          }
        }
      }
    }
  if (g.conv && rowbase < g.M && colbase < g.N) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      d2 += __shfl_xor(d2, off);
      o2 += __shfl_xor(o2, off);
    }
    // one slot per wave sub-tile (32 FM x 32 FN), added in order by the check
    const int slots_n = (g.N + 32 * FN - 1) / (32 * FN);
    const int slots = ((g.M + 32 * FM - 1) / (32 * FM)) * slots_n;
    const int slot = (rowbase / (32 * FM)) * slots_n + colbase / (32 * FN);
    if (lane == 0) {
      g.conv[((int64_t)b * slots + slot) * 2] = d2;
      g.conv[((int64_t)b * slots + slot) * 2 + 1] = o2;
    }
  }
}

// ------------------------------------------------------------------ FP32

template <int BM, int BN, bool TA, bool TB, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_gemm_f32(GemmArgs g, int tiles_m, int tiles_n,
                                                  int ntiles, int remap) {
  constexpr int BK = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int PAD = 4;
  __shared__ float As[2][BK][BM + PAD];
  __shared__ float Bs[2][BK][BN + PAD];
  int b, tile;
  if (!map_block(ntiles, g.batch, remap, b, tile)) return;
  if (g.active && !g.active[b]) return;
  if (g.ksched) {
    const int cat = sched_cat(g.ksched, b, g.kstep, g.kbf16);
    if (cat < 0 || !((g.kcatmask >> cat) & 1)) return;
  }
  int tm, tn;
  if (g.sym) sym_tile(tile, tiles_m, tm, tn);
  else { tm = tile / tiles_n; tn = tile - tm * tiles_n; }
  const int m0 = tm * BM, n0 = tn * BN;
  count_tile(g, m0, n0, BM, BN, tm, tn);
  const float* A = (const float*)((g.a_sel && g.a_sel[b]) ? g.A_alt : g.A) + b * g.sA;
  const float* B = (const float*)((g.b_sel && g.b_sel[b]) ? g.B_alt : g.B) + b * g.sB;
  const int M = g.M, N = g.N, K = g.K;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;

  // A tile: BM x BK of op(A) = BM*BK/4 float4 units, UA per thread
  constexpr int UA = BM * BK / 4 / 256;
  constexpr int UB = BN * BK / 4 / 256;
  f4v ra[UA], rb[UB];

  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      int idx = t + 256 * u;
      int i, k;
      if (TA) { k = idx / (BM / 4); i = (idx % (BM / 4)) * 4; }   // rows of k, m contiguous
      else { i = idx / (BK / 4); k = (idx % (BK / 4)) * 4; }      // rows of m, k contiguous
      int gi = m0 + i, gk = k0 + k;
      f4v v = {0.f, 0.f, 0.f, 0.f};
      if (TA) {
        if (gk < K) {
          const float* p = A + (int64_t)gk * g.lda + gi;
          if (VEC && gi + 3 < M) v = *(const f4v*)p;
          else for (int c = 0; c < 4; ++c) v[c] = (gi + c < M) ? p[c] : 0.f;
        }
      } else {
        if (gi < M) {
          const float* p = A + (int64_t)gi * g.lda + gk;
          if (VEC && gk + 3 < K) v = *(const f4v*)p;
          else for (int c = 0; c < 4; ++c) v[c] = (gk + c < K) ? p[c] : 0.f;
        }
      }
      ra[u] = v;
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int idx = t + 256 * u;
      int j, k;
      if (!TB) { k = idx / (BN / 4); j = (idx % (BN / 4)) * 4; }
      else { j = idx / (BK / 4); k = (idx % (BK / 4)) * 4; }
      int gj = n0 + j, gk = k0 + k;
      f4v v = {0.f, 0.f, 0.f, 0.f};
      if (!TB) {
        if (gk < K) {
          const float* p = B + (int64_t)gk * g.ldb + gj;
          if (VEC && gj + 3 < N) v = *(const f4v*)p;
          else for (int c = 0; c < 4; ++c) v[c] = (gj + c < N) ? p[c] : 0.f;
        }
      } else {
        if (gj < N) {
          const float* p = B + (int64_t)gj * g.ldb + gk;
          if (VEC && gk + 3 < K) v = *(const f4v*)p;
          else for (int c = 0; c < 4; ++c) v[c] = (gk + c < K) ? p[c] : 0.f;
        }
      }
      rb[u] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      int idx = t + 256 * u;
      if (TA) {
        int k = idx / (BM / 4), i = (idx % (BM / 4)) * 4;
        *(f4v*)&As[buf][k][i] = ra[u];
      } else {
        int i = idx / (BK / 4), k = (idx % (BK / 4)) * 4;
        for (int c = 0; c < 4; ++c) As[buf][k + c][i] = ra[u][c];
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int idx = t + 256 * u;
      if (!TB) {
        int k = idx / (BN / 4), j = (idx % (BN / 4)) * 4;
        *(f4v*)&Bs[buf][k][j] = rb[u];
      } else {
        int j = idx / (BK / 4), k = (idx % (BK / 4)) * 4;
        for (int c = 0; c < 4; ++c) Bs[buf][k + c][j] = rb[u][c];
      }
    }
  };

  f16v acc[FM][FN];
#pragma unroll
  for (int mi = 0; mi < FM; ++mi)
#pragma unroll
    for (int ni = 0; ni < FN; ++ni)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[mi][ni][e] = 0.f;

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      float av[FM], bv[FN];
#pragma unroll
      for (int mi = 0; mi < FM; ++mi) av[mi] = As[cur][kk + (lane >> 5)][wm * WM + mi * 32 + (lane & 31)];
#pragma unroll
      for (int ni = 0; ni < FN; ++ni) bv[ni] = Bs[cur][kk + (lane >> 5)][wn * WN + ni * 32 + (lane & 31)];
#pragma unroll
      for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
  epilogue<FM, FN>(g, b, m0 + wm * WM, n0 + wn * WN, tm, tn, acc);
}

// ------------------------------------------------------------------ BF16

template <int BM, int BN, bool TA, bool TB, bool INBF, bool VEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 4))) void k_gemm_bf16(GemmArgs g, int tiles_m, int tiles_n,
                                                   int ntiles, int remap) {
  constexpr int BK = 64;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int LDK = BK + 8;  // row stride (bf16) of the k-contiguous LDS tiles
  // An operand stored with the contraction index strided (A when TA, B when
  // !TB) stays k-major in LDS (rows of k, 16-byte vector stores); its MFMA
  // operands (8 consecutive k per lane) are then gathered with 2-byte reads
  // that are contiguous across lanes.  Transposing it on the way in would
  // make every store an 8-row-stride scatter (16-way bank conflicts).
  constexpr int LDA = TA ? BM + 8 : LDK;
  constexpr int LDB = TB ? LDK : BN + 8;
  // one LDS buffer (37 KB at 128 x 128): the next K slice waits in
  // registers during the MFMAs, so four workgroups fit a CU
  __shared__ bf16_t As[1][TA ? BK : BM][LDA];
  __shared__ bf16_t Bs[1][TB ? BN : BK][LDB];
  int b, tile;
  if (!map_block(ntiles, g.batch, remap, b, tile)) return;
  if (g.active && !g.active[b]) return;
  if (g.ksched) {
    const int cat = sched_cat(g.ksched, b, g.kstep, g.kbf16);
    if (cat < 0 || !((g.kcatmask >> cat) & 1)) return;
  }
  int tm, tn;
  if (g.sym) sym_tile(tile, tiles_m, tm, tn);
  else { tm = tile / tiles_n; tn = tile - tm * tiles_n; }
  const int m0 = tm * BM, n0 = tn * BN;
  count_tile(g, m0, n0, BM, BN, tm, tn);
  const int esz = INBF ? 2 : 4;
  const char* A = (const char*)((g.a_sel && g.a_sel[b]) ? g.A_alt : g.A) + b * g.sA * esz;
  const char* B = (const char*)((g.b_sel && g.b_sel[b]) ? g.B_alt : g.B) + b * g.sB * esz;
  const int M = g.M, N = g.N, K = g.K;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;

  constexpr int UA = BM * BK / 8 / 256;
  constexpr int UB = BN * BK / 8 / 256;
  bf8v ra[UA], rb[UB];

  // 8 consecutive elements starting at p (element units), masked by count
  auto ld8 = [&](const char* base, int64_t off, int valid) -> bf8v {
    bf8v v;
    if (INBF) {
      const bf16_t* p = (const bf16_t*)base + off;
      if (VEC && valid >= 8) v = *(const bf8v*)p;
      else for (int c = 0; c < 8; ++c) v[c] = c < valid ? p[c] : f2bf(0.f);
    } else {
      const float* p = (const float*)base + off;
      if (VEC && valid >= 8) {
        f4v x0 = *(const f4v*)p, x1 = *(const f4v*)(p + 4);
        for (int c = 0; c < 4; ++c) { v[c] = f2bf(x0[c]); v[c + 4] = f2bf(x1[c]); }
      } else {
        for (int c = 0; c < 8; ++c) v[c] = f2bf(c < valid ? p[c] : 0.f);
      }
    }
    return v;
  };
  const bf8v zero8 = {};

  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      int idx = t + 256 * u;
      if (TA) {  // A stored K x M: vectors along m
        int k = idx / (BM / 8), i = (idx % (BM / 8)) * 8;
        int gk = k0 + k, gi = m0 + i;
        ra[u] = (gk < K && gi < M) ? ld8(A, (int64_t)gk * g.lda + gi, M - gi) : zero8;
      } else {   // A stored M x K: vectors along k
        int i = idx / (BK / 8), k = (idx % (BK / 8)) * 8;
        int gk = k0 + k, gi = m0 + i;
        ra[u] = (gi < M && gk < K) ? ld8(A, (int64_t)gi * g.lda + gk, K - gk) : zero8;
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int idx = t + 256 * u;
      if (!TB) {  // B stored K x N: vectors along n
        int k = idx / (BN / 8), j = (idx % (BN / 8)) * 8;
        int gk = k0 + k, gj = n0 + j;
        rb[u] = (gk < K && gj < N) ? ld8(B, (int64_t)gk * g.ldb + gj, N - gj) : zero8;
      } else {    // B stored N x K: vectors along k
        int j = idx / (BK / 8), k = (idx % (BK / 8)) * 8;
        int gk = k0 + k, gj = n0 + j;
        rb[u] = (gj < N && gk < K) ? ld8(B, (int64_t)gj * g.ldb + gk, K - gk) : zero8;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      int idx = t + 256 * u;
      if (TA) {
        int k = idx / (BM / 8), i = (idx % (BM / 8)) * 8;
        *(bf8v*)&As[buf][k][i] = ra[u];
      } else {
        int i = idx / (BK / 8), k = (idx % (BK / 8)) * 8;
        *(bf8v*)&As[buf][i][k] = ra[u];
      }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      int idx = t + 256 * u;
      if (!TB) {
        int k = idx / (BN / 8), j = (idx % (BN / 8)) * 8;
        *(bf8v*)&Bs[buf][k][j] = rb[u];
      } else {
        int j = idx / (BK / 8), k = (idx % (BK / 8)) * 8;
        *(bf8v*)&Bs[buf][j][k] = rb[u];
      }
    }
  };

  f16v acc[FM][FN];
#pragma unroll
  for (int mi = 0; mi < FM; ++mi)
#pragma unroll
    for (int ni = 0; ni < FN; ++ni)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[mi][ni][e] = 0.f;

  const int nk = (K + BK - 1) / BK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = 0;
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 16) {
      bf8v av[FM], bv[FN];
      const int k8 = kk + (lane >> 5) * 8;
#pragma unroll
      for (int mi = 0; mi < FM; ++mi) {
        const int i = wm * WM + mi * 32 + (lane & 31);
        if (TA) {
#pragma unroll
          for (int c = 0; c < 8; ++c) av[mi][c] = As[cur][k8 + c][i];
        } else {
          av[mi] = *(const bf8v*)&As[cur][i][k8];
        }
      }
#pragma unroll
      for (int ni = 0; ni < FN; ++ni) {
        const int j = wn * WN + ni * 32 + (lane & 31);
        if (!TB) {
#pragma unroll
          for (int c = 0; c < 8; ++c) bv[ni][c] = Bs[cur][k8 + c][j];
        } else {
          bv[ni] = *(const bf8v*)&Bs[cur][j][k8];
        }
      }
#pragma unroll
      for (int mi = 0; mi < FM; ++mi)
#pragma unroll
        for (int ni = 0; ni < FN; ++ni)
          acc[mi][ni] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      __syncthreads();  // every wave is done with this slice
      store(0);
    }
    __syncthreads();
  }
  epilogue<FM, FN>(g, b, m0 + wm * WM, n0 + wn * WN, tm, tn, acc);
}

template <typename KernelT>
hipError_t launch_tiles(KernelT kern, const GemmArgs& g, int BM, int BN, hipStream_t st) {
  int tiles_m = cdiv(g.M, BM), tiles_n = cdiv(g.N, BN);
  int ntiles = g.sym ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
  int remap = g.batch >= 8 ? 1 : 0;
  int64_t blocks = remap ? (int64_t)cdiv(g.batch, 8) * 8 * ntiles : (int64_t)g.batch * ntiles;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  // algorithmic flops counted on the device by the tiles that run
  ProfScope ps(g_prof_kind, st, 0.0);
  GemmArgs ga = g;
  double* wd = prof_work_dev();
  ga.work = wd ? wd + g_prof_kind : nullptr;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, st, ga, tiles_m, tiles_n, ntiles, remap);
  return hipGetLastError();
}

template <int BM, bool TA, bool TB, bool VEC>
hipError_t dispatch_f32(const GemmArgs& g, hipStream_t st) {
  return launch_tiles(k_gemm_f32<BM, BM, TA, TB, VEC>, g, BM, BM, st);
}

template <int BM, bool TA, bool TB, bool INBF, bool VEC>
hipError_t dispatch_bf16(const GemmArgs& g, hipStream_t st) {
  return launch_tiles(k_gemm_bf16<BM, BM, TA, TB, INBF, VEC>, g, BM, BM, st);
}

template <int BM, bool VEC>
hipError_t by_trans_f32(const GemmArgs& g, int ta, int tb, hipStream_t st) {
  if (ta && tb) return dispatch_f32<BM, true, true, VEC>(g, st);
  if (ta) return dispatch_f32<BM, true, false, VEC>(g, st);
  if (tb) return dispatch_f32<BM, false, true, VEC>(g, st);
  return dispatch_f32<BM, false, false, VEC>(g, st);
}

template <int BM, bool INBF, bool VEC>
hipError_t by_trans_bf16(const GemmArgs& g, int ta, int tb, hipStream_t st) {
  if (ta && tb) return dispatch_bf16<BM, true, true, INBF, VEC>(g, st);
  if (ta) return dispatch_bf16<BM, true, false, INBF, VEC>(g, st);
  if (tb) return dispatch_bf16<BM, false, true, INBF, VEC>(g, st);
  return dispatch_bf16<BM, false, false, INBF, VEC>(g, st);
}

bool aligned(const void* p, int64_t ld, int64_t stride, int elems, int esz) {
  return ((uintptr_t)p % (elems * esz)) == 0 && ld % elems == 0 && stride % elems == 0;
}

}  // namespace

int gemm_conv_slots(int64_t M, int64_t N) {
  // the wave sub-tile of the tile size gemm_launch picks: 64 x 64 in 128 x 128
  // tiles, 32 x 32 in 64 x 64 tiles
  const int w = (M > 64 && N > 64) ? 64 : 32;
  return (int)(((M + w - 1) / w) * ((N + w - 1) / w));
}

hipError_t gemm_launch(const GemmArgs& g, int prec, int ta, int tb, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  g_prof_kind = prec == PREC_F32 ? PROF_GEMM_F32 : PROF_GEMM_BF16;
  if (g.sym && g.M != g.N) return hipErrorInvalidValue;
  const bool big = g.M > 64 && g.N > 64;
  if (prec == PREC_F32) {
    bool vec = aligned(g.A, g.lda, g.sA, 4, 4) && aligned(g.B, g.ldb, g.sB, 4, 4);
    if (big) return vec ? by_trans_f32<128, true>(g, ta, tb, st) : by_trans_f32<128, false>(g, ta, tb, st);
    return vec ? by_trans_f32<64, true>(g, ta, tb, st) : by_trans_f32<64, false>(g, ta, tb, st);
  }
  const int esz = g.in_bf16 ? 2 : 4;
  const int el = g.in_bf16 ? 8 : 4;
  bool vec = aligned(g.A, g.lda, g.sA, el, esz) && aligned(g.B, g.ldb, g.sB, el, esz);
  if (g.in_bf16) {
    if (big) return vec ? by_trans_bf16<128, true, true>(g, ta, tb, st) : by_trans_bf16<128, true, false>(g, ta, tb, st);
    return vec ? by_trans_bf16<64, true, true>(g, ta, tb, st) : by_trans_bf16<64, true, false>(g, ta, tb, st);
  }
  if (big) return vec ? by_trans_bf16<128, false, true>(g, ta, tb, st) : by_trans_bf16<128, false, false>(g, ta, tb, st);
  return vec ? by_trans_bf16<64, false, true>(g, ta, tb, st) : by_trans_bf16<64, false, false>(g, ta, tb, st);
}
