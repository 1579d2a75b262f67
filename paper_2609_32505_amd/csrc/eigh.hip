// Batched symmetric eigendecomposition H = V diag(lam) V^T by block Jacobi
// (the EVD step of the SVD-via-polar algorithm, Algorithm 1).
//
// Layout.  The index range is padded to np = 16 nb with nb a power of two
// (at least 4).  Padding rows and columns of H are zero and those of V the
// identity; a zero off-diagonal entry is never rotated, so padding stays
// inert.  H and V are stored as 16 x 16 tiles (tile (I, J) is 1 KB,
// contiguous, row-major inside); H keeps only the tiles with I <= J.
//
// Block ordering.  Step s (s = 1 .. nb - 1) of a sweep pairs block B with
// B ^ s.  Two steps (sA, sB) form a phase: the blocks fall into groups
// {B, B^sA, B^sB, B^sA^sB} that both pairings leave closed, so the rotations
// of the two steps compose to one 64 x 64 orthogonal M_G per group, and H
// and V are read and written once per two steps.
//   * k_jac_solve: one workgroup (two wavefronts) per group holds H[G, G] in
//     LDS.  Step A: wave w owns pair w, a 32 x 32 subproblem, and runs scalar
//     Jacobi rounds on it (16 disjoint rotations per round, the step's
//     rotation accumulated in registers in the solve's precision: FP32 in
//     the main sweeps, FP64 in the final sweep); wave 0 then rotates the
//     block between the two pairs with MFMA.  Step B likewise on the other
//     pairing.  It writes H[G, G] and M_G = J_A J_B.
//   * k_jac_apply: H[G1, G2] <- M_G1^T H[G1, G2] M_G2 for every pair of
//     groups and V[slab, G] <- V[slab, G] M_G for every 64-row slab of V, each
//     a 64 x 64 x 64 product pair on FP32 MFMA (32x32x2).
// Inner rounds.  Round t of a pair subproblem rotates local indices a and
// a ^ t: t < 16 pairs indices inside each 16-block, t >= 16 across the two
// blocks.  The first step of a sweep runs all 31 rounds, the others the 16
// cross rounds only, so every index pair is rotated once per sweep (a cyclic
// Jacobi ordering).
// Convergence is tested per matrix after each sweep, on the largest relative
// off-diagonal entry rotated and on the sum of squares of the rotated entries
// (normwise); converged matrices are skipped by later launches.
// Restarts.  Every block rotation rounds H and V separately, so after many
// sweeps V no longer diagonalises the input to FP32 accuracy (the backward
// error grows with the number of rotations, i.e. with n).  T = V^T H V is
// therefore re-formed from the input by two GEMMs and measured; if its
// off-diagonal part is too large, T is swept again from V' = I, whose
// rotations are small, and V <- V V'.
#include <algorithm>
#include <type_traits>
#include <cstring>
#include <vector>
#include "common.hpp"
#include "eigh.hpp"
#include "prof.hpp"

namespace {

constexpr int BS = 16;      // block width
constexpr int PB = 32;      // pair subproblem size
constexpr int GS = 64;      // group size (four blocks)
constexpr int LP = PB + 1;  // LDS pitch of 32-wide arrays
constexpr int GP = GS + 1;  // LDS pitch of 64-wide arrays
// per group: M_G (64 x 64, FP32)
constexpr int QSTRIDE = GS * GS;
// A restart sweeps T = V^T H V formed by FP32 GEMMs, resolved to about
// 2^-24 |H|_F: a pair whose 2 x 2 block (h_pp, h_qq, h_pq) lies entirely
// below that level is not rotated there.  Rotating such pairs only stirs a
// cluster of (near-)zero eigenvalues by large angles, which keeps re-filling
// its coupling to the other eigenvalues (the restart then converges
// linearly, not quadratically); pairs with a larger diagonal are rotated.
constexpr float kRestartSkip = 5.9604645e-8f;

SVDP_DEV int insert0(int x, int p) { return ((x >> p) << (p + 1)) | (x & ((1 << p) - 1)); }

// the four blocks of group gi in a phase, in local order
// [B0, B0 ^ sA, B0 ^ sB, B0 ^ sA ^ sB]: step A pairs local blocks (0, 1) and
// (2, 3), step B pairs (0, 2) and (1, 3).  B0 is the member with bits lo and
// hi clear (each group has exactly one).
SVDP_DEV void group_members(const EighPhase& ph, int gi, int* g) {
  const int b0 = insert0(insert0(gi, ph.lo), ph.hi);
  g[0] = b0;
  g[1] = b0 ^ ph.sA;
  g[2] = b0 ^ ph.sB;
  g[3] = b0 ^ ph.sA ^ ph.sB;
}

SVDP_DEV int64_t tile_off(int I, int J, int nb) { return ((int64_t)I * nb + J) * (BS * BS); }

// group rotations of phase slot `slot` of matrix b (nb / 4 groups of QSTRIDE floats)
SVDP_DEV float* qslot(const EighWs& e, int b, int slot) {
  return e.Qw + ((int64_t)b * e.nph_store + slot) * (e.nb / 4) * QSTRIDE;
}

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

SVDP_DEV f16v mfma(float a, float b, f16v acc) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0); }

SVDP_DEV f16v zero16() {
  f16v z;
#pragma unroll
  for (int i = 0; i < 16; ++i) z[i] = 0.f;
  return z;
}

template <typename R> struct RotPair { R c, s; };
template <typename R> struct XPitch { static constexpr int v = 66; };  // FP32: row stride 2 mod 32 banks
template <> struct XPitch<double> { static constexpr int v = 65; };

// position in the 64-index group of local index a (0..31) of pair w: step A
// pairs are contiguous halves, step B pairs interleave 16-blocks
template <int STEPB>
SVDP_DEV int gpos(int w, int a) {
  const int lo = STEPB ? 16 * w : 32 * w, hi = STEPB ? 32 + 16 * w : 32 * w + 16;
  return a < 16 ? lo + a : hi + (a - 16);
}

// The FP32 rotation with hardware rcp/sqrt/rsq and no branches: both cases
// of tau are computed and one is selected
SVDP_DEV void rotation_sel(float app, float aqq, float apq, float& c, float& s) {
  const float tau = (aqq - app) * __builtin_amdgcn_rcpf(2.f * apq);
  const float tl = 0.5f * __builtin_amdgcn_rcpf(tau);
  const float tn = copysignf(__builtin_amdgcn_rcpf(fabsf(tau) + __builtin_amdgcn_sqrtf(1.f + tau * tau)), tau);
  const float t = fabsf(tau) > 1e10f ? tl : tn;
  c = __builtin_amdgcn_rsqf(1.f + t * t);
  s = t * c;
}
SVDP_DEV void rotation_fast(double app, double aqq, double apq, double& c, double& s) {
  rotation(app, aqq, apq, c, s);
}

template <typename R>
struct SolveLds {
  R X[GS][XPitch<R>::v];    // H[G, G]
  float Jf[2][PB][LP];      // per-wave FP32 copy of the step's rotations
  RotPair<R> cs[2][16];     // per-wave (c, s) of the current round
};

// remove bit p of x
SVDP_DEV int compress(int x, int p) { return ((x >> (p + 1)) << p) | (x & ((1 << p) - 1)); }

template <typename T>
SVDP_DEV T lane_xor(T v, int lane, int m);
template <>
SVDP_DEV float lane_xor<float>(float v, int lane, int m) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute((lane ^ m) << 2, __float_as_int(v)));
}
template <>
SVDP_DEV double lane_xor<double>(double v, int lane, int m) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_ds_bpermute((lane ^ m) << 2, hi),
                          __builtin_amdgcn_ds_bpermute((lane ^ m) << 2, lo));
}

// DPP moves inside each row of 16 lanes (no LDS): quad_perm [1,0,3,2]
// (lane ^ 1), quad_perm [3,2,1,0] (^ 3), row_half_mirror (^ 7), row_mirror
// (^ 15)
template <int CTRL>
SVDP_DEV float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
SVDP_DEV double dpp_mov(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}
// v[u] <- v[u] of lane ^ d, for d = 2^k - 1 in {1, 3, 7, 15} (wave-uniform)
template <typename R>
SVDP_DEV void xor_row(R (&v)[8], int d) {
  if (d == 1) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = dpp_mov<0xB1>(v[u]);
  } else if (d == 3) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = dpp_mov<0x1B>(v[u]);
  } else if (d == 7) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = dpp_mov<0x141>(v[u]);
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = dpp_mov<0x140>(v[u]);
  }
}

// Scalar Jacobi rounds on pair w of the step (repeated inner_sweeps times):
// the rounds t0 .. 15 inside the two 16-blocks, then the 16 rounds across
// them.  One wavefront, no workgroup barrier.  Lane l (q = l / 16,
// kx = l % 16) updates, per round, the 2 x 2 blocks (rotation kx) x
// (rotations q + 4 u) of the subproblem, and holds rows q + 4 u of two
// columns of the accumulated rotation J in registers (jp, jq).
//   * Inside the blocks (round t < 16) a round rotates column pairs
//     (a, a ^ t): jp is column kx and jq column 16 + kx, and the partner
//     columns come from lane l ^ t by a register exchange.
//   * Across the blocks, round m = 0 .. 15 pairs index k with 16 + (k ^ m).
//     jq holds column 16 + (kx ^ m), so both columns of the lane's pair are
//     in the lane; between rounds jq moves to lane l ^ m ^ (m + 1), where
//     m ^ (m + 1) is 1, 3, 7 or 15: one DPP move inside the lane's row.
//     After the last round (m = 15) it moves back to column 16 + kx.
// A round issues all of its LDS traffic that does not depend on the round's
// rotations at once (the lane's four 2 x 2 blocks and, inside the blocks,
// the partner lanes' J entries).  The lane whose blocks include the
// diagonal block of rotation kx (q = kx mod 4, u = kx / 4) computes that
// rotation from it, so the only round trip that waits on another lane is the
// exchange of the 16 (c, s) pairs.
template <typename R, int STEPB>
SVDP_DEV void pair_solve(SolveLds<R>& L, int w, int lane, int t0, int inner_sweeps, R floor_abs, R skip_abs,
                         float& mrel, float& vsum, R (&jp)[8], R (&jq)[8]) {
  constexpr int XP = XPitch<R>::v;
  R (*X)[XP] = L.X;
  RotPair<R>* cs = L.cs[w];
  const int kx = lane & 15, q = lane >> 4;
  const bool rlane = q == (kx & 3);  // holds the diagonal block of rotation kx
  const int ud = kx >> 2;            // ... as its block ud
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    jp[u] = (q + 4 * u == kx) ? R(1) : R(0);
    jq[u] = (q + 4 * u == 16 + kx) ? R(1) : R(0);
  }
  // One round t.  CROSS (t >= 16) pairs index k of the first 16-block with
  // 16 + (k ^ (t - 16)); otherwise indices inside each 16-block are paired.
  // The two kinds are separate instantiations, so their index maps are
  // resolved at compile time.
  auto round = [&](auto cross_c, int t, int& any) {
    constexpr bool CROSS = decltype(cross_c)::value;
    const int hb = 31 - __builtin_clz(t);
    auto pair_of = [&](int k, int& x, int& y) {
      x = CROSS ? k : (((k >> 3) << 4) | insert0(k & 7, hb));
      y = x ^ t;
    };
    int x1, y1;
    pair_of(kx, x1, y1);
    R* rowx = X[gpos<STEPB>(w, x1)];
    R* rowy = X[gpos<STEPB>(w, y1)];
    // the lane's four 2 x 2 blocks are disjoint from every other lane's:
    // all loads first, then all stores (one LDS round trip)
    int cx[4], cy[4];
    R a[4], bq[4], cq[4], d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int x2, y2;
      pair_of(q + 4 * u, x2, y2);
      cx[u] = gpos<STEPB>(w, x2);
      cy[u] = gpos<STEPB>(w, y2);
      a[u] = rowx[cx[u]]; bq[u] = rowx[cy[u]]; cq[u] = rowy[cx[u]]; d[u] = rowy[cy[u]];
    }
    // inside the blocks: the partner lane's J entries, columns kx ^ t (op)
    // and 16 + (kx ^ t) (oq)
    R op[8], oq[8];
    if (!CROSS) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        op[u] = lane_xor<R>(jp[u], lane, t);
        oq[u] = lane_xor<R>(jq[u], lane, t);
      }
    }
    if (rlane) {
      R app = a[0], aqq = d[0], bd = bq[0], cd = cq[0];
#pragma unroll
      for (int u = 1; u < 4; ++u) {
        const bool sel = ud == u;  // selects, not a branch per block
        app = sel ? a[u] : app;
        aqq = sel ? d[u] : aqq;
        bd = sel ? bq[u] : bd;
        cd = sel ? cq[u] : cd;
      }
      const R apq = R(0.5) * (bd + cd);
      RotPair<R> r{R(1), R(0)};
      const bool rot =
          apq != R(0) && isfinite((float)apq) && fmax(fmax(fabs(app), fabs(aqq)), fabs(apq)) > skip_abs;
      // |apq| / sqrt(|app aqq|), a convergence statistic (no IEEE rounding needed)
      const float den2 = fabsf((float)app * (float)aqq);
      const float rel = den2 > 0.f ? fabsf((float)apq) * __builtin_amdgcn_rsqf(den2) : 1e30f;
      if constexpr (sizeof(R) == 4) {
        // straight-line code on the round's critical path: the rotation is
        // computed whatever the tests say and selected
        float c, sn;
        rotation_sel(app, aqq, apq, c, sn);
        r.c = rot ? c : 1.f;
        r.s = rot ? sn : 0.f;
        any |= rot ? 1 : 0;
        vsum += rot ? apq * apq : 0.f;
        mrel = rot && fabsf(apq) > floor_abs ? fmaxf(mrel, rel) : mrel;
      } else if (rot) {
        rotation_fast(app, aqq, apq, r.c, r.s);
        any = 1;
        vsum += (float)apq * (float)apq;
        if (fabs(apq) > floor_abs) mrel = fmaxf(mrel, rel);
      }
      cs[kx] = r;
    }
    wave_sync();
    const RotPair<R> r1 = cs[kx];
    RotPair<R> r2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) r2[u] = cs[q + 4 * u];
    // inside the blocks, the rotations of the lane's two J columns: column
    // kx pairs with the partner's kx ^ t, column 16 + kx with 16 + (kx ^ t).
    // A column that is the first of its pair becomes c x - s y, the second
    // c x + s y: the sign goes into s once per round.
    RotPair<R> rp{}, rq{};
    R sp{}, sq{};
    if (!CROSS) {
      const bool first = ((kx >> hb) & 1) == 0;
      const int xs = first ? kx : kx ^ t;
      rp = cs[compress(xs, hb)];
      rq = cs[8 + compress(xs, hb)];
      sp = first ? -rp.s : rp.s;
      sq = first ? -rq.s : rq.s;
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const R t00 = r1.c * a[u] - r1.s * cq[u], t01 = r1.c * bq[u] - r1.s * d[u];
      const R t10 = r1.s * a[u] + r1.c * cq[u], t11 = r1.s * bq[u] + r1.c * d[u];
      R y00 = r2[u].c * t00 - r2[u].s * t01, y01 = r2[u].s * t00 + r2[u].c * t01;
      R y10 = r2[u].c * t10 - r2[u].s * t11, y11 = r2[u].s * t10 + r2[u].c * t11;
      if (kx == q + 4 * u && r1.s != R(0)) { y01 = 0; y10 = 0; }
      rowx[cx[u]] = y00; rowx[cy[u]] = y01; rowy[cx[u]] = y10; rowy[cy[u]] = y11;
    }
    if (CROSS) {
      // the pair (kx, 16 + (kx ^ m)): jp = c jp - s jq, jq = s jp + c jq
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const R p = jp[u], qv = jq[u];
        jp[u] = r1.c * p - r1.s * qv;
        jq[u] = r1.s * p + r1.c * qv;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        jp[u] = rp.c * jp[u] + sp * op[u];
        jq[u] = rq.c * jq[u] + sq * oq[u];
      }
    }
    wave_sync();
  };
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    int any = 0;
    for (int t = t0; t < 16; ++t) round(std::false_type{}, t, any);
    for (int m = 0; m < 16; ++m) {
      if (m > 0) xor_row(jq, m ^ (m - 1));
      round(std::true_type{}, 16 + m, any);
    }
    xor_row(jq, 15);
    // every lane of the wave takes the same exit
    if (!__any(any)) break;
  }
}

// the step's rotations (registers) -> wave w's FP32 LDS copy
template <typename R>
SVDP_DEV void j_to_lds(SolveLds<R>& L, int w, int lane, const R (&jp)[8], const R (&jq)[8]) {
  const int kx = lane & 15, q = lane >> 4;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    L.Jf[w][q + 4 * u][kx] = (float)jp[u];
    L.Jf[w][q + 4 * u][16 + kx] = (float)jq[u];
  }
  wave_sync();
}

// The block of H[G, G] between the two pairs of a step, B = X[P0, P1]:
// B <- J0^T B J1, and its mirror X[P1, P0] = B^T.  One wavefront.
template <typename R, int STEPB>
SVDP_DEV void cross_update(SolveLds<R>& L, const float (*J0)[LP], const float (*J1)[LP], int lane) {
  constexpr int XP = XPitch<R>::v;
  R (*X)[XP] = L.X;
  const int kh = lane >> 5, ic = lane & 31;
  f16v acc = zero16();
#pragma unroll 4
  for (int kk = 0; kk < PB; kk += 2)
    acc = mfma(J0[kk + kh][ic], (float)X[gpos<STEPB>(0, kk + kh)][gpos<STEPB>(1, ic)], acc);
  wave_sync();
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) X[gpos<STEPB>(0, 8 * g + 4 * kh + r)][gpos<STEPB>(1, ic)] = (R)acc[4 * g + r];
  wave_sync();
  acc = zero16();
#pragma unroll 4
  for (int kk = 0; kk < PB; kk += 2)
    acc = mfma((float)X[gpos<STEPB>(0, ic)][gpos<STEPB>(1, kk + kh)], J1[kk + kh][ic], acc);
  wave_sync();
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = gpos<STEPB>(0, 8 * g + 4 * kh + r), j = gpos<STEPB>(1, ic);
      X[i][j] = (R)acc[4 * g + r];
      X[j][i] = (R)acc[4 * g + r];
    }
  wave_sync();
}

template <typename R>
__global__ __launch_bounds__(128) void k_jac_solve(EighWs e, EighPhase ph, int inner_sweeps, float abs_tol,
                                                   float skip_rel, int* rotmax, float* rotsq) {
  __shared__ SolveLds<R> L;
  constexpr int XP = XPitch<R>::v;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int ng = e.nb / 4;
  const int b = blockIdx.x / ng, gi = blockIdx.x - b * ng;
  if (b >= e.batch) return;
  if (e.active && !e.active[b]) return;
  if (e.work && t == 0) {
    // algorithmic flops: per pair subproblem and round, 256 two-sided 2 x 2
    // block updates (24 flops each) and 512 rotation-accumulator pairs (6)
    const int rounds = (ph.fullA ? 31 : 16) + (ph.skipB ? 0 : 16);
    atomicAdd(e.work + (sizeof(R) == 8 ? PROF_JAC_SOLVE_F64 : PROF_JAC_SOLVE_F32),
              2.0 * rounds * inner_sweeps * (256.0 * 24.0 + 512.0 * 6.0));
  }
  int g[4];
  group_members(ph, gi, g);
  float* H = e.Hw + (int64_t)b * e.np * e.np;
  // H[G, G]: 16 tiles, the ones below the diagonal read transposed; all
  // eight of a thread's loads are issued before its first LDS store
  f4v hv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int idx = t + 128 * u, tile = idx >> 6, qd = idx & 63, k1 = tile >> 2, k2 = tile & 3;
    const int I = g[k1], Jb = g[k2];
    hv[u] = *(const f4v*)(H + tile_off(I > Jb ? Jb : I, I > Jb ? I : Jb, e.nb) + qd * 4);
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int idx = t + 128 * u, tile = idx >> 6, qd = idx & 63, k1 = tile >> 2, k2 = tile & 3;
    const bool tr = g[k1] > g[k2];
    const int r = qd >> 2, c = (qd & 3) * 4;
#pragma unroll
    for (int w2 = 0; w2 < 4; ++w2) {
      // a tile below the diagonal is stored transposed (addresses selected,
      // not branched on)
      const int row = k1 * 16 + (tr ? c + w2 : r), col = k2 * 16 + (tr ? r : c + w2);
      L.X[row][col] = (R)hv[u][w2];
    }
  }
  __syncthreads();
  const R floor_abs = (R)abs_tol * (R)sqrtf(e.hnorm2[b]);
  // a pair whose 2 x 2 block lies entirely at or below skip_abs is not rotated
  const R skip_abs = (R)skip_rel * (R)sqrtf(e.hnorm2[b]);
  float mrel = 0.f, vsum = 0.f;
  float* M = qslot(e, b, e.deferred ? ph.idx : 0) + (int64_t)gi * QSTRIDE;
  R jp[8], jq[8];
  // step A
  pair_solve<R, 0>(L, w, lane, ph.fullA ? 1 : 16, inner_sweeps, floor_abs, skip_abs, mrel, vsum, jp, jq);
  j_to_lds(L, w, lane, jp, jq);
  __syncthreads();
  if (w == 0) cross_update<R, 0>(L, L.Jf[0], L.Jf[1], lane);
  __syncthreads();
  const int kh = lane >> 5, ic = lane & 31;
  // the step-A rotations (FP32, the lane's entries as in j_to_lds), kept in
  // registers through step B for M_G = J_A J_B
  float ja[8], jb[8];
  if (!ph.skipB) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      ja[u] = (float)jp[u];
      jb[u] = (float)jq[u];
    }
    // step B
    pair_solve<R, 1>(L, w, lane, 16, inner_sweeps, floor_abs, skip_abs, mrel, vsum, jp, jq);
    j_to_lds(L, w, lane, jp, jq);
    __syncthreads();
    if (w == 0) cross_update<R, 1>(L, L.Jf[0], L.Jf[1], lane);
    __syncthreads();
  }
  // H[G, G] back: the tiles on and above the diagonal
  for (int idx = t; idx < 16 * 64; idx += 128) {
    const int tile = idx >> 6, qd = idx & 63, k1 = tile >> 2, k2 = tile & 3;
    if (g[k1] > g[k2]) continue;
    const int r = qd >> 2, c = (qd & 3) * 4;
    f4v v;
#pragma unroll
    for (int w2 = 0; w2 < 4; ++w2) v[w2] = (float)L.X[k1 * 16 + r][k2 * 16 + c + w2];
    *(f4v*)(H + tile_off(g[k1], g[k2], e.nb) + qd * 4) = v;
  }
  if (ph.skipB) {
    // M_G = J_A (block diagonal)
    for (int idx = t; idx < GS * GS; idx += 128) {
      const int p = idx >> 6, qq = idx & 63;
      M[idx] = (p >> 5) == (qq >> 5) ? L.Jf[p >> 5][p & 31][qq & 31] : 0.f;
    }
  } else {
    // J_A into the space of H[G, G], which has been written back
    static_assert(sizeof(L.X) >= 2 * PB * LP * sizeof(float), "J_A fits in the space of H[G, G]");
    __syncthreads();
    float (*JA)[PB][LP] = reinterpret_cast<float (*)[PB][LP]>(&L.X[0][0]);
    {
      const int kx = lane & 15, q = lane >> 4;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        JA[w][q + 4 * u][kx] = ja[u];
        JA[w][q + 4 * u][16 + kx] = jb[u];
      }
    }
    __syncthreads();
    // M_G = J_A J_B, block (wa, wb): rows of step-A pair wa, columns of
    // step-B pair wb; the shared indices are local 32 wa + 16 wb + k, k < 16
    for (int blk = w; blk < 4; blk += 2) {
      const int wa = blk >> 1, wb = blk & 1;
      f16v acc = zero16();
#pragma unroll
      for (int kk = 0; kk < 16; kk += 2)
        acc = mfma(JA[wa][ic][16 * wb + kk + kh], L.Jf[wb][16 * wa + kk + kh][ic], acc);
#pragma unroll
      for (int gg = 0; gg < 4; ++gg)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          M[(32 * wa + 8 * gg + 4 * kh + r) * GS + gpos<1>(wb, ic)] = acc[4 * gg + r];
    }
  }
  // largest relative off-diagonal entry rotated by this wave (float bits),
  // and the sum of squares of the entries it rotated
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mrel = fmaxf(mrel, __shfl_xor(mrel, off));
    vsum += __shfl_xor(vsum, off);
  }
  if (lane == 0 && rotmax) atomicMax(rotmax + b, __float_as_int(mrel));
  // the rotated mass goes to this group's and wave's slot of the sweep (its
  // only writer in every phase), added in slot order by k_eigh_check
  if (lane == 0 && rotsq) rotsq[((int64_t)b * ng + gi) * 2 + w] += vsum;
}

// 64 x 64 quadrant products on one wavefront (32 x 32 output block (qi, qj)),
// K = 64 in 32 MFMA steps.  MFMA operand layout (32x32x2 f32): lane l
// supplies A[l % 32][k] and B[k][l % 32]; the accumulator's slot 4 g + r is
// row 8 g + 4 (l / 32) + r, column l % 32.  Step s contracts index
// s + 32 (l / 32) (a permutation of the 64 indices, the same for both
// operands), so a lane's steps 4 j .. 4 j + 3 read four consecutive entries
// of an LDS row: one 16-byte read (row pitch AP = 68: eight rows start in
// 32 different banks) feeds four MFMAs.
constexpr int AP = GS + 4;
// acc[i][j] = sum_k a_k[i] B[k][32 qj + j] with B given transposed in LDS
// (Bt[j][k] = B[k][j]); the left factor's operands in registers (a[s] for
// k = s + 32 (lane / 32))
SVDP_DEV f16v mm_rl(const float (&a)[32], const float (*Bt)[AP], int qj, int lane) {
  const int kh = lane >> 5, ic = lane & 31;
  const float* row = Bt[32 * qj + ic] + 32 * kh;
  f16v acc = zero16();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const f4v v = *(const f4v*)(row + 4 * j);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = mfma(a[4 * j + u], v[u], acc);
  }
  return acc;
}
// acc[i][j] = sum_k A[32 qi + i][k] b_k[j]: the left factor from LDS (row
// major), the right factor's operands in registers
SVDP_DEV f16v mm_lr(const float (*A)[AP], const float (&b)[32], int qi, int lane) {
  const int kh = lane >> 5, ic = lane & 31;
  const float* row = A[32 * qi + ic] + 32 * kh;
  f16v acc = zero16();
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const f4v v = *(const f4v*)(row + 4 * j);
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = mfma(v[u], b[4 * j + u], acc);
  }
  return acc;
}
SVDP_DEV void put_quadrant(float (*X)[AP], const f16v& acc, int qi, int qj, int lane) {
  const int kh = lane >> 5, ic = lane & 31;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) X[32 * qi + 8 * g + 4 * kh + r][32 * qj + ic] = acc[4 * g + r];
}
// rows s + 32 (lane / 32) of column c0 + (lane % 32) of a 64 x 64 row-major M
SVDP_DEV void load_mcol(const float* M, int c0, int lane, float (&v)[32]) {
  const int kh = lane >> 5, ic = lane & 31;
  const float* p = M + 32 * kh * GS + c0 + ic;
#pragma unroll
  for (int s2 = 0; s2 < 32; ++s2) v[s2] = p[s2 * GS];
}

// One workgroup (four wavefronts, wave w owns output quadrant (w / 2, w % 2))
// per task.  The 64 x 64 data block goes through LDS; the group rotations
// (small, shared by many tasks of the matrix, L2-resident) are read straight
// into MFMA operand registers.  An H task holds X transposed for M1^T X,
// then the intermediate row-major for (M1^T X) M2; a V task holds X
// row-major for X M.
__global__ __launch_bounds__(256) void k_jac_apply(EighWs e, EighPhase ph) {
  __shared__ __attribute__((aligned(16))) float Xs[GS][AP];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int ng = e.nb / 4;
  const int nH = ng * (ng - 1) / 2;
  // with V deferred to the end of the sweep only the H tasks run here
  const int ntask = e.deferred ? nH : nH + ng * ng;
  // matrix b runs on XCD b % 8: its group rotations stay in one L2
  const int L = blockIdx.x, x8 = L & 7, q = L >> 3;
  const int grp = q / ntask, task = q - grp * ntask;
  const int b = grp * 8 + x8;
  if (b >= e.batch) return;
  if (e.active && !e.active[b]) return;
  const int qi = w >> 1, qj = w & 1;
  const float* Qb = qslot(e, b, e.deferred ? ph.idx : 0);
  // algorithmic flops: two 64^3 products per H task, one per V task
  if (e.work && t == 0) atomicAdd(e.work + PROF_JAC_APPLY, (task < nH ? 4.0 : 2.0) * GS * GS * GS);
  if (task < nH) {
    int tt = task, G1 = 0;
    while (tt >= ng - 1 - G1) { tt -= ng - 1 - G1; ++G1; }
    const int G2 = G1 + 1 + tt;
    int g1[4], g2[4];
    group_members(ph, G1, g1);
    group_members(ph, G2, g2);
    float* H = e.Hw + (int64_t)b * e.np * e.np;
    // X = H[G1, G2] from the upper tiles.  A wave moves four 1 KB tiles; lane
    // l takes each tile's 16-byte chunk at row r = l % 16, columns c .. c + 3
    // with c = 4 (l / 16), so each group of 16 lanes covers 16 rows of one
    // column chunk: its 16-byte LDS stores (a transposed stored tile) start 4
    // banks apart and its 4-byte stores land in 64 distinct banks.  All four
    // loads are issued before the rotations' loads and before any store, so
    // their round trips overlap.
    const int r = lane & 15, c = (lane >> 4) * 4;
    f4v xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tile = w + 4 * u, k1 = tile >> 2, k2 = tile & 3;
      const int I = g1[k1], Jb = g2[k2];
      xv[u] = *(const f4v*)(H + tile_off(I > Jb ? Jb : I, I > Jb ? I : Jb, e.nb) + r * 16 + c);
    }
    // T = M1^T X needs M1[k][32 qi + i]; Y = T M2 needs M2[k][32 qj + j]
    float a1[32], b2[32];
    load_mcol(Qb + (int64_t)G1 * QSTRIDE, 32 * qi, lane, a1);
    load_mcol(Qb + (int64_t)G2 * QSTRIDE, 32 * qj, lane, b2);
    // X^T into LDS: Xs[c][r] = X[r][c]
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tile = w + 4 * u, k1 = tile >> 2, k2 = tile & 3;
      const bool tr = g1[k1] > g2[k2];
      const f4v v = xv[u];
      if (tr) {
        // the stored tile is X's block transposed: row r of it is column r of X
        *(f4v*)&Xs[k2 * 16 + r][k1 * 16 + c] = v;
      } else {
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) Xs[k2 * 16 + c + w2][k1 * 16 + r] = v[w2];
      }
    }
    __syncthreads();
    const f16v T = mm_rl(a1, Xs, qj, lane);  // M1^T X
    __syncthreads();
    put_quadrant(Xs, T, qi, qj, lane);
    __syncthreads();
    const f16v Y = mm_lr(Xs, b2, qi, lane);  // (M1^T X) M2
    __syncthreads();
    put_quadrant(Xs, Y, qi, qj, lane);
    __syncthreads();
    // back to the upper tiles, the same lane-to-chunk map: an untransposed
    // tile's chunk is one 16-byte LDS read
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int tile = w + 4 * u, k1 = tile >> 2, k2 = tile & 3;
      const int I = g1[k1], Jb = g2[k2];
      const bool tr = I > Jb;
      f4v v;
      if (tr) {
#pragma unroll
        for (int w2 = 0; w2 < 4; ++w2) v[w2] = Xs[k1 * 16 + c + w2][k2 * 16 + r];
      } else {
        v = *(const f4v*)&Xs[k1 * 16 + r][k2 * 16 + c];
      }
      *(f4v*)(H + tile_off(tr ? Jb : I, tr ? I : Jb, e.nb) + r * 16 + c) = v;
    }
  } else {
    const int v = task - nH, slab = v / ng, G = v - slab * ng;
    int gm[4];
    group_members(ph, G, gm);
    float* V = e.Vw + (int64_t)b * e.np * e.np;
    float bm[32];
    load_mcol(Qb + (int64_t)G * QSTRIDE, 32 * qj, lane, bm);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = t + 256 * u;
      const int tile = idx >> 6, qd = idx & 63, k1 = tile >> 2, k2 = tile & 3;
      const f4v x = *(const f4v*)(V + tile_off(4 * slab + k1, gm[k2], e.nb) + qd * 4);
      const int r = qd >> 2, c = (qd & 3) * 4;
      *(f4v*)&Xs[k1 * 16 + r][k2 * 16 + c] = x;
    }
    __syncthreads();
    const f16v Y = mm_lr(Xs, bm, qi, lane);  // X M
    __syncthreads();
    put_quadrant(Xs, Y, qi, qj, lane);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = t + 256 * u;
      const int tile = idx >> 6, qd = idx & 63, k1 = tile >> 2, k2 = tile & 3;
      const int r = qd >> 2, c = (qd & 3) * 4;
      *(f4v*)(V + tile_off(4 * slab + k1, gm[k2], e.nb) + qd * 4) = *(const f4v*)&Xs[k1 * 16 + r][k2 * 16 + c];
    }
  }
}

// Deferred V update: V[slab, :] <- V[slab, :] M_1 M_2 ... M_P with the group
// rotations of every phase of the sweep (block diagonal in that phase's
// grouping, one 64 x 64 orthogonal M per group of four blocks).  One
// workgroup of eight wavefronts per slab of R rows of one matrix (R = 64 up
// to NP = 512, 32 at NP = 1024: the slab takes about 128 KB of LDS); the
// slab stays in LDS for the whole sweep and the rotations are read from L2
// straight into MFMA operand registers.  A phase runs over sets of GPS
// groups (groups touch disjoint columns): wave w takes the column half
// w % 2 of group w / 2 of the set, i.e. a 64 x 32 slice of that group's M,
// and multiplies every 32-row block of the slab by it (R / 32 independent
// MFMA chains on the same operands); all waves have read the set's input
// columns at the first barrier and written their outputs at the second.
// The contraction index of MFMA step s is s + 32 (lane / 32) (any order of
// the 64 indices gives the same product), so a lane's steps 4 j .. 4 j + 3
// read four consecutive slab columns: one 16-byte LDS read (row pitch
// NP + 4: eight rows start in 32 different banks) feeds four MFMAs.  The
// next set's slice is loaded during the current set's MFMAs.  Matrices that
// were not active in the sweep are skipped (their rotation slots hold an
// earlier sweep's).
template <int NP, int R>
__global__ __launch_bounds__(512) void k_jac_vsweep(EighWs e) {
  constexpr int PITCH = NP + 4;
  constexpr int NBK = NP / BS, NG = NBK / 4, NPH = NBK / 2;
  constexpr int GPS = NG < 4 ? NG : 4;  // groups per set: 2 GPS <= 8 slices, one per wave
  constexpr int NSET = NG / GPS;
  constexpr int RB = R / 32;            // 32-row blocks of the slab
  constexpr int SLABS = NP / R;
  __shared__ __attribute__((aligned(16))) float Vs[R * PITCH];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  // matrix b on XCD b % 8: its rotations are read into one L2
  const int L = blockIdx.x, x8 = L & 7, q = L >> 3;
  const int grp = q / SLABS, slab = q - grp * SLABS;
  const int b = grp * 8 + x8;
  if (b >= e.batch) return;
  if (e.active && !e.active[b]) return;
  float* V = e.Vw + (int64_t)b * NP * NP + (int64_t)slab * R * NP;
  if (e.work && t == 0) atomicAdd(e.work + PROF_JAC_VSWEEP, (double)NPH * NG * 2.0 * R * GS * GS);
  // the slab into LDS, up to eight 16-byte loads in flight per thread
  constexpr int PER = R * NP / 4 / 512, NBT = PER < 8 ? PER : 8;
  static_assert(PER % NBT == 0, "slab load batches");
  for (int i0 = t; i0 < R * NP / 4; i0 += 512 * NBT) {
    f4v tmp[NBT];
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
      const int idx = i0 + 512 * u, r = idx / (NP / 4), c = (idx - r * (NP / 4)) * 4;
      tmp[u] = *(const f4v*)(V + (int64_t)r * NP + c);
    }
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
      const int idx = i0 + 512 * u, r = idx / (NP / 4), c = (idx - r * (NP / 4)) * 4;
      *(f4v*)(Vs + r * PITCH + c) = tmp[u];
    }
  }
  __syncthreads();
  const int kh = lane >> 5, ic = lane & 31;
  const bool busy = w < 2 * GPS;  // waves beyond the set's slices idle (NG < 4)
  const int ch = w & 1;
  float cur[32], nxt[32];
  // B operands of the slice: rows s + 32 kh of column 32 ch + ic of M
  auto load_slice = [&](int p, int set, float (&bm)[32]) {
    if (!busy) return;
    const float* M = qslot(e, b, p) + (int64_t)(set * GPS + (w >> 1)) * QSTRIDE + 32 * kh * GS + 32 * ch + ic;
#pragma unroll
    for (int s2 = 0; s2 < 32; ++s2) bm[s2] = M[s2 * GS];
  };
  load_slice(0, 0, cur);
  for (int p = 0; p < NPH; ++p) {
    const EighPhase ph = eigh_phase(p);
    // the sets of a phase rotate disjoint column groups: all of them are
    // computed from the slab before one barrier, then written before another
    f16v acc[NSET][RB];
    int gsel[NSET];  // member block of the output column 32 ch + ic, per set
#pragma unroll
    for (int set = 0; set < NSET; ++set) {
      if (set + 1 < NSET) load_slice(p, set + 1, nxt);
      else if (p + 1 < NPH) load_slice(p + 1, 0, nxt);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[set][rb] = zero16();
      int gm[4];
      group_members(ph, set * GPS + (w >> 1), gm);
      // selected, not indexed: gm stays in registers
      const int mb = 2 * ch + (ic >> 4);
      gsel[set] = mb == 0 ? gm[0] : (mb == 1 ? gm[1] : (mb == 2 ? gm[2] : gm[3]));
      if (busy) {
        // contraction index s2 + 32 kh lies in member block 2 kh + s2 / 16
        const int blk0 = kh ? gm[2] : gm[0], blk1 = kh ? gm[3] : gm[1];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int col = 16 * (j < 4 ? blk0 : blk1) + 4 * (j & 3);
          f4v a[RB];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) a[rb] = *(const f4v*)(Vs + (32 * rb + ic) * PITCH + col);
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[set][rb] = mfma(a[rb][u], cur[4 * j + u], acc[set][rb]);
        }
      }
#pragma unroll
      for (int k = 0; k < 32; ++k) cur[k] = nxt[k];
    }
    __syncthreads();
    if (busy) {
#pragma unroll
      for (int set = 0; set < NSET; ++set) {
        const int col = 16 * gsel[set] + (ic & 15);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int g4 = 0; g4 < 4; ++g4)
#pragma unroll
            for (int r4 = 0; r4 < 4; ++r4)
              Vs[(32 * rb + 8 * g4 + 4 * kh + r4) * PITCH + col] = acc[set][rb][4 * g4 + r4];
      }
    }
    __syncthreads();
  }
  for (int idx = t; idx < R * NP / 4; idx += 512) {
    const int r = idx / (NP / 4), c = (idx - r * (NP / 4)) * 4;
    *(f4v*)(V + (int64_t)r * NP + c) = *(const f4v*)(Vs + r * PITCH + c);
  }
}

// what k_eigh_setup writes: V = I (tiled), the upper tiles of sym(H), |H|_F^2
constexpr int kSetupV = 1, kSetupH = 2, kSetupNorm = 4;

// Tiled working copies: H (tiles on and above the diagonal, symmetrised,
// zero padding), V = I, |H|_F^2.  One 64 x 64 block (Ib, Jb) of tiles per
// workgroup: the block and its mirror are read row-contiguous into LDS.
__global__ __launch_bounds__(256) void k_eigh_setup(EighWs e, const float* Hin, int64_t ldh, int64_t sH,
                                                    const int* mask, int what) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  __shared__ float Ablk[GS][GP];
  __shared__ float Tblk[GS][GP];
  const int nq = e.nb / 4;
  const int Ib = blockIdx.x / nq, Jb = blockIdx.x - Ib * nq;
  const int t = threadIdx.x;
  float* Vb = e.Vw + (int64_t)b * e.np * e.np;
  if (what & kSetupV)
    for (int idx = t; idx < 16 * 64; idx += 256) {
      const int tile = idx >> 6, qd = idx & 63, I = 4 * Ib + (tile >> 2), J = 4 * Jb + (tile & 3);
      const int r = qd >> 2, c = (qd & 3) * 4;
      f4v v;
#pragma unroll
      for (int w2 = 0; w2 < 4; ++w2) v[w2] = (I == J && r == c + w2) ? 1.f : 0.f;
      // deferred V is row-major, otherwise tiled
      const int64_t off = e.deferred ? (int64_t)(16 * I + r) * e.np + 16 * J + c : tile_off(I, J, e.nb) + qd * 4;
      *(f4v*)(Vb + off) = v;
    }
  if (!(what & kSetupH) || Ib > Jb) return;  // whole workgroup: H keeps the upper tiles only
  const float* Hb = Hin + b * sH;
  for (int idx = t; idx < GS * GS; idx += 256) {
    const int r = idx >> 6, c = idx & 63;
    const int i = GS * Ib + r, j = GS * Jb + c;
    Ablk[r][c] = (i < e.n && j < e.n) ? Hb[(int64_t)i * ldh + j] : 0.f;
    const int i2 = GS * Jb + r, j2 = GS * Ib + c;
    Tblk[r][c] = (i2 < e.n && j2 < e.n) ? Hb[(int64_t)i2 * ldh + j2] : 0.f;
  }
  __syncthreads();
  float* Hw = e.Hw + (int64_t)b * e.np * e.np;
  float acc = 0.f;
  for (int idx = t; idx < 16 * 64; idx += 256) {
    const int tile = idx >> 6, qd = idx & 63, k1 = tile >> 2, k2 = tile & 3;
    const int I = 4 * Ib + k1, J = 4 * Jb + k2;
    if (I > J) continue;  // below the diagonal of a diagonal block
    const int r = qd >> 2, c = (qd & 3) * 4;
    f4v v;
#pragma unroll
    for (int w2 = 0; w2 < 4; ++w2) {
      const int rr = 16 * k1 + r, cc = 16 * k2 + c + w2;
      v[w2] = 0.5f * (Ablk[rr][cc] + Tblk[cc][rr]);
      acc += v[w2] * v[w2] * (I == J ? 1.f : 2.f);
    }
    *(f4v*)(Hw + tile_off(I, J, e.nb) + qd * 4) = v;
  }
  if (!(what & kSetupNorm)) return;
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((t & 63) == 0) e.hn_part[((int64_t)b * nq * nq + blockIdx.x) * 4 + (t >> 6)] = acc;
}

// |H|_F^2 = the setup workgroups' partial sums (blocks Ib <= Jb) in block order
__global__ void k_hnorm_finalize(EighWs e, const int* mask) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= e.batch || (mask && !mask[b])) return;
  const int nq = e.nb / 4;
  float t = 0.f;
  for (int Ib = 0; Ib < nq; ++Ib)
    for (int Jb = Ib; Jb < nq; ++Jb)
      for (int w = 0; w < 4; ++w) t += e.hn_part[((int64_t)b * nq * nq + Ib * nq + Jb) * 4 + w];
  e.hnorm2[b] = t;
}

// row-major copy of a tiled np x np matrix: one row per workgroup, a float4
// per thread and step
__global__ void k_untile(const float* src, float* dst, int np, int nb, const int* mask) {
  const int b = blockIdx.y;
  if (mask && !mask[b]) return;
  const int row = blockIdx.x;
  const int64_t off = (int64_t)b * np * np;
  for (int c4 = 4 * threadIdx.x; c4 < np; c4 += 4 * blockDim.x) {
    const f4v v = *(const f4v*)(src + off + tile_off(row >> 4, c4 >> 4, nb) + (row & 15) * BS + (c4 & 15));
    *(f4v*)(dst + off + (int64_t)row * np + c4) = v;
  }
}

// Mark matrices as converged after a sweep whose largest rotated relative
// entry was <= tol, or whose rotated entries had a sum of squares <=
// fro_tol2 |H|_F^2 (a normwise test: the next sweep leaves far less), and
// count the ones still active (single workgroup).
__global__ void k_eigh_check(EighWs e, const int* rotcnt, float* rotsq, float tol, float fro_tol2, int sweep,
                             int* sweeps_out, int* n_active) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  const int slots = (e.nb / 4) * 2;
  for (int b = threadIdx.x; b < e.batch; b += blockDim.x) {
    float* rs = rotsq + (int64_t)b * slots;
    float vs = 0.f;
    for (int q = 0; q < slots; ++q) {
      vs += rs[q];
      rs[q] = 0.f;
    }
    if (e.active[b]) {
      sweeps_out[b] = sweep + 1;
      if (__int_as_float(rotcnt[b]) <= tol || vs <= fro_tol2 * e.hnorm2[b]) e.active[b] = 0;
      else ++mine;
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

// Restart measure of T = V^T H0 V (row-major, leading dimension np) for the
// matrices of `proc`.  H0 may be unsymmetric (H = W^T A); the measure uses
// the symmetric part S = (T + T^T) / 2: off2[b] += sum_{i != j} S_ij^2 (FP64)
// over the 32 x 32 tile pairs (I <= J) this workgroup takes, and the
// diagonal tiles give lamr = diag(T), the Rayleigh quotients of V's columns.
__global__ __launch_bounds__(256) void k_restart_offnorm(EighWs e, const float* T, const int* proc) {
  const int b = blockIdx.y;
  if (proc && !proc[b]) return;
  __shared__ float X[32][33], Y[32][33];
  __shared__ double red[4];
  const int n = e.n, nt = (n + 31) / 32, npairs = nt * (nt + 1) / 2;
  const float* Tb = T + (int64_t)b * e.np * e.np;
  const int t = threadIdx.x, r = t >> 3, c0 = (t & 7) * 4;
  double acc = 0.0;
  for (int p = blockIdx.x; p < npairs; p += gridDim.x) {
    int I = 0, rem = p;  // p -> (I, J), I <= J, row by row over the upper triangle
    while (rem >= nt - I) { rem -= nt - I; ++I; }
    const int J = I + rem;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = c0 + w;
      const int i1 = 32 * I + r, j1 = 32 * J + c, i2 = 32 * J + r, j2 = 32 * I + c;
      X[r][c] = (i1 < n && j1 < n) ? Tb[(int64_t)i1 * e.np + j1] : 0.f;
      Y[r][c] = (i2 < n && j2 < n) ? Tb[(int64_t)i2 * e.np + j2] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int c = c0 + w;
      const double sv = 0.5 * ((double)X[r][c] + (double)Y[c][r]);
      if (I != J) acc += 2.0 * sv * sv;
      else if (r != c) acc += sv * sv;
      else if (32 * I + r < n) e.lamr[(int64_t)b * n + 32 * I + r] = X[r][c];
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((t & 63) == 0) red[t >> 6] = acc;
  __syncthreads();
  if (t == 0) e.off_part[(int64_t)b * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// After a restart measure: a matrix of `proc` stays active for another sweep
// of T when off2 > off_tol2 |H0|_F^2 and `last` is 0 (the others leave the
// active set); *counter gains the number of active matrices, and their sweep
// counts the nsweeps sweeps of the restart.
__global__ void k_restart_decide(EighWs e, const int* proc, int chunks, float off_tol2, int last, int* counter,
                                 int* sweeps_out, int nsweeps) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= e.batch) return;
  int act = 0;
  if (!proc || proc[b]) {
    // the measure's workgroup partials in order
    double off2 = 0.0;
    for (int q = 0; q < chunks; ++q) off2 += e.off_part[(int64_t)b * chunks + q];
    e.off2[b] = off2;
    act = !last && off2 > (double)off_tol2 * (double)e.hnorm2[b];
  }
  e.active[b] = act;
  if (act) {
    atomicAdd(counter, 1);
    sweeps_out[b] += nsweeps;
  }
}

// dst[b][:n, :n] = src[b][:n, :n] (leading dimension np) for the active matrices
__global__ void k_copy_active(const float* src, float* dst, int n, int np, const int* active) {
  const int b = blockIdx.y;
  if (!active[b]) return;
  const int64_t off = (int64_t)b * np * np;
  for (int i = blockIdx.x; i < n; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x) dst[off + (int64_t)i * np + j] = src[off + (int64_t)i * np + j];
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

int eigh_blocks(int64_t n) {
  int nb = 4;
  while ((int64_t)nb * BS < n) nb <<= 1;
  return nb;
}

// V is deferred (updated once per sweep by k_jac_vsweep) when a slab of it
// fits in LDS: np <= 1024
static bool eigh_deferred(int64_t np) { return np <= 1024; }

// workgroups per matrix of the restart measure (each a run of 32 x 32 tile pairs)
static int restart_chunks(int64_t n, int64_t batch) {
  const int64_t nt = (n + 31) / 32, npairs = nt * (nt + 1) / 2;
  const int64_t per = batch > 0 ? (2048 + batch - 1) / batch : 2048;  // an empty batch sizes nothing
  return (int)std::max<int64_t>(1, std::min<int64_t>(npairs, per));
}

size_t eigh_ws_bytes(int64_t batch, int64_t n, int max_sweeps) {
  const int64_t nb = eigh_blocks(n), np = nb * BS, ng = nb / 4;
  const int64_t nph = eigh_deferred(np) ? nb / 2 : 1;
  size_t f = 0;
  f += 3 * batch * np * np;          // Hw, Vw, V2
  f += batch * n;                    // lamr
  f += batch * nph * ng * QSTRIDE;   // Qw
  f += batch;                        // hnorm2
  f += 2 * batch;                    // off2 (FP64)
  f += 2 * batch * n;                // sign, (perm as int)
  f += batch * ng * 2;               // rotated-mass slots
  f += batch * ng * ng * 4;          // |H|_F^2 slots
  f += 2 * batch * (size_t)restart_chunks(n, batch);  // restart-measure slots (FP64)
  size_t i = batch * (size_t)(max_sweeps + 2) + batch + 16;  // rotcnt, active, counters
  return (f + i) * 4 + 16 * 256;
}

EighWs eigh_ws_carve(void* ws, int64_t batch, int64_t n, int max_sweeps) {
  EighWs e;
  e.batch = (int)batch;
  e.n = (int)n;
  e.nb = eigh_blocks(n);
  e.np = e.nb * BS;
  const int64_t np = e.np, ng = e.nb / 4;
  e.deferred = eigh_deferred(np) ? 1 : 0;
  e.nph_store = e.deferred ? e.nb / 2 : 1;
  char* p = (char*)ws;
  auto take = [&](size_t bytes) { char* r = p; p += (bytes + 255) / 256 * 256; return (void*)r; };
  e.Hw = (float*)take(batch * np * np * 4);
  e.Vw = (float*)take(batch * np * np * 4);
  e.V2 = (float*)take(batch * np * np * 4);
  e.lamr = (float*)take(batch * n * 4);
  e.Qw = (float*)take(batch * e.nph_store * ng * QSTRIDE * 4);
  e.hnorm2 = (float*)take(batch * 4);
  e.off2 = (double*)take(batch * 8);
  e.sgn = (float*)take(batch * n * 4);
  e.perm = (int*)take(batch * n * 4);
  e.rotcnt = (int*)take(batch * (size_t)(max_sweeps + 2) * 4);
  e.rotsq = (float*)take(batch * ng * 2 * 4);
  e.hn_part = (float*)take(batch * ng * ng * 4 * 4);
  e.off_part = (double*)take(batch * (size_t)restart_chunks(n, batch) * 8);
  e.active = (int*)take(batch * 4);
  e.counter = (int*)take(64);
  e.max_sweeps = max_sweeps;
  return e;
}

std::vector<EighPhase> eigh_phases(int nb) {
  std::vector<EighPhase> out;
  for (int p = 0; p < nb / 2; ++p) out.push_back(eigh_phase(p));
  return out;
}

// The deferred V update of one sweep for the matrices of E (V row-major).
static hipError_t vsweep_launch(const EighWs& E, hipStream_t st) {
  ProfScope ps(PROF_JAC_VSWEEP, st);
  const unsigned groups8 = (unsigned)cdiv(E.batch, 8) * 8;
  switch (E.np) {
    case 64: hipLaunchKernelGGL((k_jac_vsweep<64, 64>), dim3(groups8 * 1), dim3(512), 0, st, E); break;
    case 128: hipLaunchKernelGGL((k_jac_vsweep<128, 64>), dim3(groups8 * 2), dim3(512), 0, st, E); break;
    case 256: hipLaunchKernelGGL((k_jac_vsweep<256, 64>), dim3(groups8 * 4), dim3(512), 0, st, E); break;
    case 512: hipLaunchKernelGGL((k_jac_vsweep<512, 64>), dim3(groups8 * 8), dim3(512), 0, st, E); break;
    case 1024: hipLaunchKernelGGL((k_jac_vsweep<1024, 32>), dim3(groups8 * 32), dim3(512), 0, st, E); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// View of matrices [b0, b0 + cnt) of a workspace; part h uses its own
// device counter.
// Sweeps that run in stream-parallel parts: the sweep counts at which
// matrices converge grow slowly with n (at most 10 at n = 512, 14 at 4096
// on the test spectra, restarts included)
int eigh_par_sweeps(int64_t n) {
  int s = 11;
  for (int64_t k = 1024; k <= n; k <<= 1) ++s;
  return s;
}

static EighWs eigh_sub(const EighWs& e, int b0, int cnt, int h) {
  EighWs s = e;
  const int64_t m2 = (int64_t)e.np * e.np, ng = e.nb / 4;
  s.batch = cnt;
  s.Hw += b0 * m2;
  s.Vw += b0 * m2;
  s.V2 += b0 * m2;
  s.lamr += (int64_t)b0 * e.n;
  s.Qw += b0 * e.nph_store * ng * QSTRIDE;
  s.hnorm2 += b0;
  s.off2 += b0;
  s.rotsq += (int64_t)b0 * ng * 2;
  s.sgn += (int64_t)b0 * e.n;
  s.perm += (int64_t)b0 * e.n;
  s.active += b0;
  s.counter += 4 * h;
  return s;
}

// Full eigendecomposition of a batch of symmetric n x n matrices.
hipError_t eigh_run(EighWs e, const float* H, int64_t ldh, int64_t sH, int mode,
                    const EighOpts& o, float* lam, int64_t slam, float* Vout, int64_t ldv,
                    int64_t sV, int* sweeps_out, int* flags, const int* mask,
                    const EighAux* aux, hipStream_t st) {
  hipError_t err;
  const int batch = e.batch;
  e.work = prof_work_dev();
  const int rslots = (e.nb / 4) * 2;  // rotated-mass slots per matrix (k_eigh_check clears them)
  if ((err = fill_i32(e.rotcnt, 0, (int64_t)batch * (e.max_sweeps + 2), st))) return err;
  if ((err = fill_f32(e.rotsq, 0.f, (int64_t)batch * rslots, st))) return err;
  if (mask) { if ((err = copy_i32(e.active, mask, batch, st))) return err; }
  else if ((err = fill_i32(e.active, 1, batch, st))) return err;
  hipLaunchKernelGGL(k_eigh_setup, dim3((e.nb / 4) * (e.nb / 4), batch), dim3(256), 0, st, e, H, ldh, sH, mask,
                     kSetupV | kSetupH | kSetupNorm);
  if ((err = hipGetLastError())) return err;
  hipLaunchKernelGGL(k_hnorm_finalize, dim3(cdiv(batch, 256)), dim3(256), 0, st, e, mask);
  if ((err = hipGetLastError())) return err;
  const int ng = e.nb / 4;
  const int nH = ng * (ng - 1) / 2;
  const int ntask = nH + ng * ng;
  const std::vector<EighPhase> phases = eigh_phases(e.nb);
  // Parts of the batch on parallel streams (when extra streams are given):
  // the LDS/VALU-bound pair solves of one part run beside the MFMA/HBM-bound
  // rotations of the others.  The first par_sweeps sweeps, in which most
  // matrices are still active, and the final FP64 sweep run in parts; the
  // tail of the sweep budget and the restarts, which touch few matrices,
  // run as a single part on the caller's stream, a quarter of the launches.
  struct Parts {
    int P;
    int b0[kEighParts], bc[kEighParts];
    hipStream_t ss[kEighParts];
    EighWs eh[kEighParts];
  };
  Parts multi, single;
  multi.P = std::min(aux ? std::min(std::max(aux->parts, 1), kEighParts) : 1, batch);
  for (int h = 0; h < multi.P; ++h) {
    multi.b0[h] = (int)((int64_t)batch * h / multi.P);
    multi.bc[h] = (int)((int64_t)batch * (h + 1) / multi.P) - multi.b0[h];
    multi.ss[h] = h == 0 ? st : aux->st[h - 1];
    multi.eh[h] = eigh_sub(e, multi.b0[h], multi.bc[h], h);
  }
  single.P = 1;
  single.b0[0] = 0;
  single.bc[0] = batch;
  single.ss[0] = st;
  single.eh[0] = eigh_sub(e, 0, batch, 0);
  auto fork = [&](const Parts& S) -> hipError_t {
    if (S.P < 2) return hipSuccess;
    hipError_t e2 = hipEventRecord(aux->fork, st);
    for (int h = 1; h < S.P && !e2; ++h) e2 = hipStreamWaitEvent(S.ss[h], aux->fork, 0);
    return e2;
  };
  auto join = [&](const Parts& S) -> hipError_t {
    hipError_t e2 = hipSuccess;
    for (int h = 1; h < S.P && !e2; ++h) {
      e2 = hipEventRecord(aux->join[h], S.ss[h]);
      if (!e2) e2 = hipStreamWaitEvent(st, aux->join[h], 0);
    }
    return e2;
  };
  auto phase_launches = [&](const Parts& S, int h, const EighPhase& ph, bool fp64, float skip_rel, int* rc,
                            float* vs, bool mark_skew) -> hipError_t {
    const EighWs& E = S.eh[h];
    hipStream_t sh = S.ss[h];
    const unsigned sblocks = (unsigned)(E.batch * ng);
    const unsigned ablocks = (unsigned)((int64_t)cdiv(E.batch, 8) * 8 * (e.deferred ? nH : ntask));
    if (fp64) {
      ProfScope ps(PROF_JAC_SOLVE_F64, sh);
      hipLaunchKernelGGL(k_jac_solve<double>, dim3(sblocks), dim3(128), 0, sh, E, ph, o.fp64_inner, o.abs_tol,
                         skip_rel, (int*)nullptr, (float*)nullptr);
    } else {
      ProfScope ps(PROF_JAC_SOLVE_F32, sh);
      hipLaunchKernelGGL(k_jac_solve<float>, dim3(sblocks), dim3(128), 0, sh, E, ph, o.inner_sweeps, o.abs_tol,
                         skip_rel, rc, vs);
    }
    hipError_t e2 = hipGetLastError();
    if (e2) return e2;
    if (mark_skew && (e2 = hipEventRecord(aux->skew[h], sh))) return e2;
    if (ablocks > 0) {
      ProfScope ps(PROF_JAC_APPLY, sh);
      hipLaunchKernelGGL(k_jac_apply, dim3(ablocks), dim3(256), 0, sh, E, ph);
    }
    return hipGetLastError();
  };
  // one pass over the phases for every part; part h starts after part
  // h - 1's first pair solve
  auto sweep_launches = [&](const Parts& S, bool fp64, float skip_rel, int* rc, float* vs) -> hipError_t {
    bool first = true;
    for (const EighPhase& ph : phases) {
      for (int h = 0; h < S.P; ++h) {
        hipError_t e2;
        if (first && h > 0 && (e2 = hipStreamWaitEvent(S.ss[h], aux->skew[h - 1], 0))) return e2;
        if ((e2 = phase_launches(S, h, ph, fp64, skip_rel, rc ? rc + S.b0[h] : nullptr,
                                 vs ? vs + (int64_t)S.b0[h] * rslots : nullptr, first && S.P > 1))) return e2;
      }
      first = false;
    }
    if (e.deferred)
      for (int h = 0; h < S.P; ++h) {
        hipError_t e2 = vsweep_launch(S.eh[h], S.ss[h]);
        if (e2) return e2;
      }
    return hipSuccess;
  };
  // The sweep loop runs its full budget without reading anything back: a
  // matrix leaves the active set on the device after the sweep that
  // converges it (k_eigh_check), and every later launch skips it.
  const int par_sweeps = std::min(e.max_sweeps, eigh_par_sweeps(e.n));
  if ((err = fork(multi))) return err;
  for (int sweep = 0; sweep < e.max_sweeps; ++sweep) {
    if (sweep == par_sweeps && (err = join(multi))) return err;
    const Parts& S = sweep < par_sweeps ? multi : single;
    int* rc = e.rotcnt + (int64_t)batch * sweep;
    float* vs = e.rotsq;
    if ((err = sweep_launches(S, false, 0.f, rc, vs))) return err;
    for (int h = 0; h < S.P; ++h) {
      hipLaunchKernelGGL(k_eigh_check, dim3(1), dim3(1024), 0, S.ss[h], S.eh[h], rc + S.b0[h],
                         vs + (int64_t)S.b0[h] * rslots,
                         o.tol, o.fro_tol * o.fro_tol, sweep, sweeps_out + S.b0[h], S.eh[h].counter);
      if ((err = hipGetLastError())) return err;
    }
  }
  if (par_sweeps >= e.max_sweeps && (err = join(multi))) return err;
  // matrices still active after max_sweeps did not converge
  hipLaunchKernelGGL(k_flag_active, dim3(cdiv(batch, 256)), dim3(256), 0, st, e.active, batch, flags,
                     (int)SVDP_FLAG_EIGH_NOT_CONVERGED);
  if ((err = hipGetLastError())) return err;
  // final sweep(s) with FP64 pair solves on every matrix
  if (o.fp64_sweeps > 0) {
    if (mask) { if ((err = copy_i32(e.active, mask, batch, st))) return err; }
    else if ((err = fill_i32(e.active, 1, batch, st))) return err;
    if ((err = fork(multi))) return err;
    for (int f = 0; f < o.fp64_sweeps; ++f)
      if ((err = sweep_launches(multi, true, 0.f, nullptr, nullptr))) return err;
    if ((err = join(multi))) return err;
  }
  const int np = e.np;
  const int64_t m2 = (int64_t)np * np;
  // V row-major: Vw itself when deferred, else untiled into Hw; one
  // Newton-Schulz step re-orthonormalises it, V2 = V (3 I - V^T V) / 2 (V^T V
  // in the other of Hw / Vw; H is no longer needed)
  {
    float* Vrow = e.Vw;
    float* Gram = e.Hw;
    if (!e.deferred) {
      hipLaunchKernelGGL(k_untile, dim3(np, batch), dim3(256), 0, st, e.Vw, e.Hw, np, e.nb, mask);
      if ((err = hipGetLastError())) return err;
      Vrow = e.Hw;
      Gram = e.Vw;
    }
    GemmArgs g;
    memset(&g, 0, sizeof(g));
    g.M = np; g.N = np; g.K = np; g.batch = batch;
    g.A = Vrow; g.lda = np; g.sA = m2;
    g.B = Vrow; g.ldb = np; g.sB = m2;
    g.C = Gram; g.ldc = np; g.sC = m2;
    g.alpha = 1.f; g.sym = 1; g.active = mask;
    if ((err = gemm_launch(g, PREC_F32, 1, 0, st))) return err;
    GemmArgs u;
    memset(&u, 0, sizeof(u));
    u.M = np; u.N = np; u.K = np; u.batch = batch;
    u.A = Vrow; u.lda = np; u.sA = m2;
    u.B = Gram; u.ldb = np; u.sB = m2;
    u.C = e.V2; u.ldc = np; u.sC = m2;
    u.Cin = Vrow; u.ldcin = np; u.sCin = m2;
    u.alpha = -0.5f; u.beta = 1.5f; u.active = mask;
    if ((err = gemm_launch(u, PREC_F32, 0, 0, st))) return err;
  }
  // Restarts.  T = V^T H V is formed from the input (H V in Hw, T in Vw):
  // its diagonal holds the eigenvalues (Rayleigh quotients) and its
  // off-diagonal norm the backward error of the decomposition, which the
  // rounding of many FP32 block rotations raises with n.  While that norm
  // exceeds off_tol |H|_F, T itself is swept from V' = I -- its rotations are
  // small, so they add little rounding; pairs entirely within T's own
  // rounding (kRestartSkip) are left alone -- and V <- V V'.
  {
    const int* proc = mask;
    const int chunks = restart_chunks(e.n, batch);
    const float tol2 = o.off_tol * o.off_tol;
    for (int r = 0;; ++r) {
      const int last = r >= o.restarts;
      GemmArgs y;
      memset(&y, 0, sizeof(y));
      y.M = e.n; y.N = e.n; y.K = e.n; y.batch = batch;
      y.A = H; y.lda = ldh; y.sA = sH;
      y.B = e.V2; y.ldb = np; y.sB = m2;
      y.C = e.Hw; y.ldc = np; y.sC = m2;
      y.alpha = 1.f; y.active = proc;
      if ((err = gemm_launch(y, PREC_F32, 0, 0, st))) return err;
      GemmArgs tt;
      memset(&tt, 0, sizeof(tt));
      tt.M = e.n; tt.N = e.n; tt.K = e.n; tt.batch = batch;
      tt.A = e.V2; tt.lda = np; tt.sA = m2;
      tt.B = e.Hw; tt.ldb = np; tt.sB = m2;
      tt.C = e.Vw; tt.ldc = np; tt.sC = m2;
      tt.alpha = 1.f; tt.active = proc;
      if ((err = gemm_launch(tt, PREC_F32, 1, 0, st))) return err;
      if ((err = fill_i32(e.counter, 0, 1, st))) return err;
      hipLaunchKernelGGL(k_restart_offnorm, dim3(chunks, batch), dim3(256), 0, st, e, e.Vw, proc);
      if ((err = hipGetLastError())) return err;
      hipLaunchKernelGGL(k_restart_decide, dim3(cdiv(batch, 256)), dim3(256), 0, st, e, proc, chunks, tol2, last,
                         e.counter, sweeps_out, std::max(1, o.fp64_sweeps));
      if ((err = hipGetLastError())) return err;
      if (last) break;
      // the restart's launches skip the matrices k_restart_decide left out
      proc = e.active;
      const dim3 sgrid((e.nb / 4) * (e.nb / 4), batch);
      hipLaunchKernelGGL(k_eigh_setup, sgrid, dim3(256), 0, st, e, e.Vw, (int64_t)np, m2, proc, kSetupH);
      if ((err = hipGetLastError())) return err;
      hipLaunchKernelGGL(k_eigh_setup, sgrid, dim3(256), 0, st, e, (const float*)nullptr, (int64_t)0, (int64_t)0,
                         proc, kSetupV);
      if ((err = hipGetLastError())) return err;
      for (int f = 0; f < std::max(1, o.fp64_sweeps); ++f)
        if ((err = sweep_launches(single, o.fp64_sweeps > 0, kRestartSkip, nullptr, nullptr))) return err;
      // V' row-major (Vw itself when deferred, else untiled into Hw); V2 V'
      // into the other buffer, then copied to V2 for the restarted matrices
      const float* Vp = e.Vw;
      float* VV = e.Hw;
      if (!e.deferred) {
        hipLaunchKernelGGL(k_untile, dim3(np, batch), dim3(256), 0, st, e.Vw, e.Hw, np, e.nb, proc);
        if ((err = hipGetLastError())) return err;
        Vp = e.Hw;
        VV = e.Vw;
      }
      GemmArgs v;
      memset(&v, 0, sizeof(v));
      v.M = e.n; v.N = e.n; v.K = e.n; v.batch = batch;
      v.A = e.V2; v.lda = np; v.sA = m2;
      v.B = Vp; v.ldb = np; v.sB = m2;
      v.C = VV; v.ldc = np; v.sC = m2;
      v.alpha = 1.f; v.active = proc;
      if ((err = gemm_launch(v, PREC_F32, 0, 0, st))) return err;
      hipLaunchKernelGGL(k_copy_active, dim3(std::min(e.n, 512), batch), dim3(256), 0, st, VV, e.V2, e.n, np,
                         proc);
      if ((err = hipGetLastError())) return err;
    }
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
