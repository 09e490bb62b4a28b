// Direct Cauchy sum on gfx950 (FP64):
//   S_i = sum_{j != i} w_j / (eta_i - eta_j)          (matrix E of eq. (e:fmm-E))
// for several weight columns w at once. This single product carries every
// operator of the method: Im and Re of A_i S_i give B x and D x
// (eqs. (e:(I-B)x), (e:hD-bt)); (eta'/A) S with w = A x gives B^T x
// (eq. (e:BTx)); w = eta' gives the vector e (eq. (e:bve)).
//
// Mapping (VALU-bound, no matrix cores: every pair needs its own reciprocal):
//   * sources are packed records {eta_j, eta'_j, w_j,q.., b_j,q..} (16 B each
//     field; eta' = eta - centre of the node's 64-node tile, b = w conj(eta'));
//     the source loop index is wave-uniform, so whole records arrive with wide
//     scalar loads into SGPRs and are broadcast to all lanes (no LDS traffic,
//     no bank conflicts); near tiles fetch four sources per iteration so one
//     wait covers four reciprocals; far tiles (FP64 far form: two sources per
//     step with one column, one with two) and the near tiles of 8-column
//     mixed products stream their sources, the next step's fields loading
//     during the current step;
//   * each lane owns TPT target nodes (a tile of TPT*64 consecutive targets),
//     which reuses every fetched source TPT times and gives independent chains;
//   * the four wavefronts of a workgroup share the tile and split its source
//     chunk four ways, then add their sums through LDS in wave order;
//   * the work is a list of items (domain, target tile, source split, column
//     group) covering every domain of a batch in one launch per column-group
//     width, one workgroup per item (largest domains first); the consumer
//     adds the split partial sums in a fixed order, so results are bitwise
//     reproducible;
//   * 1/|d|^2 comes from v_rcp_f64 refined by one Newton step; two pairs
//     share one reciprocal: 1/a = b/(ab), 1/b = a/(ab) (simultaneous
//     inversion), which halves the v_rcp_f64 issues; the pairs are two
//     sources against one target, or, in the one-source steps, one source
//     against the lane's two targets. The one-column far form and the
//     near tiles with <= 2 columns share one reciprocal among four pairs
//     (two sources and two targets, or four sources);
//   * only the window of sources equal to the wave's own targets needs the
//     j != i test; it runs a separate masked loop.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "gnk_device.h"
#include "gnk_internal.h"

namespace gnk {

namespace {

#include "pair_steps.inl"

// Far source tiles in FP64, one column. With z' = z_i - c and
// eta'_j = eta_j - c (c the source tile's centre) and m = 1/|z' - eta'_j|^2,
//   S_i = sum_j w_j conj(z' - eta'_j) m = conj(z') sum_j w_j m - sum_j b_j m,
// b_j = w_j conj(eta'_j) taken from the record: per pair two FMAs per part
// and no product for q. The squared distance comes from the record's
// u_j = -2 eta'_j and a_j = |eta'_j|^2 and the target's |z'|^2 as
// a_j + |z'|^2 + u_j . z' (one add, two FMAs). The tile pair is far (centres
// more than 1.5 (r_t + r_s) apart), so |z'| > 1.5 |eta'_j|: |z' - eta'_j|^2 is
// at least a thirteenth of a_j + |z'|^2 and the distance keeps all but about
// four bits; |z'| + |eta'_j| is at most five times |z' - eta'_j|, which bounds
// the cancellation of conj(z') A against B the same way.
template <int NR, int TPT>
struct AccAB {
  double ax[TPT][NR], ay[TPT][NR], bx[TPT][NR], by[TPT][NR];
};

template <int NR, int TPT, class P>
__device__ __forceinline__ void accumulate_ab(AccAB<NR, TPT>& a, int t, P r, int wo, int wb, double m) {
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    const double2 w = r[wo + q], b = r[wb + q];
    a.ax[t][q] = __builtin_fma(w.x, m, a.ax[t][q]);
    a.ay[t][q] = __builtin_fma(w.y, m, a.ay[t][q]);
    a.bx[t][q] = __builtin_fma(b.x, m, a.bx[t][q]);
    a.by[t][q] = __builtin_fma(b.y, m, a.by[t][q]);
  }
}

// |z' - eta'_j|^2 from the record head (u_j at [1], a_j at [2].x) and the
// target (z', |z'|^2)
template <class P>
__device__ __forceinline__ double far_dist2(P r, double zx, double zy, double zz) {
  const double2 u = r[1];
  return __builtin_fma(u.x, zx, __builtin_fma(u.y, zy, r[2].x + zz));
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void pair_step_far(AccAB<NR, TPT>& acc, const double (&zx)[TPT], const double (&zy)[TPT],
                                              const double (&zz)[TPT], P ra, P rb, int wo, int wb) {
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double da = far_dist2(ra, zx[t], zy[t], zz[t]);
    const double db = far_dist2(rb, zx[t], zy[t], zz[t]);
    const double R = refine_rcp(da * db);
    accumulate_ab<NR, TPT>(acc, t, ra, wo, wb, db * R);
    accumulate_ab<NR, TPT>(acc, t, rb, wo, wb, da * R);
  }
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void single_step_far(AccAB<NR, TPT>& acc, const double (&zx)[TPT],
                                                const double (&zy)[TPT], const double (&zz)[TPT], P r, int wo,
                                                int wb) {
#pragma unroll
  for (int t = 0; t < TPT; ++t)
    accumulate_ab<NR, TPT>(acc, t, r, wo, wb, refine_rcp(far_dist2(r, zx[t], zy[t], zz[t])));
}


// The far form with one source per step (TPT even): the lane's targets are
// taken in twos that share one reciprocal (m_0 = d_1/(d_0 d_1)), and the next
// source's fields (u, a, w, b: 7 + 4(NR - 1) doubles) load into scalar
// registers during the step's arithmetic, issued after the current fields'
// first use (scalar loads may return out of order, so the wait before that
// use covers every scalar load issued before it).
template <int NR>
struct FarRec {
  double2 u;
  double a;
  double2 w[NR], b[NR];
};

template <int NR, class P>
__device__ __forceinline__ void load_far(FarRec<NR>& s, P r, int wo, int wb) {
  s.u = r[1];
  s.a = r[2].x;
#pragma unroll
  for (int q = 0; q < NR; ++q) {
    s.w[q] = r[wo + q];
    s.b[q] = r[wb + q];
  }
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void stream_step_far(AccAB<NR, TPT>& acc, const double (&zx)[TPT],
                                                const double (&zy)[TPT], const double (&zz)[TPT],
                                                const FarRec<NR>& s, FarRec<NR>& nx, P rn, int wo, int wb) {
  double d[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) d[t] = __builtin_fma(s.u.x, zx[t], __builtin_fma(s.u.y, zy[t], s.a + zz[t]));
  __builtin_amdgcn_sched_barrier(0);
  load_far<NR>(nx, rn, wo, wb);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < TPT; t += 2) {
    const double R = refine_rcp(d[t] * d[t + 1]);
    const double m[2] = {d[t + 1] * R, d[t] * R};
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        acc.ax[t + v][q] = __builtin_fma(s.w[q].x, m[v], acc.ax[t + v][q]);
        acc.ay[t + v][q] = __builtin_fma(s.w[q].y, m[v], acc.ay[t + v][q]);
        acc.bx[t + v][q] = __builtin_fma(s.b[q].x, m[v], acc.bx[t + v][q]);
        acc.by[t + v][q] = __builtin_fma(s.b[q].y, m[v], acc.by[t + v][q]);
      }
  }
}

// Two sources per step: one reciprocal for the four pairs of two sources and
// the lane's two targets (R = 1/(d00 d01 d10 d11), m00 = R d01 (d10 d11), ...;
// the product stays in range while every squared distance lies in
// [1e-75, 1e75]); the next two sources' fields load during the step.
template <int NR, int TPT, class P>
__device__ __forceinline__ void stream_step_far2(AccAB<NR, TPT>& acc, const double (&zx)[TPT],
                                                 const double (&zy)[TPT], const double (&zz)[TPT],
                                                 const FarRec<NR>& s0, const FarRec<NR>& s1, FarRec<NR>& n0,
                                                 FarRec<NR>& n1, P rn0, P rn1, int wo, int wb) {
  double d0[TPT], d1[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    d0[t] = __builtin_fma(s0.u.x, zx[t], __builtin_fma(s0.u.y, zy[t], s0.a + zz[t]));
    d1[t] = __builtin_fma(s1.u.x, zx[t], __builtin_fma(s1.u.y, zy[t], s1.a + zz[t]));
  }
  __builtin_amdgcn_sched_barrier(0);
  load_far<NR>(n0, rn0, wo, wb);
  load_far<NR>(n1, rn1, wo, wb);
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int t = 0; t < TPT; t += 2) {
    const double p0 = d0[t] * d0[t + 1], p1 = d1[t] * d1[t + 1];
    const double R = refine_rcp(p0 * p1);
    const double r0 = R * p1, r1 = R * p0;
    const double m[2][2] = {{r0 * d0[t + 1], r0 * d0[t]}, {r1 * d1[t + 1], r1 * d1[t]}};
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        acc.ax[t + v][q] = __builtin_fma(s0.w[q].x, m[0][v], acc.ax[t + v][q]);
        acc.ay[t + v][q] = __builtin_fma(s0.w[q].y, m[0][v], acc.ay[t + v][q]);
        acc.bx[t + v][q] = __builtin_fma(s0.b[q].x, m[0][v], acc.bx[t + v][q]);
        acc.by[t + v][q] = __builtin_fma(s0.b[q].y, m[0][v], acc.by[t + v][q]);
        acc.ax[t + v][q] = __builtin_fma(s1.w[q].x, m[1][v], acc.ax[t + v][q]);
        acc.ay[t + v][q] = __builtin_fma(s1.w[q].y, m[1][v], acc.ay[t + v][q]);
        acc.bx[t + v][q] = __builtin_fma(s1.b[q].x, m[1][v], acc.bx[t + v][q]);
        acc.by[t + v][q] = __builtin_fma(s1.b[q].y, m[1][v], acc.by[t + v][q]);
      }
  }
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void stream_far4(AccAB<NR, TPT>& acc, const double (&zx)[TPT], const double (&zy)[TPT],
                                            const double (&zz)[TPT], P rec, int stride, int wo, int wb, int ja,
                                            int jb) {
  static_assert(TPT % 2 == 0, "targets are paired");
  if (jb - ja < 4) {
    // short tail segment
    FarRec<NR> a, b;
    if (ja >= jb) return;
    load_far<NR>(a, rec + (size_t)ja * stride, wo, wb);
    for (int j = ja; j < jb; ++j) {
      stream_step_far<NR, TPT>(acc, zx, zy, zz, a, b, rec + (size_t)min(j + 1, jb - 1) * stride, wo, wb);
      a = b;
    }
    return;
  }
  FarRec<NR> a0, a1, b0, b1;
  load_far<NR>(a0, rec + (size_t)ja * stride, wo, wb);
  load_far<NR>(a1, rec + (size_t)(ja + 1) * stride, wo, wb);
  int j = ja;
  const int last = jb - 1;
  for (; j + 3 < jb; j += 4) {
    stream_step_far2<NR, TPT>(acc, zx, zy, zz, a0, a1, b0, b1, rec + (size_t)(j + 2) * stride,
                              rec + (size_t)(j + 3) * stride, wo, wb);
    stream_step_far2<NR, TPT>(acc, zx, zy, zz, b0, b1, a0, a1, rec + (size_t)min(j + 4, last) * stride,
                              rec + (size_t)min(j + 5, last) * stride, wo, wb);
  }
  // 0-3 sources left: a0, a1 hold sources j and j + 1 when they exist
  if (j + 1 < jb) {
    stream_step_far2<NR, TPT>(acc, zx, zy, zz, a0, a1, b0, b1, rec + (size_t)min(j + 2, last) * stride,
                              rec + (size_t)min(j + 3, last) * stride, wo, wb);
    j += 2;
    a0 = b0;
  }
  if (j < jb) stream_step_far<NR, TPT>(acc, zx, zy, zz, a0, b0, rec + (size_t)j * stride, wo, wb);
}

// sources [ja, jb) of a far tile; the last prefetch re-reads source jb - 1
template <int NR, int TPT, class P>
__device__ __forceinline__ void stream_far(AccAB<NR, TPT>& acc, const double (&zx)[TPT], const double (&zy)[TPT],
                                           const double (&zz)[TPT], P rec, int stride, int wo, int wb, int ja,
                                           int jb) {
  static_assert(TPT % 2 == 0, "targets are paired");
  if (ja >= jb) return;
  FarRec<NR> a, b;
  load_far<NR>(a, rec + (size_t)ja * stride, wo, wb);
  int j = ja;
  for (; j + 1 < jb; j += 2) {
    stream_step_far<NR, TPT>(acc, zx, zy, zz, a, b, rec + (size_t)(j + 1) * stride, wo, wb);
    stream_step_far<NR, TPT>(acc, zx, zy, zz, b, a, rec + (size_t)min(j + 2, jb - 1) * stride, wo, wb);
  }
  if (j < jb) stream_step_far<NR, TPT>(acc, zx, zy, zz, a, b, rec + (size_t)j * stride, wo, wb);
}

// ---------------------------------------------------------------------------
// Mixed precision: well-separated source tiles in FP32, the rest in FP64.
// A source tile is 64 consecutive nodes with bounding circle (c_s, r_s); the
// workgroup's target tile has (c_t, r_t). The tile pair is far when
// |c_t - c_s| > (1 + theta)(r_t + r_s). The FP32 records hold the offsets in
// units of the tile radius, v_j = (eta_j - c_s)/r_s (formed in FP64, then
// rounded), a_j = |v_j|^2, the weights w_j and b_j = w_j conj(v_j); every
// lane forms z' = (z_i - c_s)/r_s in FP64 and rounds it. As in the FP64 far
// form,
//   r_s S_i = conj(z') sum_j w_j m_j - sum_j b_j m_j,  m_j = 1/|z' - v_j|^2,
//   |z' - v_j|^2 = a_j + |z'|^2 - 2 v_j . z'   (one add, two FMAs),
// with one FP32 reciprocal for two sources (m_a = d_b/(d_a d_b)): in tile
// radii the squared distances lie between about 1 and the square of the
// domain's size in tile radii, so their product stays within the FP32 range
// whatever the scale of the domain. Four FMAs per column and pair. The tile's
// 64 terms are summed in FP32; the combination with conj(z') and the factor
// 1/r_s are applied in FP64 and added to the FP64 accumulators. The pair is
// far, so |z'| > 2 |v_j| and the distance keeps all but a few bits (it is at
// least a fifth of a_j + |z'|^2).
template <int NR, int TPT>
struct AccAB32 {
  float ax[TPT][NR], ay[TPT][NR], bx[TPT][NR], by[TPT][NR];
};

// one source (record fields already loaded) against the lane's TPT targets
template <int NR, int TPT>
__device__ __forceinline__ void step_far32(AccAB32<NR, TPT>& a, const float (&m2x)[TPT], const float (&m2y)[TPT],
                                           const float (&zz)[TPT], float2 v, float av, const float2 (&w)[NR],
                                           const float2 (&b)[NR]) {
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const float m = __builtin_amdgcn_rcpf(__builtin_fmaf(v.x, m2x[t], __builtin_fmaf(v.y, m2y[t], av + zz[t])));
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      a.ax[t][q] = __builtin_fmaf(w[q].x, m, a.ax[t][q]);
      a.ay[t][q] = __builtin_fmaf(w[q].y, m, a.ay[t][q]);
      a.bx[t][q] = __builtin_fmaf(b[q].x, m, a.bx[t][q]);
      a.by[t][q] = __builtin_fmaf(b[q].y, m, a.by[t][q]);
    }
  }
}

// two sources (record fields already loaded), one reciprocal
template <int NR, int TPT>
__device__ __forceinline__ void pair_step_far32(AccAB32<NR, TPT>& a, const float (&m2x)[TPT],
                                                const float (&m2y)[TPT], const float (&zz)[TPT], const float2 (&v)[2],
                                                const float (&av)[2], const float2 (&w)[2][NR],
                                                const float2 (&b)[2][NR]) {
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const float da = __builtin_fmaf(v[0].x, m2x[t], __builtin_fmaf(v[0].y, m2y[t], av[0] + zz[t]));
    const float db = __builtin_fmaf(v[1].x, m2x[t], __builtin_fmaf(v[1].y, m2y[t], av[1] + zz[t]));
    const float r = __builtin_amdgcn_rcpf(da * db);
    const float m[2] = {db * r, da * r};
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        a.ax[t][q] = __builtin_fmaf(w[k][q].x, m[k], a.ax[t][q]);
        a.ay[t][q] = __builtin_fmaf(w[k][q].y, m[k], a.ay[t][q]);
        a.bx[t][q] = __builtin_fmaf(b[k][q].x, m[k], a.bx[t][q]);
        a.by[t][q] = __builtin_fmaf(b[k][q].y, m[k], a.by[t][q]);
      }
  }
}

// the sources [ts, te) of one far tile: FB32 records fetched (wave-uniform
// scalar loads) before their arithmetic, so one wait covers them; two rather
// than four leave fewer scalar registers to spill into vector lanes (46
// against 69 in the one-column variant; the close-boundary mixed solve
// 1.47 s against 1.51 s)
constexpr int FB32 = 2;   // a pair: one reciprocal
template <int NR, int TPT, class P>
__device__ __forceinline__ void tile_far32(AccAB32<NR, TPT>& a, const float (&m2x)[TPT], const float (&m2y)[TPT],
                                           const float (&zz)[TPT], P rec32, int stride32, int wo, int wb, int ts,
                                           int te) {
  int j = ts;
  for (; j + FB32 - 1 < te; j += FB32) {
    P r = rec32 + (size_t)j * stride32;
    float2 v[FB32], w[FB32][NR], b[FB32][NR];
    float av[FB32];
#pragma unroll
    for (int k = 0; k < FB32; ++k) {
      P rk = r + k * stride32;
      v[k] = rk[0];
      av[k] = rk[1].x;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        w[k][q] = rk[wo + q];
        b[k][q] = rk[wb + q];
      }
    }
    pair_step_far32<NR, TPT>(a, m2x, m2y, zz, v, av, w, b);
  }
  for (; j < te; ++j) {
    P r = rec32 + (size_t)j * stride32;
    float2 w[NR], b[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      w[q] = r[wo + q];
      b[q] = r[wb + q];
    }
    step_far32<NR, TPT>(a, m2x, m2y, zz, r[0], r[1].x, w, b);
  }
}

// Far tiles on the matrix cores (4 and 8 columns), in the A/B form of the
// FP32 far tiles above, with every offset taken from the centre of the target
// tile and divided by its radius r_t: for targets u_i and sources v_k so
// scaled and m_ik = 1/|u_i - v_k|^2,
//   sum_k w_k / (u_i - v_k) = conj(u_i) sum_k m_ik w_k - sum_k m_ik b_k,
// b_k = w_k conj(v_k), and the sum for the unscaled offsets is this one
// divided by r_t. One v_mfma_f32_32x32x2f32 per 32 targets and two sources
// forms both sums: its A operand holds 32 rows, the (Re, Im) components of
// the 8 columns' weights (rows 0-15) and of their b (rows 16-31), lane l
// supplying A[row = l%32][k = l/32]; its B operand is the one real factor m of
// the pair (target l%32, source l/32). Each lane so forms one m per MFMA, and
// the two target groups of a wave share one reciprocal (m_0 = a_1/(a_0 a_1),
// m_1 = a_0/(a_0 a_1), the scaled squared distances lying between about 1 and
// the square of the domain's size in tile radii). The FP32 matrix cores and
// the VALU do not overlap on this chip, so the pair's VALU work is what the
// MFMAs cannot hide. Row 8(r/4) + 4(l/32) + r%4 of the result sits in
// register r of lane l (column l%32): a lane holds W and B of the same
// components eight registers apart, Re and Im side by side, and combines them
// with its target's u once the wave's far tiles for the slot are summed. Every
// source of a far tile is further from each target than the target's own
// offset |u_i|, so conj(u_i) W never dominates B and the difference does not
// cancel.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// Records of one far tile are staged in the wave's LDS area (lane k copies
// source ts + k): its scaled offset v, the 16 weight components and the 16
// components of b = w conj(v), zero for columns beyond the item's width and
// for rows beyond the tile, so a K-step reads its A operand directly.
constexpr int kFarStage = 36;   // floats per staged source: v.x, v.y, 2 pad, w[16], b[16]

// The 32 K-steps (two sources each) of one staged tile for two groups of 32
// targets. Rows past a short tile's end hold zero weights.
__device__ __forceinline__ void far_ksteps(f32x16 (&acc)[2], const float (&ux)[2], const float (&uy)[2],
                                           const float* stg) {
  const int lane = threadIdx.x & 63;
  const int k = lane >> 5, i = lane & 31;
#pragma unroll 4
  for (int p = 0; p < 32; ++p) {
    const float* r = stg + (2 * p + k) * kFarStage;
    const float2 v = *reinterpret_cast<const float2*>(r);
    const float a = r[4 + i];
    const float dx0 = ux[0] - v.x, dy0 = uy[0] - v.y;
    const float dx1 = ux[1] - v.x, dy1 = uy[1] - v.y;
    const float s0 = __builtin_fmaf(dy0, dy0, dx0 * dx0);
    const float s1 = __builtin_fmaf(dy1, dy1, dx1 * dx1);
    const float rr = __builtin_amdgcn_rcpf(s0 * s1);
    acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, s1 * rr, acc[0], 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, s0 * rr, acc[1], 0, 0, 0);
  }
}

// One far source tile: stage it (offsets from the target tile's centre,
// scaled: (v_s + c_s - c_t) / r_t, the stored v_s being relative to the
// source tile's centre c_s) and run its K-steps. Rows past the tile's end get
// the source tile's centre and zero weights, which keeps m finite.
template <int NR>
__device__ __forceinline__ void far_tile_mfma(f32x16 (&acc)[2], const float (&ux)[2], const float (&uy)[2], float dcx,
                                              float dcy, float sc, gptr<const float2> far, int len, float* stg,
                                              int width) {
  const int lane = threadIdx.x & 63;
  {
    float2 v = make_float2(dcx * sc, dcy * sc);
    float2 w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) w[q] = make_float2(0.f, 0.f);
    if (lane < len) {
      gptr<const float2> r = far + lane;
      const float2 vs = r[0];
      v = make_float2((vs.x + dcx) * sc, (vs.y + dcy) * sc);
#pragma unroll
      for (int q = 0; q < NR; ++q)
        if (q < width) w[q] = r[64 * (1 + q)];
    }
    float* o = stg + lane * kFarStage;
    *reinterpret_cast<f32x4*>(o) = f32x4{v.x, v.y, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      const float2 b0 = make_float2(__builtin_fmaf(w[q].x, v.x, w[q].y * v.y), __builtin_fmaf(w[q].y, v.x, -w[q].x * v.y));
      const float2 b1 = make_float2(__builtin_fmaf(w[q + 1].x, v.x, w[q + 1].y * v.y),
                                    __builtin_fmaf(w[q + 1].y, v.x, -w[q + 1].x * v.y));
      *reinterpret_cast<f32x4*>(o + 4 + 2 * q) = f32x4{w[q].x, w[q].y, w[q + 1].x, w[q + 1].y};
      *reinterpret_cast<f32x4*>(o + 20 + 2 * q) = f32x4{b0.x, b0.y, b1.x, b1.y};
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  far_ksteps(acc, ux, uy, stg);
  // the next tile's staging overwrites stg
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Launch modes of the pair kernel:
//   M_FP64  every pair in FP64;
//   M_MIXED near tiles FP64, far tiles FP32 on the VALU (1-2 columns);
//   M_NEAR  near tiles only, FP64 (4-8 columns of a mixed product), added to
//           the partial sums that k_far (below) wrote for the same items just
//           before; items without a near tile store nothing.
// k_far takes the far tiles on the matrix cores. Splitting a mixed product in
// two keeps each kernel's register footprint small (the FP64 loops and the
// MFMA accumulators do not share a register file).
enum : int { M_FP64 = 0, M_MIXED = 1, M_NEAR = 2, M_EXT = 3 };

// One work item: the tile of 64*TPT targets pts[base ..] (the nodes, read from
// their own 16-byte array rather than the records, or for M_EXT the separate
// points), a range of sources of the domain, weight columns col0 .. col0+NR-1. The four
// wavefronts of the workgroup take consecutive parts [j0, j1) of the range;
// their sums are added through LDS in wave order. MIXED: far source tiles of 64
// nodes are summed in FP32 (see above). All pointers are restrict-qualified
// parameters, so after inlining the record loads are known not to alias the
// partial-sum stores and stay scalar (wave-uniform) loads.
template <int NR, int TPT, int MODE>
__device__ __forceinline__ void pair_item(gptr<const double2> rec, gptr<const float2> rec32, gptr<const double4> sb,
                                          gptr<const double4> sbf, gptr<const double4> tb, gptr<double2> part, int N,
                                          gptr<const double2> pts, int Nt, int stride, int stride32, int wcols,
                                          int col0, int width, int base, int tile_idx, int g, int j0, int j1,
                                          double far2, double (&red)[3][TPT][2][64]) {
  constexpr int kTile = 64 * TPT;
  const int wo = kRecHead + col0;            // FP64 record: weights of the item's first column
  const int wb = kRecHead + wcols + col0;    // FP64 record: its b = w conj(eta')
  const int wo32 = 2 + col0;          // FP32 record: weights of the item's first column
  const int wb32 = 2 + wcols + col0;  // FP32 record: its b = w conj(v)
  constexpr bool MIXED = MODE == M_MIXED || MODE == M_NEAR;
  // M_EXT: FP64 with targets pts[0..Nt) that are not nodes (no j != i window)
  constexpr bool EXT = MODE == M_EXT;
  const int NT = EXT ? Nt : N;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  double2 tg[TPT];
  int ti[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    ti[t] = base + t * 64 + lane;
    tg[t] = pts[min(ti[t], NT - 1)];
  }
  Acc<NR, TPT> acc;
#pragma unroll
  for (int t = 0; t < TPT; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) { acc.x[t][r] = 0.0; acc.y[t][r] = 0.0; }

  // sources outside the tile's own window need no j != i test
  auto plain = [&](int ja, int jb) {
    if constexpr (MODE == M_NEAR && NR >= 8 && TPT % 2 == 0) {
      stream_range<NR, TPT>(acc, tg, rec, stride, wo, ja, jb);
      return;
    }
    int j = ja;
    for (; j + 3 < jb; j += 4) {
      gptr<const double2> r = rec + (size_t)j * stride;
      if constexpr (NR <= 2) {
        quad_step<NR, TPT>(acc, tg, r, r + stride, r + 2 * stride, r + 3 * stride, wo);
      } else {
        // four wide records would not fit in scalar registers together
        if constexpr (NR == 8 && TPT % 2 == 0) {
          // one reciprocal for two sources and two targets (4 columns: the
          // extra registers cost a wave per SIMD)
          pair_step_t2<NR, TPT>(acc, tg, r, r + stride, wo);
          pair_step_t2<NR, TPT>(acc, tg, r + 2 * stride, r + 3 * stride, wo);
        } else {
          pair_step<NR, TPT>(acc, tg, r, r + stride, wo);
          pair_step<NR, TPT>(acc, tg, r + 2 * stride, r + 3 * stride, wo);
        }
      }
    }
    for (; j + 1 < jb; j += 2) {
      gptr<const double2> r = rec + (size_t)j * stride;
      pair_step<NR, TPT>(acc, tg, r, r + stride, wo);
    }
    if (j < jb) single_step<NR, TPT>(acc, tg, ti, rec + (size_t)j * stride, wo, j, false);
  };
  auto fp64_range = [&](int ja, int jb) {
    if constexpr (EXT) {
      plain(ja, jb);
      return;
    }
    plain(ja, min(jb, base));
    const int ma = max(ja, base), mb = min(jb, base + kTile);
    for (int j = ma; j < mb; ++j) single_step<NR, TPT>(acc, tg, ti, rec + (size_t)j * stride, wo, j, true);
    plain(max(ja, base + kTile), jb);
  };

  bool any_near = false;
  if constexpr (!MIXED && (NR == 1 || (NR == 2 && !EXT))) {
    // source tiles of kFarTile nodes (segments of them at the range ends): far
    // ones by the A/B form on coordinates relative to the tile centre, the
    // rest as above (one column, or two with node targets: separate points in
    // the caller's order seldom make far tiles, and the two-column far form
    // needs more registers)
    const double4 tbd = tb[tile_idx];
    for (int ts = j0; ts < j1;) {
      const int te = min(((ts >> kFarTileLog2) + 1) << kFarTileLog2, j1);
      const double4 sbd = sbf[ts >> kFarTileLog2];
      const double dcx = tbd.x - sbd.x, dcy = tbd.y - sbd.y;
      const double rr = tbd.z + sbd.z;
      if ((dcx * dcx + dcy * dcy) > far2 * rr * rr) {
        double zx[TPT], zy[TPT], zz[TPT];
        AccAB<NR, TPT> ab;
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
          zx[t] = tg[t].x - sbd.x;
          zy[t] = tg[t].y - sbd.y;
          zz[t] = __builtin_fma(zy[t], zy[t], zx[t] * zx[t]);
#pragma unroll
          for (int r = 0; r < NR; ++r) ab.ax[t][r] = ab.ay[t][r] = ab.bx[t][r] = ab.by[t][r] = 0.0;
        }
        if constexpr (NR == 1 && TPT % 2 == 0) {
          stream_far4<NR, TPT>(ab, zx, zy, zz, rec, stride, wo, wb, ts, te);
        } else if constexpr (TPT % 2 == 0) {
          // two columns: four records of two-column fields would spill
          stream_far<NR, TPT>(ab, zx, zy, zz, rec, stride, wo, wb, ts, te);
        } else {
          int j = ts;
          // one target per lane: two sources per reciprocal (four records
          // would not fit in the scalar registers of an 8-wave launch)
          for (; j + 1 < te; j += 2) {
            gptr<const double2> r = rec + (size_t)j * stride;
            pair_step_far<NR, TPT>(ab, zx, zy, zz, r, r + stride, wo, wb);
          }
          for (; j < te; ++j) single_step_far<NR, TPT>(ab, zx, zy, zz, rec + (size_t)j * stride, wo, wb);
        }
#pragma unroll
        for (int t = 0; t < TPT; ++t)
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            acc.x[t][r] += __builtin_fma(zx[t], ab.ax[t][r], zy[t] * ab.ay[t][r]) - ab.bx[t][r];
            acc.y[t][r] += __builtin_fma(zx[t], ab.ay[t][r], -zy[t] * ab.ax[t][r]) - ab.by[t][r];
          }
      } else {
        fp64_range(ts, te);
      }
      ts = te;
    }
  } else if (!MIXED) {
    fp64_range(j0, j1);
  } else {
    const double4 tbd = tb[tile_idx];
    for (int ts = j0; ts < j1; ts += 64) {
      const int te = min(ts + 64, j1);
      const double4 sbd = sb[ts >> 6];
      const double dcx = tbd.x - sbd.x, dcy = tbd.y - sbd.y;
      const double rr = tbd.z + sbd.z;
      const bool far = (dcx * dcx + dcy * dcy) > far2 * rr * rr;
      if constexpr (MODE == M_NEAR) {
        if (!far) {
          fp64_range(ts, te);
          any_near = true;
        }
      } else if (far) {
        double zx[TPT], zy[TPT];
        float m2x[TPT], m2y[TPT], zz[TPT];
        AccAB32<NR, TPT> a32;
        const double inv_r = 1.0 / sbd.z;
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
          zx[t] = (tg[t].x - sbd.x) * inv_r;
          zy[t] = (tg[t].y - sbd.y) * inv_r;
          const float fx = (float)zx[t], fy = (float)zy[t];
          m2x[t] = -2.f * fx;
          m2y[t] = -2.f * fy;
          zz[t] = __builtin_fmaf(fy, fy, fx * fx);
#pragma unroll
          for (int r = 0; r < NR; ++r) a32.ax[t][r] = a32.ay[t][r] = a32.bx[t][r] = a32.by[t][r] = 0.f;
        }
        tile_far32<NR, TPT>(a32, m2x, m2y, zz, rec32, stride32, wo32, wb32, ts, te);
#pragma unroll
        for (int t = 0; t < TPT; ++t)
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const double ax = a32.ax[t][r], ay = a32.ay[t][r];
            acc.x[t][r] += (__builtin_fma(zx[t], ax, zy[t] * ay) - (double)a32.bx[t][r]) * inv_r;
            acc.y[t][r] += (__builtin_fma(zx[t], ay, -zy[t] * ax) - (double)a32.by[t][r]) * inv_r;
          }
      } else {
        fp64_range(ts, te);
      }
    }
  }

  if constexpr (MODE == M_NEAR) {
    if (!__syncthreads_or(any_near ? 1 : 0)) return;   // k_far's sums are complete
  }
  // fixed-order reduction over the four wavefronts, one column at a time
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (wv > 0) {
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        red[wv - 1][t][0][lane] = acc.x[t][r];
        red[wv - 1][t][1][lane] = acc.y[t][r];
      }
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        double x = acc.x[t][r], y = acc.y[t][r];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          x += red[q][t][0][lane];
          y += red[q][t][1][lane];
        }
        if (ti[t] < NT && r < width) {
          const size_t o = ((size_t)g * wcols + col0 + r) * NT + ti[t];
          if constexpr (MODE == M_NEAR) {
            const double2 p = part[o];
            x += p.x;
            y += p.y;
          }
          // streamed past the L2 (read once, by the epilogue), so that the
          // source and target records stay there
          typedef double nt2 __attribute__((ext_vector_type(2)));
          __builtin_nontemporal_store(nt2{x, y}, (gptr<nt2>)(part + o));
        }
      }
    }
    __syncthreads();
  }
}

// One launch: one workgroup per item of the list. (A workgroup that looped
// over several items would store partial sums before loading the next item's
// records, and the records could then no longer be fetched with scalar loads.)
// The one-column variants (but M_NEAR) and the two-column one with separate
// targets are held to 64 VGPRs (8 waves per SIMD), which they reach without
// spilling; the two-column FP64 one, whose far form keeps A and B sums of
// both columns, to 80 (6 waves); the others keep their registers.
template <int NR, int TPT, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(((NR == 1 && MODE != M_NEAR) || (NR == 2 && MODE == M_EXT)) ? 8 : ((NR == 2 && MODE == M_FP64) ? 6 : 1)))) void k_pairs(const DomDev* __restrict__ doms, const int4* __restrict__ items,
                                               int nitems, int lead, int data, const int* __restrict__ active) {
  __shared__ double red[3][TPT][2][64];
  constexpr bool MIXED = MODE == M_MIXED || MODE == M_NEAR;
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 w = items[it];
  const DomDev& D = doms[w.x];
  const int wcols = lead + data * D.ncols;
  // first column, and the group's width (an 8-column group padded from fewer
  // columns carries its width in bits 20 and up)
  const int col0 = w.w & 0xFFFFF;
  const int width = (w.w >> 20) ? (w.w >> 20) : NR;
  if (active != nullptr) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int col = col0 + q - lead;
      any = any || (q < width && (col < 0 || active[D.c0 + col] != 0));
    }
    if (!any) return;
  }
  // the wave's sources: a quarter of the item's chunk (a multiple of 4 in
  // FP64, whole 64-node tiles in mixed precision)
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int chunk = D.chunk;
  const int jb0 = w.z * chunk;
  const int jb1 = min(D.N, jb0 + chunk);
  const int wchunk = MIXED ? (chunk >> 2) : (((chunk + 15) >> 4) << 2);
  const int j0 = min(jb1, jb0 + wv * wchunk);
  const int j1 = min(jb1, j0 + wchunk);
  pair_item<NR, TPT, MODE>((gptr<const double2>)D.rec, (gptr<const float2>)D.rec32, (gptr<const double4>)D.sb,
                            (gptr<const double4>)D.sbf, (gptr<const double4>)D.tb, (gptr<double2>)D.parts, D.N,
                            (gptr<const double2>)(MODE == M_EXT ? D.tz : D.eta), MODE == M_EXT ? D.Nt : D.N,
                            rec_stride(wcols), rec32_stride(wcols), wcols, col0,
                            width,
                            w.y * 64 * TPT, w.y, w.z, j0, j1, MIXED ? D.far2 : D.far2d, red);
}

// Far tiles of one item (the items of an M_NEAR launch, 4 or 8 columns) on
// the matrix cores, one slot of 64 targets at a time (an item of 64 TPT
// targets takes TPT passes over its sources). Each wave keeps W and B in the
// MFMA output layout over its far tiles; at the end of a slot it forms
// conj(u) W - B in FP32, the four waves' results meet in LDS in FP64 and the
// threads write the complex outputs to the partial sums (the M_NEAR launch
// that follows adds the near tiles).
template <int NR, int TPT>
__device__ __forceinline__ void far_item(gptr<const double2> eta, gptr<const float2> far32, gptr<const double4> sb,
                                         gptr<const double4> tb, gptr<double2> part, int N,
                                         int wcols, int col0, int width, int base, int tile_idx, int g, int jb0,
                                         int jb1, double far2, double (*fl)[64][17], float* stg) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double4 tbd = tb[tile_idx];
  const double inv_r = 1.0 / tbd.z;
  const float sc = (float)inv_r;
  const int j = lane & 31, h = lane >> 5;
  // the item's 8-column block of the far-tile sources (col0 is a multiple of 8)
  const gptr<const float2> blk = far32 + (size_t)(col0 >> 3) * ((N + 63) / 64) * (kFar32Fields * 64);
  for (int t = 0; t < TPT; ++t) {
    // targets relative to the target tile's centre, over its radius; target
    // 32q + j of the slot is held by the lanes j and j + 32
    float ux[2], uy[2];
    {
      const double2 tg = eta[min(base + t * 64 + lane, N - 1)];
      const float fx = (float)((tg.x - tbd.x) * inv_r), fy = (float)((tg.y - tbd.y) * inv_r);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        ux[q] = __shfl(fx, 32 * q + j, 64);
        uy[q] = __shfl(fy, 32 * q + j, 64);
      }
    }
    f32x16 acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[q][e] = 0.f;
    // the waves take the range's 64-node tiles in turn: near tiles (left to
    // the M_NEAR launch) come in runs, and contiguous quarters of the range
    // would leave some waves idle at the barrier below
    for (int ts = jb0 + 64 * wv; ts < jb1; ts += 256) {
      const int te = min(ts + 64, jb1);
      const double4 sbd = sb[ts >> 6];
      const double dcx = sbd.x - tbd.x, dcy = sbd.y - tbd.y;
      const double rr = tbd.z + sbd.z;
      if ((dcx * dcx + dcy * dcy) > far2 * rr * rr)
        far_tile_mfma<NR>(acc, ux, uy, (float)dcx, (float)dcy, sc, blk + (size_t)(ts >> 6) * (kFar32Fields * 64),
                          te - ts, stg, width);
    }
    // Register e (< 8) holds W and register e + 8 B of component
    // 8(e/4) + 4h + e%4; e even: Re, e + 1: Im of column 4(e/4) + 2h + (e%4)/2.
    // Multiplied by 1/r_t, conj(u) W - B is the sum for the unscaled offsets.
    double F[2][8];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        const float wr = acc[q][e], wi = acc[q][e + 1];
        F[q][e] = (double)__builtin_fmaf(ux[q], wr, __builtin_fmaf(uy[q], wi, -acc[q][e + 8])) * inv_r;
        F[q][e + 1] = (double)__builtin_fmaf(ux[q], wi, __builtin_fmaf(-uy[q], wr, -acc[q][e + 9])) * inv_r;
      }
    // The four waves' sums meet in two rounds through a tile of two waves'
    // sums, which shares its LDS with the staging areas: (w0 + w2) + (w1 + w3).
    // Lane l holds target 32q + j, components 8(e/4) + 4h + e%4 in F[q][e].
    auto slot = [&](int q, int e) -> double& { return fl[0][32 * q + j][8 * (e >> 2) + 4 * h + (e & 3)]; };
    __syncthreads();
    if (wv >= 2) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) (&slot(q, e))[(wv - 2) * 64 * 17] = F[q][e];
    }
    __syncthreads();
    if (wv < 2) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) F[q][e] += (&slot(q, e))[wv * 64 * 17];
    }
    __syncthreads();
    if (wv == 1) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) (&slot(q, e))[64 * 17] = F[q][e];
    }
    __syncthreads();
    if (wv == 0) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int e = 0; e < 8; ++e) slot(q, e) = F[q][e] + (&slot(q, e))[64 * 17];
    }
    __syncthreads();
    // 64 targets x NR complex columns; thread k takes (target k % 64, columns k / 64 + 4 m)
    const int tgt = threadIdx.x & 63;
    const int ti = base + t * 64 + tgt;
#pragma unroll
    for (int m = 0; m < (NR + 3) / 4; ++m) {
      const int cc = (threadIdx.x >> 6) + 4 * m;
      if (cc < width && ti < N) part[((size_t)g * wcols + col0 + cc) * N + ti] = make_double2(fl[0][tgt][2 * cc], fl[0][tgt][2 * cc + 1]);
    }
    __syncthreads();
  }
}

template <int NR, int TPT>
__global__ __launch_bounds__(256) void k_far(const DomDev* __restrict__ doms, const int4* __restrict__ items,
                                             int nitems, int lead, int data, const int* __restrict__ active) {
  // the four waves' staging areas (64 sources x kFarStage floats each) and,
  // after them, the reduction tile (2 x 64 x 17 doubles) share one buffer
  __shared__ double smem[4 * 64 * kFarStage / 2];
  static_assert(2 * 64 * 17 <= 4 * 64 * kFarStage / 2, "the reduction tile exceeds the shared buffer");
  double(*fl)[64][17] = reinterpret_cast<double(*)[64][17]>(smem);
  float* stg = reinterpret_cast<float*>(smem) + (threadIdx.x >> 6) * 64 * kFarStage;
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 w = items[it];
  const DomDev& D = doms[w.x];
  const int wcols = lead + data * D.ncols;
  // first column, and the group's width (an 8-column group padded from fewer
  // columns carries its width in bits 20 and up)
  const int col0 = w.w & 0xFFFFF;
  const int width = (w.w >> 20) ? (w.w >> 20) : NR;
  if (active != nullptr) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int col = col0 + q - lead;
      any = any || (q < width && (col < 0 || active[D.c0 + col] != 0));
    }
    if (!any) return;
  }
  const int chunk = D.chunk;
  const int jb0 = w.z * chunk;
  const int jb1 = min(D.N, jb0 + chunk);
  far_item<NR, TPT>((gptr<const double2>)D.eta, (gptr<const float2>)D.far32, (gptr<const double4>)D.sb,
                    (gptr<const double4>)D.tb, (gptr<double2>)D.parts, D.N, wcols,
                    col0, width, w.y * 64 * TPT, w.y, w.z, jb0, jb1, D.far2, fl, stg);
}

// bounding circle {cx, cy, r, 0} (centre of the bounding box) of tile b of
// `tile` consecutive nodes (which 0, 1, 2: of the nodes into sb, tb, sbf;
// 3: of the target points into tb); one wavefront per (tile, domain)
__device__ __forceinline__ void tile_bounds(const DomDev& D, int tile, int which, int b) {
  const int lane = threadIdx.x;
  const double2* pts = which == 3 ? D.tz : D.eta;
  const int np = which == 3 ? D.Nt : D.N;
  const int i0 = b * tile;
  if (i0 >= np) return;
  const int i1 = min(np, i0 + tile);
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int i = i0 + lane; i < i1; i += 64) {
    const double2 e = pts[i];
    xmin = fmin(xmin, e.x); xmax = fmax(xmax, e.x);
    ymin = fmin(ymin, e.y); ymax = fmax(ymax, e.y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    xmin = fmin(xmin, __shfl_xor(xmin, off, 64));
    xmax = fmax(xmax, __shfl_xor(xmax, off, 64));
    ymin = fmin(ymin, __shfl_xor(ymin, off, 64));
    ymax = fmax(ymax, __shfl_xor(ymax, off, 64));
  }
  const double cx = 0.5 * (xmin + xmax), cy = 0.5 * (ymin + ymax);
  double r = 0.0;
  for (int i = i0 + lane; i < i1; i += 64) {
    const double2 e = pts[i];
    r = fmax(r, sqrt((e.x - cx) * (e.x - cx) + (e.y - cy) * (e.y - cy)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
  // widen by a relative margin so rounding of the centre cannot hide a node
  double4* out = (which == 1 || which == 3) ? D.tb : (which == 2 ? D.sbf : D.sb);
  if (lane == 0) out[b] = make_double4(cx, cy, r * (1.0 + 1e-12) + 1e-300, 0.0);
}

__global__ __launch_bounds__(64) void k_tile_bounds(const DomDev* __restrict__ doms, int tile, int which) {
  tile_bounds(doms[blockIdx.y], tile, which, blockIdx.x);
}

// the three node tilings in one launch (grid.z = which): 64-node source
// tiles, 64 tpt-node target tiles and the far-form tiles of kFarTile nodes
__global__ __launch_bounds__(64) void k_node_tile_bounds(const DomDev* __restrict__ doms, int tpt) {
  const int which = blockIdx.z;
  tile_bounds(doms[blockIdx.y], which == 0 ? 64 : (which == 1 ? 64 * tpt : kFarTile), which, blockIdx.x);
}

// FP32 records {v_j = (eta_j - c_s)/r_s ((c_s, r_s) the node's 64-node tile),
// (|v_j|^2, 0), w_j,q.., b_j,q = w_j,q conj(v_j)..} (stride 2 + 2 wcols) from
// the FP64 records (head, w.., b..), and the far-tile sources of the matrix
// cores (eta_j - c_s unscaled, and the weights by 8-column block)
__global__ void k_records32(const DomDev* __restrict__ doms, int lead, int data) {
  // one thread per (node, weight column), the columns padded to a multiple of
  // 8 where the matrix-core sources are kept, so that the consecutive lanes of
  // a wave read and write consecutive fields
  const DomDev& D = doms[blockIdx.y];
  const int wcols = lead + data * D.ncols;
  const int Q = D.far32 != nullptr ? (wcols + 7) / 8 * 8 : wcols;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)D.N * Q) return;
  const int j = (int)(t / Q), q = (int)(t - (int64_t)j * Q);
  const double2* r = D.rec + (size_t)j * rec_stride(wcols);
  float2* o = D.rec32 + (size_t)j * rec32_stride(wcols);
  const double4 c = D.sb[j >> 6];
  const double dx = r[0].x - c.x, dy = r[0].y - c.y;
  const double inv_r = 1.0 / c.z;
  const float2 vs = make_float2((float)(dx * inv_r), (float)(dy * inv_r));
  const double vx = vs.x, vy = vs.y;
  if (q == 0) {
    o[0] = vs;
    o[1] = make_float2((float)(vx * vx + vy * vy), 0.f);
  }
  float2 w32 = make_float2(0.f, 0.f);
  if (q < wcols) {
    const double2 w = r[kRecHead + q];
    w32 = make_float2((float)w.x, (float)w.y);
    o[2 + q] = w32;
    o[2 + wcols + q] = make_float2((float)(w.x * vx + w.y * vy), (float)(w.y * vx - w.x * vy));
  }
  if (D.far32 != nullptr) {
    const int ntl = (D.N + 63) / 64;
    float2* f = D.far32 + ((size_t)((q >> 3) * ntl + (j >> 6)) * kFar32Fields) * 64 + (j & 63);
    if ((q & 7) == 0) f[0] = make_float2((float)dx, (float)dy);
    f[64 * (1 + (q & 7))] = w32;
  }
}

template <int NR, int TPT, int MODE>
void launch_k(const DomDev* doms, const int4* items, int nitems, int lead, int data, const int* active, int grid,
              hipStream_t st) {
  k_pairs<NR, TPT, MODE><<<grid, 256, 0, st>>>(doms, items, nitems, lead, data, active);
}

// FP64: one launch. Mixed: 1-2 columns in one M_MIXED launch; 4-8 columns as
// k_far then M_NEAR over the same items (the second adds to the first's sums).
template <int NR, int TPT>
void launch_t(const DomDev* doms, const int4* items, int nitems, int lead, int data, bool mixed, bool ext,
              const int* active, int grid, hipStream_t st) {
  if (ext) {
    launch_k<NR, TPT, M_EXT>(doms, items, nitems, lead, data, active, grid, st);
  } else if (!mixed) {
    launch_k<NR, TPT, M_FP64>(doms, items, nitems, lead, data, active, grid, st);
  } else if constexpr (NR >= 4) {
    k_far<NR, TPT><<<grid, 256, 0, st>>>(doms, items, nitems, lead, data, active);
    launch_k<NR, TPT, M_NEAR>(doms, items, nitems, lead, data, active, grid, st);
  } else {
    launch_k<NR, TPT, M_MIXED>(doms, items, nitems, lead, data, active, grid, st);
  }
}

template <int NR>
void launch_w(const DomDev* doms, const int4* items, int nitems, int tpt, int lead, int data, bool mixed, bool ext,
              const int* active, int grid, hipStream_t st) {
  if (tpt == 2) launch_t<NR, 2>(doms, items, nitems, lead, data, mixed, ext, active, grid, st);
  else launch_t<NR, 1>(doms, items, nitems, lead, data, mixed, ext, active, grid, st);
}

template <int NR, int TPT, int MODE>
int occupancy_of() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pairs<NR, TPT, MODE>, 256, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 8;
  }
  return nb;
}

template <int NR, int TPT>
int occupancy_t(bool mixed) {
  if (!mixed) return occupancy_of<NR, TPT, M_FP64>();
  if constexpr (NR >= 4) return occupancy_of<NR, TPT, M_NEAR>();
  return occupancy_of<NR, TPT, M_MIXED>();
}

template <int NR>
int occupancy_w(int tpt, bool mixed) {
  return tpt == 2 ? occupancy_t<NR, 2>(mixed) : occupancy_t<NR, 1>(mixed);
}

}  // namespace

int pairs_blocks_per_cu(int width, int tpt, bool mixed) {
  // resident 256-thread workgroups per CU of each pair-kernel variant (register
  // and LDS limits), cached after the first query
  static int cache[4][2][2] = {};
  const int wi = width >= 8 ? 0 : (width >= 4 ? 1 : (width >= 2 ? 2 : 3));
  const int ti = tpt == 2 ? 1 : 0;
  int& v = cache[wi][ti][mixed ? 1 : 0];
  if (v == 0) {
    switch (wi) {
      case 0: v = occupancy_w<8>(tpt, mixed); break;
      case 1: v = occupancy_w<4>(tpt, mixed); break;
      case 2: v = occupancy_w<2>(tpt, mixed); break;
      default: v = occupancy_w<1>(tpt, mixed); break;
    }
  }
  return v;
}

hipError_t launch_pairs(const DomDev* doms, const int4* items, int nitems, int width, int tpt, int lead, int data,
                        bool mixed, bool ext, const int* active, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (ext && mixed) return hipErrorInvalidValue;
  const int grid = nitems;
  switch (width) {
    case 8: launch_w<8>(doms, items, nitems, tpt, lead, data, mixed, ext, active, grid, st); break;
    case 4: launch_w<4>(doms, items, nitems, tpt, lead, data, mixed, ext, active, grid, st); break;
    case 2: launch_w<2>(doms, items, nitems, tpt, lead, data, mixed, ext, active, grid, st); break;
    default: launch_w<1>(doms, items, nitems, tpt, lead, data, mixed, ext, active, grid, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_tile_bounds(const DomDev* doms, int ndom, int maxN, int tile, int which, hipStream_t st) {
  dim3 grid((unsigned)((maxN + tile - 1) / tile), (unsigned)ndom);
  k_tile_bounds<<<grid, 64, 0, st>>>(doms, tile, which);
  return hipGetLastError();
}

hipError_t launch_node_tile_bounds(const DomDev* doms, int ndom, int maxN, int tpt, hipStream_t st) {
  // the 64-node tiling has the most tiles
  dim3 grid((unsigned)((maxN + 63) / 64), (unsigned)ndom, 3);
  k_node_tile_bounds<<<grid, 64, 0, st>>>(doms, tpt);
  return hipGetLastError();
}

hipError_t launch_records32(const DomDev* doms, int ndom, int64_t threads, int lead, int data, hipStream_t st) {
  dim3 grid((unsigned)((threads + 255) / 256), (unsigned)ndom);
  k_records32<<<grid, 256, 0, st>>>(doms, lead, data);
  return hipGetLastError();
}

}  // namespace gnk
