// Direct Cauchy sum on gfx950 (FP64):
//   S_i = sum_{j != i} w_j / (eta_i - eta_j)          (matrix E of eq. (e:fmm-E))
// for several weight columns w at once. This single product carries every
// operator of the method: Im and Re of A_i S_i give B x and D x
// (eqs. (e:(I-B)x), (e:hD-bt)); (eta'/A) S with w = A x gives B^T x
// (eq. (e:BTx)); w = eta' gives the vector e (eq. (e:bve)).
//
// Mapping (VALU-bound, no matrix cores: every pair needs its own reciprocal):
//   * sources are packed records {eta_j, w_j,0 .. w_j,ncols-1} (16 B each
//     field); the source loop index is wave-uniform, so whole records arrive
//     with wide scalar loads into SGPRs and are broadcast to all lanes (no LDS
//     traffic, no bank conflicts); four sources are fetched per iteration so
//     one wait covers four reciprocals;
//   * each lane owns TPT target nodes (a tile of TPT*64 consecutive targets),
//     which reuses every fetched source TPT times and gives independent chains;
//   * the four wavefronts of a workgroup share the tile and split its source
//     chunk four ways, then add their sums through LDS in wave order;
//   * the work is a list of items (domain, target tile, source split, column
//     group) covering every domain of a batch in one launch per column-group
//     width, one workgroup per item (largest domains first); the consumer
//     adds the split partial sums in a fixed order, so results are bitwise
//     reproducible;
//   * 1/|d|^2 comes from v_rcp_f64 refined by one Newton step; two sources
//     share one reciprocal: 1/a = b/(ab), 1/b = a/(ab) (simultaneous
//     inversion), which halves the v_rcp_f64 issues;
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

template <int NR, int TPT>
struct Acc {
  double x[TPT][NR];
  double y[TPT][NR];
};

// acc[t] += w * q for NR columns, q = conj(d)/|d|^2 = (qx, qy)
template <int NR, int TPT, class P>
__device__ __forceinline__ void accumulate(Acc<NR, TPT>& a, int t, P wj, double qx, double qy) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double2 w = wj[r];
    a.x[t][r] = __builtin_fma(w.x, qx, a.x[t][r]);
    a.x[t][r] = __builtin_fma(-w.y, qy, a.x[t][r]);
    a.y[t][r] = __builtin_fma(w.x, qy, a.y[t][r]);
    a.y[t][r] = __builtin_fma(w.y, qx, a.y[t][r]);
  }
}

// two sources a, b (records ra, rb) against every target of the lane
// ra, rb: source records (eta at [0]); the launch's weight columns start at [wo]
template <int NR, int TPT, class P>
__device__ __forceinline__ void pair_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], P ra, P rb, int wo) {
  const double2 ea = ra[0], eb = rb[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double dxa = tg[t].x - ea.x, dya = tg[t].y - ea.y;
    const double dxb = tg[t].x - eb.x, dyb = tg[t].y - eb.y;
    const double da = __builtin_fma(dya, dya, dxa * dxa);
    const double db = __builtin_fma(dyb, dyb, dxb * dxb);
    const double R = refine_rcp(da * db);
    const double qa = db * R, qb = da * R;
    accumulate<NR, TPT>(acc, t, ra + wo, dxa * qa, -dya * qa);
    accumulate<NR, TPT>(acc, t, rb + wo, dxb * qb, -dyb * qb);
  }
}

// four sources a..d against every target of the lane, one reciprocal for all
// four: with R = 1/(|da|^2 |db|^2 |dc|^2 |dd|^2), 1/|da|^2 = R |db|^2 (|dc|^2 |dd|^2)
// and so on (the product stays in range while every distance lies in
// [1e-38, 1e38])
template <int NR, int TPT, class P>
__device__ __forceinline__ void quad_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], P ra, P rb, P rc, P rd,
                                          int wo) {
  const double2 ea = ra[0], eb = rb[0], ec = rc[0], ed = rd[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double dxa = tg[t].x - ea.x, dya = tg[t].y - ea.y;
    const double dxb = tg[t].x - eb.x, dyb = tg[t].y - eb.y;
    const double dxc = tg[t].x - ec.x, dyc = tg[t].y - ec.y;
    const double dxd = tg[t].x - ed.x, dyd = tg[t].y - ed.y;
    const double da = __builtin_fma(dya, dya, dxa * dxa);
    const double db = __builtin_fma(dyb, dyb, dxb * dxb);
    const double dc = __builtin_fma(dyc, dyc, dxc * dxc);
    const double dd = __builtin_fma(dyd, dyd, dxd * dxd);
    const double ab = da * db, cd = dc * dd;
    const double R = refine_rcp(ab * cd);
    const double Rab = R * cd, Rcd = R * ab;
    const double qa = db * Rab, qb = da * Rab, qc = dd * Rcd, qd = dc * Rcd;
    accumulate<NR, TPT>(acc, t, ra + wo, dxa * qa, -dya * qa);
    accumulate<NR, TPT>(acc, t, rb + wo, dxb * qb, -dyb * qb);
    accumulate<NR, TPT>(acc, t, rc + wo, dxc * qc, -dyc * qc);
    accumulate<NR, TPT>(acc, t, rd + wo, dxd * qd, -dyd * qd);
  }
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void single_step(Acc<NR, TPT>& acc, const double2 (&tg)[TPT], const int (&ti)[TPT], P rj,
                                            int wo, int j, bool masked) {
  const double2 e = rj[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const double dx = tg[t].x - e.x, dy = tg[t].y - e.y;
    double r = refine_rcp(__builtin_fma(dy, dy, dx * dx));
    if (masked) r = (j == ti[t]) ? 0.0 : r;
    accumulate<NR, TPT>(acc, t, rj + wo, dx * r, -dy * r);
  }
}

// ---------------------------------------------------------------------------
// Mixed precision: well-separated source tiles in FP32, the rest in FP64.
// A source tile is 64 consecutive nodes with bounding circle (c_s, r_s); the
// workgroup's target tile has (c_t, r_t). The tile pair is far when
// |c_t - c_s| > (1 + theta)(r_t + r_s). For a far tile every lane forms
// u = (eta_i - c_s) in FP64 and rounds it to FP32; the records hold
// v_j = (eta_j - c_s) in FP32, so d = u - v keeps a relative error of a few
// FP32 ulps however far the tiles are from the origin. The tile's 64 terms
// are summed in FP32 and added to the FP64 accumulators.
template <int NR, int TPT>
struct Acc32 {
  float x[TPT][NR];
  float y[TPT][NR];
};

template <int NR, int TPT, class P>
__device__ __forceinline__ void accumulate32(Acc32<NR, TPT>& a, int t, P wj, float qx, float qy) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const float2 w = wj[r];
    a.x[t][r] = __builtin_fmaf(w.x, qx, a.x[t][r]);
    a.x[t][r] = __builtin_fmaf(-w.y, qy, a.x[t][r]);
    a.y[t][r] = __builtin_fmaf(w.x, qy, a.y[t][r]);
    a.y[t][r] = __builtin_fmaf(w.y, qx, a.y[t][r]);
  }
}

template <int NR, int TPT, class P>
__device__ __forceinline__ void pair_step32(Acc32<NR, TPT>& acc, const float2 (&u)[TPT], P ra, P rb, int wo) {
  const float2 ea = ra[0], eb = rb[0];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    const float dxa = u[t].x - ea.x, dya = u[t].y - ea.y;
    const float dxb = u[t].x - eb.x, dyb = u[t].y - eb.y;
    const float da = __builtin_fmaf(dya, dya, dxa * dxa);
    const float db = __builtin_fmaf(dyb, dyb, dxb * dxb);
    const float R = __builtin_amdgcn_rcpf(da * db);
    const float qa = db * R, qb = da * R;
    accumulate32<NR, TPT>(acc, t, ra + wo, dxa * qa, -dya * qa);
    accumulate32<NR, TPT>(acc, t, rb + wo, dxb * qb, -dyb * qb);
  }
}

// One work item: the tile of 64*TPT targets starting at `base`, sources
// [jb0, jb1) of the domain, weight columns wo-1 .. wo-1+NR-1. The four
// wavefronts of the workgroup take consecutive quarters of the sources; their
// sums are added through LDS in wave order. MIXED: far source tiles of 64
// nodes are summed in FP32 (see above). All pointers are restrict-qualified
// parameters, so after inlining the record loads are known not to alias the
// partial-sum stores and stay scalar (wave-uniform) loads.
template <int NR, int TPT, bool MIXED>
__device__ __forceinline__ void pair_item(gptr<const double2> rec, gptr<const float2> rec32, gptr<const double4> sb,
                                          gptr<const double4> tb, gptr<double2> part, int N, int stride, int wcols, int wo,
                                          int base, int tile_idx, int g, int jb0, int jb1, int wchunk, double far2,
                                          double (&red)[3][TPT][2][64]) {
  constexpr int kTile = 64 * TPT;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int j0 = min(jb1, jb0 + wv * wchunk);
  const int j1 = min(jb1, j0 + wchunk);

  double2 tg[TPT];
  int ti[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    ti[t] = base + t * 64 + lane;
    tg[t] = rec[(size_t)min(ti[t], N - 1) * stride];
  }
  Acc<NR, TPT> acc;
#pragma unroll
  for (int t = 0; t < TPT; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) { acc.x[t][r] = 0.0; acc.y[t][r] = 0.0; }

  // sources outside the tile's own window need no j != i test
  auto plain = [&](int ja, int jb) {
    int j = ja;
    for (; j + 3 < jb; j += 4) {
      gptr<const double2> r = rec + (size_t)j * stride;
      if constexpr (NR <= 2) {
        quad_step<NR, TPT>(acc, tg, r, r + stride, r + 2 * stride, r + 3 * stride, wo);
      } else {
        // four wide records would not fit in scalar registers together
        pair_step<NR, TPT>(acc, tg, r, r + stride, wo);
        pair_step<NR, TPT>(acc, tg, r + 2 * stride, r + 3 * stride, wo);
      }
    }
    for (; j + 1 < jb; j += 2) {
      gptr<const double2> r = rec + (size_t)j * stride;
      pair_step<NR, TPT>(acc, tg, r, r + stride, wo);
    }
    if (j < jb) single_step<NR, TPT>(acc, tg, ti, rec + (size_t)j * stride, wo, j, false);
  };
  auto fp64_range = [&](int ja, int jb) {
    plain(ja, min(jb, base));
    const int ma = max(ja, base), mb = min(jb, base + kTile);
    for (int j = ma; j < mb; ++j) single_step<NR, TPT>(acc, tg, ti, rec + (size_t)j * stride, wo, j, true);
    plain(max(ja, base + kTile), jb);
  };

  if (!MIXED) {
    fp64_range(j0, j1);
  } else {
    const double4 tbd = tb[tile_idx];
    for (int ts = j0; ts < j1; ts += 64) {
      const int te = min(ts + 64, j1);
      const double4 sbd = sb[ts >> 6];
      const double dcx = tbd.x - sbd.x, dcy = tbd.y - sbd.y;
      const double rr = tbd.z + sbd.z;
      if ((dcx * dcx + dcy * dcy) > far2 * rr * rr) {
        float2 u[TPT];
#pragma unroll
        for (int t = 0; t < TPT; ++t) u[t] = make_float2((float)(tg[t].x - sbd.x), (float)(tg[t].y - sbd.y));
        Acc32<NR, TPT> a32;
#pragma unroll
        for (int t = 0; t < TPT; ++t)
#pragma unroll
          for (int r = 0; r < NR; ++r) { a32.x[t][r] = 0.f; a32.y[t][r] = 0.f; }
        int j = ts;
#pragma unroll 2
        for (; j + 1 < te; j += 2) {
          gptr<const float2> r = rec32 + (size_t)j * stride;
          pair_step32<NR, TPT>(a32, u, r, r + stride, wo);
        }
        if (j < te) {
          gptr<const float2> r = rec32 + (size_t)j * stride;
          const float2 e = r[0];
#pragma unroll
          for (int t = 0; t < TPT; ++t) {
            const float dx = u[t].x - e.x, dy = u[t].y - e.y;
            const float q = __builtin_amdgcn_rcpf(__builtin_fmaf(dy, dy, dx * dx));
            accumulate32<NR, TPT>(a32, t, r + wo, dx * q, -dy * q);
          }
        }
#pragma unroll
        for (int t = 0; t < TPT; ++t)
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            acc.x[t][r] += (double)a32.x[t][r];
            acc.y[t][r] += (double)a32.y[t][r];
          }
      } else {
        fp64_range(ts, te);
      }
    }
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
        if (ti[t] < N) part[((size_t)g * wcols + wo - 1 + r) * N + ti[t]] = make_double2(x, y);
      }
    }
    __syncthreads();
  }
}

// One launch: one workgroup per item of the list. (A workgroup that looped
// over several items would store partial sums before loading the next item's
// records, and the records could then no longer be fetched with scalar loads.)
// Variants with one or two columns are held to 64 VGPRs (8 waves per SIMD),
// which they reach without spilling; wider ones keep their registers.
template <int NR, int TPT, bool MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NR <= 2 ? 8 : 1))) void k_pairs(const DomDev* __restrict__ doms, const int4* __restrict__ items,
                                               int nitems, int lead, int data, const int* __restrict__ active) {
  __shared__ double red[3][TPT][2][64];
  const int it = blockIdx.x;
  if (it >= nitems) return;
  const int4 w = items[it];
  const DomDev& D = doms[w.x];
  const int wcols = lead + data * D.ncols;
  if (active != nullptr) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int col = w.w + q - lead;
      any = any || col < 0 || active[D.c0 + col] != 0;
    }
    if (!any) return;
  }
  const int chunk = D.chunk;
  const int jb0 = w.z * chunk;
  const int jb1 = min(D.N, jb0 + chunk);
  // quarter of the chunk per wave: multiple of 4 (FP64) or whole 64-node tiles (mixed)
  const int wchunk = MIXED ? (chunk >> 2) : (((chunk + 15) >> 4) << 2);
  pair_item<NR, TPT, MIXED>((gptr<const double2>)D.rec, (gptr<const float2>)D.rec32, (gptr<const double4>)D.sb,
                            (gptr<const double4>)D.tb, (gptr<double2>)D.parts, D.N, wcols + 1, wcols, 1 + w.w, w.y * 64 * TPT,
                            w.y, w.z, jb0, jb1, wchunk, D.far2, red);
}

// bounding circle {cx, cy, r, 0} (centre of the bounding box) of each tile of
// `tile` consecutive nodes; one wavefront per (tile, domain)
__global__ __launch_bounds__(64) void k_tile_bounds(const DomDev* __restrict__ doms, int tile, int target) {
  const DomDev& D = doms[blockIdx.y];
  const int b = blockIdx.x, lane = threadIdx.x;
  const int i0 = b * tile;
  if (i0 >= D.N) return;
  const int i1 = min(D.N, i0 + tile);
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int i = i0 + lane; i < i1; i += 64) {
    const double2 e = D.eta[i];
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
    const double2 e = D.eta[i];
    r = fmax(r, sqrt((e.x - cx) * (e.x - cx) + (e.y - cy) * (e.y - cy)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
  // widen by a relative margin so rounding of the centre cannot hide a node
  if (lane == 0) (target ? D.tb : D.sb)[b] = make_double4(cx, cy, r * (1.0 + 1e-12) + 1e-300, 0.0);
}

// FP32 records: v_j = eta_j - c_{tile(j)}, then the weights rounded to FP32
__global__ void k_records32(const DomDev* __restrict__ doms, int lead, int data) {
  const DomDev& D = doms[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.N) return;
  const int stride = lead + data * D.ncols + 1;
  const double2* r = D.rec + (size_t)j * stride;
  float2* o = D.rec32 + (size_t)j * stride;
  const double4 c = D.sb[j >> 6];
  o[0] = make_float2((float)(r[0].x - c.x), (float)(r[0].y - c.y));
  for (int q = 1; q < stride; ++q) o[q] = make_float2((float)r[q].x, (float)r[q].y);
}

template <int NR, int TPT, bool MIXED>
void launch_k(const DomDev* doms, const int4* items, int nitems, int lead, int data, const int* active, int grid,
              hipStream_t st) {
  k_pairs<NR, TPT, MIXED><<<grid, 256, 0, st>>>(doms, items, nitems, lead, data, active);
}

template <int NR>
void launch_w(const DomDev* doms, const int4* items, int nitems, int tpt, int lead, int data, bool mixed,
              const int* active, int grid, hipStream_t st) {
  if (tpt == 2) {
    if (mixed) launch_k<NR, 2, true>(doms, items, nitems, lead, data, active, grid, st);
    else launch_k<NR, 2, false>(doms, items, nitems, lead, data, active, grid, st);
  } else {
    if (mixed) launch_k<NR, 1, true>(doms, items, nitems, lead, data, active, grid, st);
    else launch_k<NR, 1, false>(doms, items, nitems, lead, data, active, grid, st);
  }
}


template <int NR, int TPT, bool MIXED>
int occupancy_of() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_pairs<NR, TPT, MIXED>, 256, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 8;
  }
  return nb;
}

template <int NR>
int occupancy_w(int tpt, bool mixed) {
  if (tpt == 2) return mixed ? occupancy_of<NR, 2, true>() : occupancy_of<NR, 2, false>();
  return mixed ? occupancy_of<NR, 1, true>() : occupancy_of<NR, 1, false>();
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
                        bool mixed, const int* active, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  const int grid = nitems;
  switch (width) {
    case 8: launch_w<8>(doms, items, nitems, tpt, lead, data, mixed, active, grid, st); break;
    case 4: launch_w<4>(doms, items, nitems, tpt, lead, data, mixed, active, grid, st); break;
    case 2: launch_w<2>(doms, items, nitems, tpt, lead, data, mixed, active, grid, st); break;
    default: launch_w<1>(doms, items, nitems, tpt, lead, data, mixed, active, grid, st); break;
  }
  return hipGetLastError();
}

hipError_t launch_tile_bounds(const DomDev* doms, int ndom, int maxN, int tile, bool target, hipStream_t st) {
  dim3 grid((unsigned)((maxN + tile - 1) / tile), (unsigned)ndom);
  k_tile_bounds<<<grid, 64, 0, st>>>(doms, tile, target ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_records32(const DomDev* doms, int ndom, int maxN, int lead, int data, hipStream_t st) {
  dim3 grid((unsigned)((maxN + 255) / 256), (unsigned)ndom);
  k_records32<<<grid, 256, 0, st>>>(doms, lead, data);
  return hipGetLastError();
}

}  // namespace gnk
