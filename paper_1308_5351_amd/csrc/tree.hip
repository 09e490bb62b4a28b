// Far-field compression of the Cauchy sums S_i = sum_{j != i} w_j/(eta_i - eta_j)
// for large N (the paper evaluates these sums with a fast multipole method;
// this is a treecode on the GPU, FP64 throughout):
//   * boxes: level 0 holds the leaves of kLeaf = 256 consecutive nodes (the
//     node order follows the boundary curves, so a range of nodes is compact),
//     level l + 1 pairs the boxes of level l; each box has a bounding circle;
//   * multipole moments of box b about its centre c_b, for one weight column:
//     a_k = sum_{j in b} w_j (eta_j - c_b)^k, k < p; leaves from their nodes,
//     parents from their children by the binomial shift;
//   * a far box contributes sum_{k<p} a_k u^{k+1}, u = 1/(z - c_b), to a
//     target z: the expansion of 1/(z - eta_j) in powers of (eta_j - c_b)/(z - c_b),
//     truncated with error below (r_b/|z - c_b|)^p times sum |w_j|/(|z - c_b| - r_b);
//   * every other source is summed directly, in blocks of 64 nodes, by the
//     FP64 pair loops (j != i excluded);
//   * the interaction lists (far boxes and near blocks per target tile) come
//     from the host; each (target tile, split) workgroup takes four
//     cost-balanced ranges of its tile's list, one per wavefront, and writes
//     one partial sum, which the consumer adds in split order like those of
//     the direct kernels.
#include <algorithm>
#include <cmath>

#include "gnk_device.h"
#include "gnk_internal.h"

namespace gnk {

namespace {

#include "pair_steps.inl"

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Bounding circles {cx, cy, r, 0} of the boxes of every level: the centre of
// the box's bounding box and the largest distance of its nodes from it. The
// leaves (256 consecutive nodes) take the slots of level 0 in an order chosen
// on the host (perm: slot -> leaf, invp: leaf -> slot); the box of slots
// [b 2^l, (b + 1) 2^l) is box b of level l. Leaf bounding boxes come from
// their nodes (one wavefront per leaf), a parent's from its two children
// (exact: min and max), and the radii of all levels from one pass over the
// nodes (one 256-thread block per leaf, whose nodes lie in a single box of
// every level; a block maximum, then an atomic maximum on the radius's bit
// pattern, which orders non-negative doubles as unsigned integers).
__global__ __launch_bounds__(64) void k_leaf_bbox(const double2* __restrict__ eta, int N,
                                                  double4* __restrict__ bbox) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const int i0 = b * kLeaf;
  if (i0 >= N) return;
  const int i1 = min(N, i0 + kLeaf);
  double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
  for (int i = i0 + lane; i < i1; i += 64) {
    const double2 e = eta[i];
    xmin = fmin(xmin, e.x);
    xmax = fmax(xmax, e.x);
    ymin = fmin(ymin, e.y);
    ymax = fmax(ymax, e.y);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    xmin = fmin(xmin, __shfl_xor(xmin, off, 64));
    xmax = fmax(xmax, __shfl_xor(xmax, off, 64));
    ymin = fmin(ymin, __shfl_xor(ymin, off, 64));
    ymax = fmax(ymax, __shfl_xor(ymax, off, 64));
  }
  if (lane == 0) bbox[b] = make_double4(xmin, xmax, ymin, ymax);
}

__global__ void k_bbox_gather(const double4* __restrict__ leafbox, const int* __restrict__ perm, int nleaf,
                              double4* __restrict__ slotbox) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nleaf) slotbox[s] = leafbox[perm[s]];
}

__global__ void k_bbox_merge(const double4* __restrict__ child, int nchild, double4* __restrict__ parent, int npar) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= npar) return;
  double4 v = child[2 * b];
  if (2 * b + 1 < nchild) {
    const double4 u = child[2 * b + 1];
    v = make_double4(fmin(v.x, u.x), fmax(v.y, u.y), fmin(v.z, u.z), fmax(v.w, u.w));
  }
  parent[b] = v;
}

// centres of all boxes; radii (as bits) cleared for the maximum that follows
__global__ void k_box_centres(const double4* __restrict__ bbox, int nbox, double4* __restrict__ out,
                              unsigned long long* __restrict__ rbits) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  const double4 v = bbox[b];
  out[b] = make_double4(0.5 * (v.x + v.y), 0.5 * (v.z + v.w), 0.0, 0.0);
  rbits[b] = 0ull;
}

struct LevelTable {
  int off[32];   // first box of each level
  int nb[32];    // boxes of each level
};

__global__ __launch_bounds__(256) void k_box_radii(const double2* __restrict__ eta, int N, LevelTable lv, int levels,
                                                   const int* __restrict__ invp, const double4* __restrict__ out,
                                                   unsigned long long* __restrict__ rbits) {
  __shared__ double sh[4];
  const int leaf = blockIdx.x, t = threadIdx.x;
  const int slot = invp[leaf];
  const int i = leaf * kLeaf + t;
  const bool in = i < N;
  const double2 e = in ? eta[i] : make_double2(0.0, 0.0);
  for (int l = 0; l < levels; ++l) {
    const int box = lv.off[l] + (slot >> l);
    const double4 c = out[box];
    double r = in ? sqrt((e.x - c.x) * (e.x - c.x) + (e.y - c.y) * (e.y - c.y)) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
    if ((t & 63) == 0) sh[t >> 6] = r;
    __syncthreads();
    if (t == 0)
      atomicMax(rbits + box, (unsigned long long)__double_as_longlong(fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]))));
    __syncthreads();
  }
}

// widen by a relative margin so rounding of the centre cannot hide a node
__global__ void k_box_finish(const unsigned long long* __restrict__ rbits, int nbox, double4* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbox) return;
  const double r = __longlong_as_double((long long)rbits[b]);
  out[b].z = r * (1.0 + 1e-12) + 1e-300;
}

// Leaf moments of weight column wo (record field) about the leaf centres:
// one wavefront per level-0 slot (leaf perm[slot]), each lane holding up to four nodes; moment k is
// the wave sum of w_j (eta_j - c)^k, the powers advanced one k at a time.
__global__ __launch_bounds__(64) void k_leaf_moments(const double2* __restrict__ rec, int stride, int wo, int N,
                                                     const double4* __restrict__ bounds, const int* __restrict__ perm,
                                                     int p, double2* __restrict__ mom) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const int leaf = perm[b];
  const double4 c = bounds[b];
  double dx[kLeaf / 64], dy[kLeaf / 64], tx[kLeaf / 64], ty[kLeaf / 64];
#pragma unroll
  for (int m = 0; m < kLeaf / 64; ++m) {
    const int j = leaf * kLeaf + m * 64 + lane;
    if (j < N) {
      const double2 e = rec[(size_t)j * stride], w = rec[(size_t)j * stride + wo];
      dx[m] = e.x - c.x;
      dy[m] = e.y - c.y;
      tx[m] = w.x;
      ty[m] = w.y;
    } else {
      dx[m] = dy[m] = tx[m] = ty[m] = 0.0;
    }
  }
  for (int k = 0; k < p; ++k) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int m = 0; m < kLeaf / 64; ++m) {
      sx += tx[m];
      sy += ty[m];
      const double nx = tx[m] * dx[m] - ty[m] * dy[m];
      ty[m] = tx[m] * dy[m] + ty[m] * dx[m];
      tx[m] = nx;
    }
    sx = wave_sum64(sx);
    sy = wave_sum64(sy);
    if (lane == 0) mom[(size_t)b * p + k] = make_double2(sx, sy);
  }
}

// Moments of levels l0 + 1 .. l0 + nlev from those of level l0 in one launch:
// a_k(parent) = sum over its two children sum_{q <= k} C(k, q) a_q(child) d^(k-q),
// d = c_child - c_parent. One workgroup per box B of level l0 + nlev takes the
// boxes of its subtree level by level (at most 2^kM2MLevels of the lowest),
// the children's moments of each level in LDS, one thread per (parent, k).
// C(k, q) comes from a table that the workgroup fills first (integers below
// 2^53, exact). Each parent's sums run in the same order whatever the
// grouping of levels.
constexpr int kM2MLevels = 4;
constexpr int kM2MThreads = 512;

__global__ __launch_bounds__(kM2MThreads) void k_m2m_levels(const double4* __restrict__ bounds, LevelTable lt,
                                                            int l0, int nlev, int p, double2* __restrict__ mom) {
  __shared__ double2 sm[2][(1 << kM2MLevels) * kTreeMaxP];
  __shared__ double binom[kTreeMaxP][kTreeMaxP];
  const int B = blockIdx.x;
  for (int k = threadIdx.x; k < p; k += blockDim.x) {
    double c = 1.0;   // C(k, k), then C(k, q - 1) from C(k, q)
    for (int q = k; q >= 0; --q) {
      binom[k][q] = c;
      c = c * (double)q / (double)(k - q + 1);
    }
  }
  int c0 = B << nlev;   // first box of the subtree at the child level
  int cnt = min(lt.nb[l0] - c0, 1 << nlev);
  for (int i = threadIdx.x; i < cnt * p; i += blockDim.x) sm[0][i] = mom[(size_t)(lt.off[l0] + c0) * p + i];
  __syncthreads();
  int cur = 0;
  for (int lev = 1; lev <= nlev; ++lev) {
    const int l = l0 + lev;
    const int p0 = B << (nlev - lev);
    const int np = min(lt.nb[l] - p0, 1 << (nlev - lev));
    for (int tid = threadIdx.x; tid < np * p; tid += blockDim.x) {
      const int b = tid / p, k = tid - b * p;
      const double4 cp = bounds[lt.off[l] + p0 + b];
      double ax = 0.0, ay = 0.0;
      for (int ch = 2 * b; ch < min(2 * b + 2, cnt); ++ch) {
        const double4 cc = bounds[lt.off[l - 1] + c0 + ch];
        const double ddx = cc.x - cp.x, ddy = cc.y - cp.y;
        const double2* a = &sm[cur][ch * p];
        double px = 1.0, py = 0.0;
        for (int q = k; q >= 0; --q) {
          const double2 aq = a[q];
          const double tx = aq.x * px - aq.y * py, ty = aq.x * py + aq.y * px;
          ax = __builtin_fma(binom[k][q], tx, ax);
          ay = __builtin_fma(binom[k][q], ty, ay);
          const double nx = px * ddx - py * ddy;
          py = px * ddy + py * ddx;
          px = nx;
        }
      }
      sm[cur ^ 1][b * p + k] = make_double2(ax, ay);
      mom[(size_t)(lt.off[l] + p0 + b) * p + k] = make_double2(ax, ay);
    }
    __syncthreads();
    cur ^= 1;
    c0 = p0;
    cnt = np;
  }
}

// One workgroup per (target tile, split): wave wv takes the entries
// [seg[4 split + wv], seg[4 split + wv + 1]) of its tile's list. Entries >= 0
// are far boxes: global index in bits 0..23, the number of terms this box
// needs for this tile in bits 24..29; entries < 0 are near blocks ~blk of 64
// nodes.
// Partial sums of weight column col go to slot split, like the direct kernels'.
template <int TPT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_tree(const DomDev* __restrict__ doms, const int* __restrict__ seg,
                                              const int* __restrict__ list, const double4* __restrict__ bounds,
                                              const double2* __restrict__ mom, int p, int splits, int col, int wcols,
                                              const int* __restrict__ active, int lead, int ext) {
  __shared__ double red[3][TPT][2][64];
  constexpr int kTile = 64 * TPT;
  const DomDev& D = doms[0];
  if (active != nullptr && col >= lead && active[D.c0 + col - lead] == 0) return;
  const int N = D.N;
  const int NT = ext ? D.Nt : N;   // targets: the points tz (ext) or the nodes
  const int tile = blockIdx.x / splits, g = blockIdx.x - tile * splits;
  const int base = tile * kTile;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int stride = rec_stride(wcols);
  const int wo = kRecHead + col;
  const gptr<const double2> rec = (gptr<const double2>)D.rec;
  const gptr<const int> sg = (gptr<const int>)seg + (size_t)tile * (4 * splits + 1) + 4 * g + wv;
  const int e0 = __builtin_amdgcn_readfirstlane(sg[0]);
  const int e1 = __builtin_amdgcn_readfirstlane(sg[1]);

  double2 tg[TPT];
  int ti[TPT];
#pragma unroll
  for (int t = 0; t < TPT; ++t) {
    ti[t] = base + t * 64 + lane;
    tg[t] = ext ? D.tz[min(ti[t], NT - 1)] : D.eta[min(ti[t], N - 1)];
  }
  Acc<1, TPT> acc;
#pragma unroll
  for (int t = 0; t < TPT; ++t) acc.x[t][0] = acc.y[t][0] = 0.0;

  auto plain = [&](int ja, int jb) {
    int j = ja;
    for (; j + 3 < jb; j += 4) {
      gptr<const double2> r = rec + (size_t)j * stride;
      quad_step<1, TPT>(acc, tg, r, r + stride, r + 2 * stride, r + 3 * stride, wo);
    }
    for (; j + 1 < jb; j += 2) {
      gptr<const double2> r = rec + (size_t)j * stride;
      pair_step<1, TPT>(acc, tg, r, r + stride, wo);
    }
    if (j < jb) single_step<1, TPT>(acc, tg, ti, rec + (size_t)j * stride, wo, j, false);
  };

  const gptr<const int> ls = (gptr<const int>)list;
  const gptr<const double4> bd = (gptr<const double4>)bounds;
  const gptr<const double2> mm = (gptr<const double2>)mom;
  for (int e = e0; e < e1; ++e) {
    const int ent = ls[e];
    if (ent >= 0) {
      const int box = ent & 0xFFFFFF, pe = ent >> 24;
      const double4 c = bd[box];
      const gptr<const double2> a = mm + (size_t)box * p;
      // Horner in u = 1/(z - c) for every target at once: each moment is loaded
      // once for the TPT targets, four at a time
      double ux[TPT], uy[TPT], sx[TPT], sy[TPT];
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        const double dx = tg[t].x - c.x, dy = tg[t].y - c.y;
        const double inv = refine_rcp(__builtin_fma(dy, dy, dx * dx));
        ux[t] = dx * inv;
        uy[t] = -dy * inv;
        sx[t] = 0.0;
        sy[t] = 0.0;
      }
      auto horner = [&](double2 ak) {
#pragma unroll
        for (int t = 0; t < TPT; ++t) {
          const double nx = __builtin_fma(ux[t], sx[t], __builtin_fma(-uy[t], sy[t], ak.x));
          sy[t] = __builtin_fma(ux[t], sy[t], __builtin_fma(uy[t], sx[t], ak.y));
          sx[t] = nx;
        }
      };
      int k = pe - 1;
      for (; k >= 3; k -= 4) {
        const double2 a0 = a[k], a1 = a[k - 1], a2 = a[k - 2], a3 = a[k - 3];
        horner(a0);
        horner(a1);
        horner(a2);
        horner(a3);
      }
      for (; k >= 0; --k) horner(a[k]);
#pragma unroll
      for (int t = 0; t < TPT; ++t) {
        acc.x[t][0] += ux[t] * sx[t] - uy[t] * sy[t];
        acc.y[t][0] += ux[t] * sy[t] + uy[t] * sx[t];
      }
    } else {
      const int ja = (~ent) * 64, jb = min(N, ja + 64);
      if (ext) {
        plain(ja, jb);
        continue;
      }
      plain(ja, min(jb, base));
      const int ma = max(ja, base), mb = min(jb, base + kTile);
      for (int j = ma; j < mb; ++j) single_step<1, TPT>(acc, tg, ti, rec + (size_t)j * stride, wo, j, true);
      plain(max(ja, base + kTile), jb);
    }
  }

  // fixed-order reduction over the four wavefronts
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      red[wv - 1][t][0][lane] = acc.x[t][0];
      red[wv - 1][t][1][lane] = acc.y[t][0];
    }
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int t = 0; t < TPT; ++t) {
      double x = acc.x[t][0], y = acc.y[t][0];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        x += red[q][t][0][lane];
        y += red[q][t][1][lane];
      }
      if (ti[t] < NT) D.parts[((size_t)g * wcols + col) * NT + ti[t]] = make_double2(x, y);
    }
  }
}

}  // namespace

hipError_t launch_leaf_boxes(const double2* eta, int N, int nleaf, double4* leafbox, hipStream_t st) {
  k_leaf_bbox<<<nleaf, 64, 0, st>>>(eta, N, leafbox);
  return hipGetLastError();
}

hipError_t launch_box_bounds(const double2* eta, int N, const int* level_off, const int* level_nb, int levels,
                             const double4* leafbox, const int* perm, const int* invp, double4* bbox,
                             unsigned long long* rbits, double4* out, hipStream_t st) {
  if (levels < 1 || levels > 32) return hipErrorInvalidValue;
  k_bbox_gather<<<(level_nb[0] + 255) / 256, 256, 0, st>>>(leafbox, perm, level_nb[0], bbox);
  hipError_t e = hipGetLastError();
  for (int l = 0; l + 1 < levels && e == hipSuccess; ++l) {
    const int npar = level_nb[l + 1];
    k_bbox_merge<<<(npar + 255) / 256, 256, 0, st>>>(bbox + level_off[l], level_nb[l], bbox + level_off[l + 1], npar);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  const int nbox = level_off[levels - 1] + level_nb[levels - 1];
  k_box_centres<<<(nbox + 255) / 256, 256, 0, st>>>(bbox, nbox, out, rbits);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  LevelTable lv{};
  for (int l = 0; l < levels; ++l) lv.off[l] = level_off[l];
  k_box_radii<<<level_nb[0], 256, 0, st>>>(eta, N, lv, levels, invp, out, rbits);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_box_finish<<<(nbox + 255) / 256, 256, 0, st>>>(rbits, nbox, out);
  return hipGetLastError();
}

hipError_t launch_tree_moments(const double2* rec, int stride, int wo, int N, const double4* bounds, const int* perm,
                               const int* level_off, const int* level_nb, int levels, int p, double2* mom,
                               hipStream_t st) {
  k_leaf_moments<<<level_nb[0], 64, 0, st>>>(rec, stride, wo, N, bounds, perm, p, mom);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (levels > 32 || p > kTreeMaxP) return hipErrorInvalidValue;
  LevelTable lt{};
  for (int l = 0; l < levels; ++l) {
    lt.off[l] = level_off[l];
    lt.nb[l] = level_nb[l];
  }
  for (int l = 0; l + 1 < levels;) {
    const int nlev = min(kM2MLevels, levels - 1 - l);
    k_m2m_levels<<<level_nb[l + nlev], kM2MThreads, 0, st>>>(bounds, lt, l, nlev, p, mom);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    l += nlev;
  }
  return hipSuccess;
}

hipError_t launch_tree_eval(const DomDev* doms, int tiles, int tpt, const int* seg, const int* list,
                            const double4* bounds, const double2* mom, int p, int splits, int col, int wcols,
                            const int* active, int lead, bool ext, hipStream_t st) {
  const unsigned grid = (unsigned)tiles * (unsigned)splits;
  const int e = ext ? 1 : 0;
  if (tpt == 2)
    k_tree<2><<<grid, 256, 0, st>>>(doms, seg, list, bounds, mom, p, splits, col, wcols, active, lead, e);
  else
    k_tree<1><<<grid, 256, 0, st>>>(doms, seg, list, bounds, mom, p, splits, col, wcols, active, lead, e);
  return hipGetLastError();
}

}  // namespace gnk
