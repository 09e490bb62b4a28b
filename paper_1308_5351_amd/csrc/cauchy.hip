// Direct Cauchy sum on gfx950 (FP64):
//   S_i = sum_{j != i} w_j / (eta_i - eta_j)          (matrix E of eq. (e:fmm-E))
// for several weight columns w at once. This single product carries every
// operator of the method: Im and Re of A_i S_i give B x and D x
// (eqs. (e:(I-B)x), (e:hD-bt)); (eta'/A) S with w = A x gives B^T x
// (eq. (e:BTx)); w = eta' gives the vector e (eq. (e:bve)).
//
// Mapping (VALU-bound, no matrix cores: every pair needs its own reciprocal):
//   * one target node per lane, 64 consecutive targets per wavefront;
//   * the source loop index is wave-uniform, so eta_j and w_j are fetched with
//     scalar loads into SGPRs and broadcast to all lanes for free (no LDS
//     traffic, no bank conflicts); the targets stay in VGPRs;
//   * the source range is split over grid.y so that small problems still
//     launch >> 256 workgroups; the partial sums of the splits are reduced in a
//     fixed order by the consumer, so results are bitwise reproducible;
//   * 1/|d|^2 comes from v_rcp_f64 refined by one Newton step; two sources share one reciprocal: 1/a = b/(ab), 1/b = a/(ab)
//     (Montgomery's simultaneous inversion), which removes half of the
//     quarter-rate v_rcp_f64 issues;
//   * only the 64-source window that contains the wave's own targets needs
//     the j != i test; it runs a separate masked loop.
#include "gnk_internal.h"

namespace gnk {

namespace {

// v_rcp_f64 is accurate to about 2^-24 on gfx950; one Newton step brings the
// reciprocal to about 2^-48 (a few ulp), below the rounding of the sums.
constexpr int kNewton = 1;

__device__ __forceinline__ double refine_rcp(double d) {
  double r = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int k = 0; k < kNewton; ++k) {
    const double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
  }
  return r;
}

// acc += w * q for NR columns, q = conj(d)/|d|^2 = (qx, qy)
template <int NR>
__device__ __forceinline__ void accumulate(double (&ax)[NR], double (&ay)[NR], const double2* __restrict__ wj,
                                           double qx, double qy) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double2 w = wj[r];
    ax[r] = __builtin_fma(w.x, qx, ax[r]);
    ax[r] = __builtin_fma(-w.y, qy, ax[r]);
    ay[r] = __builtin_fma(w.x, qy, ay[r]);
    ay[r] = __builtin_fma(w.y, qx, ay[r]);
  }
}

template <int NR>
__global__ __launch_bounds__(256) void k_cauchy_fp64(const double2* __restrict__ eta, const double2* __restrict__ W,
                                                     int N, int nrhs, int r0, int chunk,
                                                     double2* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // first target of this wavefront (uniform)
  const int iw = __builtin_amdgcn_readfirstlane(blockIdx.x * blockDim.x + (threadIdx.x & ~63));
  const int g = blockIdx.y;
  const int j0 = g * chunk;
  const int j1 = min(N, j0 + chunk);
  const double2 t = eta[min(i, N - 1)];
  const double2* __restrict__ Wr = W + r0;

  double ax[NR], ay[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) { ax[r] = 0.0; ay[r] = 0.0; }

  // sources before / after the wave's own 64-node window need no j != i test
  auto plain = [&](int ja, int jb) {
    int j = ja;
    for (; j + 1 < jb; j += 2) {
      const double2 ea = eta[j], eb = eta[j + 1];
      const double dxa = t.x - ea.x, dya = t.y - ea.y;
      const double dxb = t.x - eb.x, dyb = t.y - eb.y;
      const double da = __builtin_fma(dya, dya, dxa * dxa);
      const double db = __builtin_fma(dyb, dyb, dxb * dxb);
      const double R = refine_rcp(da * db);
      const double ra = db * R, rb = da * R;
      accumulate<NR>(ax, ay, Wr + (size_t)j * nrhs, dxa * ra, -dya * ra);
      accumulate<NR>(ax, ay, Wr + (size_t)(j + 1) * nrhs, dxb * rb, -dyb * rb);
    }
    if (j < jb) {
      const double2 ea = eta[j];
      const double dx = t.x - ea.x, dy = t.y - ea.y;
      const double r = refine_rcp(__builtin_fma(dy, dy, dx * dx));
      accumulate<NR>(ax, ay, Wr + (size_t)j * nrhs, dx * r, -dy * r);
    }
  };

  plain(j0, min(j1, iw));
  {
    const int ja = max(j0, iw), jb = min(j1, iw + 64);
    for (int j = ja; j < jb; ++j) {
      const double2 e = eta[j];
      const double dx = t.x - e.x, dy = t.y - e.y;
      double r = refine_rcp(__builtin_fma(dy, dy, dx * dx));
      r = (j == i) ? 0.0 : r;
      accumulate<NR>(ax, ay, Wr + (size_t)j * nrhs, dx * r, -dy * r);
    }
  }
  plain(max(j0, iw + 64), j1);

  if (i < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      part[((size_t)g * nrhs + r0 + r) * N + i] = make_double2(ax[r], ay[r]);
  }
}

}  // namespace

CauchyPlan plan_cauchy(int64_t N, int nrhs, int num_cu) {
  CauchyPlan p;
  p.tpb = 256;
  const int64_t blocks = (N + p.tpb - 1) / p.tpb;
  // aim for about 8 resident workgroups per CU over the whole launch
  const int64_t want = 8LL * num_cu;
  int64_t s = (want + blocks - 1) / blocks;
  // keep at least ~512 sources per split so the loop overhead stays small
  const int64_t max_s = N / 512 > 1 ? N / 512 : 1;
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  if (s > 64) s = 64;
  p.splits = (int)s;
  int64_t chunk = (N + s - 1) / s;
  chunk = (chunk + 1) & ~int64_t(1);
  p.chunk = chunk;
  p.splits = (int)((N + chunk - 1) / chunk);
  (void)nrhs;
  return p;
}

hipError_t launch_cauchy_fp64(const double2* eta, const double2* W, int64_t N, int nrhs, const CauchyPlan& plan,
                              double2* S_part, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  dim3 grid((unsigned)((N + plan.tpb - 1) / plan.tpb), (unsigned)plan.splits);
  int r0 = 0;
  while (r0 < nrhs) {
    const int left = nrhs - r0;
    if (left >= 8) {
      k_cauchy_fp64<8><<<grid, plan.tpb, 0, st>>>(eta, W, (int)N, nrhs, r0, (int)plan.chunk, S_part);
      r0 += 8;
    } else if (left >= 4) {
      k_cauchy_fp64<4><<<grid, plan.tpb, 0, st>>>(eta, W, (int)N, nrhs, r0, (int)plan.chunk, S_part);
      r0 += 4;
    } else if (left >= 2) {
      k_cauchy_fp64<2><<<grid, plan.tpb, 0, st>>>(eta, W, (int)N, nrhs, r0, (int)plan.chunk, S_part);
      r0 += 2;
    } else {
      k_cauchy_fp64<1><<<grid, plan.tpb, 0, st>>>(eta, W, (int)N, nrhs, r0, (int)plan.chunk, S_part);
      r0 += 1;
    }
  }
  return hipGetLastError();
}

}  // namespace gnk
