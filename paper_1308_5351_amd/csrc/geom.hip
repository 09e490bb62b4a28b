// Derivatives of the discrete operators with respect to the boundary data, and
// Fourier boundary curves with their reverse-mode derivative.
//
// Geometry. Every geometry-dependent entry of f_B = 2I + diag(B1) - B and of
// fC = D - diag(D1) + Lhat comes from K_ij = (2/n) a_i b_j / (eta_j - eta_i),
// a = A, b = eta'/A (B = Im K, D = Re K, eqs. (e:B), (e:M); Lhat depends on n
// only). For s = sum_t c_t u_t^T Op_t v_t (Op_t = f_B or fC, u_t, v_t real)
//   s = const + Re sum_{i != j} K_ij W_ij,  W_ij = sum_t z_t u_t,i (v_t,j - v_t,i),
// with z_t = i c_t for f_B (B = Re(-i K), and the rows of diag(B1) - B give
// u_i (v_i - v_j)) and z_t = c_t for fC. Grouping the terms by v (groups g with
// vector V_g and U_g = sum_{t in g} z_t u_t, P = sum_g U_g V_g), the partial
// derivatives of F = sum_{i != j} K_ij W_ij need only row and column sums:
//   R1_i = sum_j K_ij W_ij = -kappa a_i [sum_g U_g,i S1(b V_g)_i - P_i S1(b)_i]
//   R2_i = sum_j K_ij W_ij / (eta_j - eta_i) = kappa a_i [sum_g U_g,i S2(b V_g)_i - P_i S2(b)_i]
//   T1_i = sum_g V_g,i S1(a U_g)_i - S1(a P)_i,   T2_i likewise with S2
//   dF/deta_i = R2_i - kappa b_i T2_i,  dF/deta'_i = kappa T1_i / A_i,
//   dF/dA_i = (R1_i - kappa b_i T1_i) / A_i,
// kappa = 2/n, S1(w)_i = sum_{j != i} w_j/(eta_i - eta_j) (the matrix E of
// eq. (e:fmm-E)) and S2(w)_i = sum_{j != i} w_j/(eta_i - eta_j)^2. The
// gradients returned are conj(dF/dz) = ds/dRe z + i ds/dIm z.
//
// The first- and second-order sums share each pair's reciprocal q = 1/d
// (q^2 costs one complex square). The kernel follows the operator pair
// kernel: wave-uniform source records {eta_j, w_j,0..} fetched with scalar
// loads, four wavefronts splitting the sources of a workgroup and adding
// their sums through LDS in a fixed order, partial sums per source split
// added in a fixed order by the epilogue (bitwise reproducible).
#include <cstdint>

#include "gnk_device.h"
#include "gnk_internal.h"

namespace gnk {

namespace {

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
  const double m = 1.0 / (b.x * b.x + b.y * b.y);
  return make_double2((a.x * b.x + a.y * b.y) * m, (a.y * b.x - a.x * b.y) * m);
}
__device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 zscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// records: rec[j*stride] = eta_j, rec[j*stride + 1 + q] = w_q,j for q < nw
// (nw = 2G + 2 columns: b V_g, b, a U_g, a P), padded with zeros to nwpad.
__global__ void k_geom_weights(const double2* __restrict__ eta, const double2* __restrict__ etap,
                               const double2* __restrict__ A, int N, const GeomTerm* __restrict__ terms,
                               const GeomGroup* __restrict__ groups, int G, int nwpad, double2* __restrict__ rec,
                               double2* __restrict__ Ut, double2* __restrict__ P) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int stride = 1 + nwpad;
  double2* r = rec + (size_t)j * stride;
  const double2 a = A[j];
  const double2 b = zdiv(etap[j], a);
  r[0] = eta[j];
  double2 p = make_double2(0.0, 0.0);
  for (int g = 0; g < G; ++g) {
    const GeomGroup gr = groups[g];
    double2 U = make_double2(0.0, 0.0);
    for (int t = gr.t0; t < gr.t1; ++t) U = zadd(U, zscale(terms[t].u[j], terms[t].z));
    const double v = gr.v[j];
    Ut[(size_t)g * N + j] = U;
    p = zadd(p, zscale(v, U));
    r[1 + g] = zscale(v, b);
    r[1 + G + 1 + g] = zmul(a, U);
  }
  r[1 + G] = b;
  r[1 + 2 * G + 1] = zmul(a, p);
  for (int q = 2 * G + 2; q < nwpad; ++q) r[1 + q] = make_double2(0.0, 0.0);
  P[j] = p;
}

// First- and second-order sums of NR weight columns (q0 = blockIdx.z * NR) for
// the 64 targets of blockIdx.x over the sources of split blockIdx.y:
//   parts[((g*nw + q)*2 + o)*N + i] = sum_{j in split g, j != i} w_qj / (eta_i - eta_j)^(o+1)
template <int NR>
__global__ __launch_bounds__(256) void k_cauchy12(const double2* __restrict__ rec_, int stride, int N, int nw,
                                                  int chunk, double2* __restrict__ parts_) {
  __shared__ double red[3][4 * NR][64];
  gptr<const double2> rec = (gptr<const double2>)rec_;
  gptr<double2> parts = (gptr<double2>)parts_;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blockIdx.x * 64 + lane;
  const int g = blockIdx.y;
  const int q0 = blockIdx.z * NR;
  const double2 ti = rec[(size_t)min(i, N - 1) * stride];
  const int jb0 = g * chunk;
  const int jb1 = min(N, jb0 + chunk);
  const int wchunk = (chunk + 3) >> 2;
  const int j0 = min(jb1, jb0 + wv * wchunk);
  const int j1 = min(jb1, j0 + wchunk);
  double s1x[NR], s1y[NR], s2x[NR], s2y[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) s1x[r] = s1y[r] = s2x[r] = s2y[r] = 0.0;
  for (int j = j0; j < j1; ++j) {
    gptr<const double2> rj = rec + (size_t)j * stride;
    const double2 e = rj[0];
    const double dx = ti.x - e.x, dy = ti.y - e.y;
    double m = refine_rcp(__builtin_fma(dy, dy, dx * dx));
    m = (j == i) ? 0.0 : m;
    const double qx = dx * m, qy = -dy * m;                        // 1/d
    const double px = __builtin_fma(qx, qx, -qy * qy), py = 2.0 * qx * qy;   // 1/d^2
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double2 w = rj[1 + q0 + r];
      s1x[r] = __builtin_fma(w.x, qx, s1x[r]);
      s1x[r] = __builtin_fma(-w.y, qy, s1x[r]);
      s1y[r] = __builtin_fma(w.x, qy, s1y[r]);
      s1y[r] = __builtin_fma(w.y, qx, s1y[r]);
      s2x[r] = __builtin_fma(w.x, px, s2x[r]);
      s2x[r] = __builtin_fma(-w.y, py, s2x[r]);
      s2y[r] = __builtin_fma(w.x, py, s2y[r]);
      s2y[r] = __builtin_fma(w.y, px, s2y[r]);
    }
  }
  if (wv > 0) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      red[wv - 1][4 * r + 0][lane] = s1x[r];
      red[wv - 1][4 * r + 1][lane] = s1y[r];
      red[wv - 1][4 * r + 2][lane] = s2x[r];
      red[wv - 1][4 * r + 3][lane] = s2y[r];
    }
  }
  __syncthreads();
  if (wv == 0 && i < N) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      double a = s1x[r], b = s1y[r], c = s2x[r], d = s2y[r];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a += red[k][4 * r + 0][lane];
        b += red[k][4 * r + 1][lane];
        c += red[k][4 * r + 2][lane];
        d += red[k][4 * r + 3][lane];
      }
      const int q = q0 + r;
      if (q < nw) {
        parts[(((size_t)g * nw + q) * 2 + 0) * N + i] = make_double2(a, b);
        parts[(((size_t)g * nw + q) * 2 + 1) * N + i] = make_double2(c, d);
      }
    }
  }
}

__global__ void k_geom_epilogue(const double2* __restrict__ etap, const double2* __restrict__ A, int N, int n,
                                const GeomGroup* __restrict__ groups, int G, const double2* __restrict__ Ut,
                                const double2* __restrict__ P, const double2* __restrict__ parts, int nw, int splits,
                                double2* g_eta, double2* g_etap, double2* g_A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  auto S = [&](int q, int o) {
    double2 s = make_double2(0.0, 0.0);
    for (int g = 0; g < splits; ++g) s = zadd(s, parts[(((size_t)g * nw + q) * 2 + o) * N + i]);
    return s;
  };
  const double kappa = 2.0 / (double)n;
  const double2 a = A[i];
  const double2 b = zdiv(etap[i], a);
  double2 R1 = make_double2(0.0, 0.0), R2 = R1, T1 = R1, T2 = R1;
  for (int g = 0; g < G; ++g) {
    const double2 U = Ut[(size_t)g * N + i];
    const double v = groups[g].v[i];
    R1 = zadd(R1, zmul(U, S(g, 0)));
    R2 = zadd(R2, zmul(U, S(g, 1)));
    T1 = zadd(T1, zscale(v, S(G + 1 + g, 0)));
    T2 = zadd(T2, zscale(v, S(G + 1 + g, 1)));
  }
  const double2 p = P[i];
  R1 = zsub(R1, zmul(p, S(G, 0)));
  R2 = zsub(R2, zmul(p, S(G, 1)));
  T1 = zsub(T1, S(2 * G + 1, 0));
  T2 = zsub(T2, S(2 * G + 1, 1));
  R1 = zscale(-kappa, zmul(a, R1));
  R2 = zscale(kappa, zmul(a, R2));
  const double2 C1 = zscale(kappa, zmul(b, T1));
  const double2 C2 = zscale(-kappa, zmul(b, T2));
  const double2 de = zadd(R2, C2);
  const double2 dp = zscale(kappa, zdiv(T1, a));
  const double2 da = zdiv(zsub(R1, C1), a);
  if (g_eta) g_eta[i] = make_double2(de.x, -de.y);
  if (g_etap) g_etap[i] = make_double2(dp.x, -dp.y);
  if (g_A) g_A[i] = make_double2(da.x, -da.y);
}

// e^{2 pi i m / n} for an integer m reduced into [0, n) (exact argument)
__device__ __forceinline__ double2 unit_root(int64_t m, int64_t n) {
  double s, c;
  sincospi(2.0 * (double)m / (double)n, &s, &c);
  return make_double2(c, s);
}

__device__ __forceinline__ int64_t mod_n(int64_t x, int64_t n) {
  int64_t r = x % n;
  return r < 0 ? r + n : r;
}

// eta_j(t_p) = sum_k c_{j,k} e^{i s k t_p}, t_p = 2 pi p / n, and the first two
// derivatives (factors i s k and -k^2); grid (blocks over n, m1)
__global__ void k_fourier_curve(const double2* __restrict__ coef, int n, int kmin, int nk, int sgn,
                                double2* __restrict__ eta, double2* __restrict__ etap, double2* __restrict__ etapp) {
  const int j = blockIdx.y;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  double2 e0 = make_double2(0.0, 0.0), e1 = e0, e2 = e0;
  for (int q = 0; q < nk; ++q) {
    const int64_t k = kmin + q;
    const double2 cp = zmul(coef[(size_t)j * nk + q], unit_root(mod_n((int64_t)sgn * k * p, n), n));
    const double sk = (double)(sgn * k);
    e0 = zadd(e0, cp);
    e1 = zadd(e1, make_double2(-sk * cp.y, sk * cp.x));
    e2 = zadd(e2, zscale(-(double)(k * k), cp));
  }
  const size_t o = (size_t)j * n + p;
  eta[o] = e0;
  if (etap) etap[o] = e1;
  if (etapp) etapp[o] = e2;
}

// g_c[j,k] = sum_p (g_eta + conj(i s k) g_eta' + conj(-k^2) g_eta'')_p e^{-i s k t_p};
// one 256-thread block per (coefficient, component), fixed-order reduction
__global__ __launch_bounds__(256) void k_fourier_vjp(const double2* __restrict__ g_eta,
                                                     const double2* __restrict__ g_etap,
                                                     const double2* __restrict__ g_etapp, int n, int kmin, int nk,
                                                     int sgn, double2* __restrict__ g_coef) {
  __shared__ double2 sh[256];
  const int q = blockIdx.x, j = blockIdx.y;
  const int64_t k = kmin + q;
  const double sk = (double)(sgn * k);
  double2 acc = make_double2(0.0, 0.0);
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const size_t o = (size_t)j * n + p;
    double2 w = g_eta ? g_eta[o] : make_double2(0.0, 0.0);
    if (g_etap) {
      const double2 z = g_etap[o];
      w = zadd(w, make_double2(sk * z.y, -sk * z.x));     // (-i s k) z
    }
    if (g_etapp) w = zadd(w, zscale(-(double)(k * k), g_etapp[o]));
    acc = zadd(acc, zmul(w, unit_root(mod_n(-(int64_t)sgn * k * p, n), n)));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = zadd(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) g_coef[(size_t)j * nk + q] = sh[0];
}

}  // namespace

hipError_t launch_geom_weights(const double2* eta, const double2* etap, const double2* A, int N,
                               const GeomTerm* terms, const GeomGroup* groups, int G, int nwpad, double2* rec,
                               double2* Ut, double2* P, hipStream_t st) {
  k_geom_weights<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(eta, etap, A, N, terms, groups, G, nwpad, rec, Ut, P);
  return hipGetLastError();
}

int geom_width(int nw) { return nw % 6 == 0 ? 6 : 2; }

hipError_t launch_cauchy12(const double2* rec, int nwpad, int N, int nw, int chunk, int splits, double2* parts,
                           hipStream_t st) {
  const int w = geom_width(nwpad);
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)splits, (unsigned)(nwpad / w));
  if (w == 6) k_cauchy12<6><<<grid, 256, 0, st>>>(rec, 1 + nwpad, N, nw, chunk, parts);
  else k_cauchy12<2><<<grid, 256, 0, st>>>(rec, 1 + nwpad, N, nw, chunk, parts);
  return hipGetLastError();
}

hipError_t launch_geom_epilogue(const double2* etap, const double2* A, int N, int n, const GeomGroup* groups, int G,
                                const double2* Ut, const double2* P, const double2* parts, int nw, int splits,
                                double2* g_eta, double2* g_etap, double2* g_A, hipStream_t st) {
  k_geom_epilogue<<<(unsigned)((N + 255) / 256), 256, 0, st>>>(etap, A, N, n, groups, G, Ut, P, parts, nw, splits,
                                                               g_eta, g_etap, g_A);
  return hipGetLastError();
}

hipError_t launch_fourier_curve(const double2* coef, int m1, int n, int kmin, int nk, int sgn, double2* eta,
                                double2* etap, double2* etapp, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)m1);
  k_fourier_curve<<<grid, 256, 0, st>>>(coef, n, kmin, nk, sgn, eta, etap, etapp);
  return hipGetLastError();
}

hipError_t launch_fourier_vjp(const double2* g_eta, const double2* g_etap, const double2* g_etapp, int m1, int n,
                              int kmin, int nk, int sgn, double2* g_coef, hipStream_t st) {
  dim3 grid((unsigned)nk, (unsigned)m1);
  k_fourier_vjp<<<grid, 256, 0, st>>>(g_eta, g_etap, g_etapp, n, kmin, nk, sgn, g_coef);
  return hipGetLastError();
}

}  // namespace gnk
