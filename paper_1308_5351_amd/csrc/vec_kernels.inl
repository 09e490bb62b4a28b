// Per-node and per-column kernels around the Cauchy sums (validation, source
// records, operator epilogues) and the kernels of the device-resident
// restarted GMRES (classical Gram-Schmidt with one re-orthogonalisation,
// Givens rotations, back substitution), for a batch of domains and ragged
// columns. Column c (domain d = cols[c].d, local column r) has N_d entries
// at flat offset cols[c].off. All reductions run in a fixed order, so
// repeated runs are bitwise identical.
// Included by solver.hip (one translation unit with the host driver).
#pragma once
#include "gnk_device.h"
#include "gnk_vec.h"

namespace gnk {

namespace {

constexpr int kT = 256;   // threads per block of the vector kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

__device__ __forceinline__ bool finite2(double2 v) { return isfinite(v.x) && isfinite(v.y); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace

// per-node coefficient selectors of the records and epilogues
enum CSel : int { C_RHO = 0, C_A = 1, C_ETAP = 2 };
enum DSel : int { D_NONE = 0, D_B = 1, D_D = 2, D_E = 3, D_BU = 4 };

__device__ __forceinline__ double2 coef(const DomDev& D, int sel, int i) {
  return sel == C_RHO ? D.rho[i] : (sel == C_A ? D.A[i] : D.etap[i]);
}
// eta_j relative to the centre of its far-form tile (the pair kernels' far form)
__device__ __forceinline__ double2 eta_rel(const DomDev& D, int j) {
  const double2 e = D.eta[j];
  const double4 c = D.sbf[j >> kFarTileLog2];
  return make_double2(e.x - c.x, e.y - c.y);
}
// record head {eta, u = -2 eta', (|eta'|^2, 0)}
__device__ __forceinline__ void record_head(double2* rj, double2 eta, double2 ep) {
  rj[0] = eta;
  rj[1] = make_double2(-2.0 * ep.x, -2.0 * ep.y);
  rj[2] = make_double2(__builtin_fma(ep.y, ep.y, ep.x * ep.x), 0.0);
}
// a * conj(b)
__device__ __forceinline__ double2 cmul_conj(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double diagv(const DomDev& D, int sel, int i) {
  return sel == D_B ? D.dB[i] : (sel == D_D ? D.dD[i] : (sel == D_E ? D.e[i] : (sel == D_BU ? D.bu[i] : 0.0)));
}

// ---------------------------------------------------------------- validation
// grid (blocks over max N, ndom)
__global__ void k_validate(const DomDev* __restrict__ doms, int adjoint, int* flags) {
  const DomDev& D = doms[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  int f = 0;
  const double2 a = D.A[i];
  if (!finite2(a) || !finite2(D.eta[i]) || !finite2(D.etap[i])) f |= 1;
  if (a.x == 0.0 && a.y == 0.0) f |= 2;
  if (adjoint) {
    if (!finite2(D.etapp[i]) || !finite2(D.Ap[i])) f |= 1;
    const double2 ep = D.etap[i];
    if (ep.x == 0.0 && ep.y == 0.0) f |= 4;
  }
  if (f) atomicOr(flags, f);
}

// The node checks of k_validate and the finiteness of x (len entries) in one
// launch (grid (blocks over max(max N, len), ndom + 1); row ndom takes x),
// with one flag word per failure (plain stores of 1 into host-mapped memory
// that the host zeroes before the launch): fl[0] non-finite, fl[1] A = 0,
// fl[2] eta' = 0 (adjoint).
__global__ void k_validate_inputs(const DomDev* __restrict__ doms, int ndom, int adjoint,
                                  const double* __restrict__ x, int64_t len, int* fl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((int)blockIdx.y == ndom) {
    if (i < len && !isfinite(x[i])) fl[0] = 1;
    return;
  }
  const DomDev& D = doms[blockIdx.y];
  if (i >= D.N) return;
  const double2 a = D.A[i];
  if (!finite2(a) || !finite2(D.eta[i]) || !finite2(D.etap[i])) fl[0] = 1;
  if (a.x == 0.0 && a.y == 0.0) fl[1] = 1;
  if (adjoint) {
    if (!finite2(D.etapp[i]) || !finite2(D.Ap[i])) fl[0] = 1;
    const double2 ep = D.etap[i];
    if (ep.x == 0.0 && ep.y == 0.0) fl[2] = 1;
  }
}

__global__ void k_check_finite(const double* x, int64_t n, int* flags) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicOr(flags, 1);
}

// ------------------------------------------------------------ per-node setup
// rho = eta' / A  (the weight factor of eqs. (e:hD-bt), (e:(I-B)x))
__global__ void k_rho(const DomDev* __restrict__ doms) {
  const DomDev& D = doms[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  const double2 p = D.etap[i], a = D.A[i];
  const double d = a.x * a.x + a.y * a.y;
  D.rho[i] = make_double2((p.x * a.x + p.y * a.y) / d, (p.y * a.x - p.x * a.y) / d);
}

// sum over the splits of weight column q (of wcols) of a domain's partial
// sums, added in split order; the loads go out eight at a time
__device__ __forceinline__ double2 reduce_parts(const DomDev& D, int wcols, int q, int i) {
  constexpr int kG = 8;
  const gptr<const double2> p = (gptr<const double2>)D.parts + (size_t)q * D.N + i;
  const size_t gs = (size_t)wcols * D.N;
  const int splits = D.splits;
  double2 s = make_double2(0.0, 0.0);
  for (int g = 0; g < splits; g += kG) {
    double2 v[kG];
#pragma unroll
    for (int k = 0; k < kG; ++k)
      if (g + k < splits) v[k] = p[(size_t)(g + k) * gs];
#pragma unroll
    for (int k = 0; k < kG; ++k)
      if (g + k < splits) {
        s.x += v[k].x;
        s.y += v[k].y;
      }
  }
  return s;
}

// From S = E(eta'/A) in weight column 0 (wcols columns):
//   dB = diag(B1) = -(2/n) Im(A S),  dD = diag(D1) = -(2/n) Re(A S)
// (eqs. (e:(I-B)x), (e:hD-bt) with x = 1)
__global__ void k_diag_fbie(const DomDev* __restrict__ doms, int lead, int data) {
  const DomDev& D = doms[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  const int wcols = lead + data * D.ncols;
  const double2 s = reduce_parts(D, wcols, 0, i);
  const double2 as = cmul(D.A[i], s);
  const double two_n = 2.0 / (double)D.n;
  D.dB[i] = -two_n * as.y;
  D.dD[i] = -two_n * as.x;
}

// (2 pi/n) N(t_i, t_i) = (2/n) (1/2 Im(eta''/eta') - Im(A'/A))   (eq. (e:N-tt)),
// the diagonal of the kernel N for the equations without singularity subtraction
__global__ void k_ndiag(const DomDev* __restrict__ doms) {
  const DomDev& D = doms[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  const double2 p = D.etap[i], pp = D.etapp[i], a = D.A[i], ap = D.Ap[i];
  const double dp = p.x * p.x + p.y * p.y, da = a.x * a.x + a.y * a.y;
  const double im1 = (pp.y * p.x - pp.x * p.y) / dp;   // Im(eta''/eta')
  const double im2 = (ap.y * a.x - ap.x * a.y) / da;   // Im(A'/A)
  D.bu[i] = (2.0 / (double)D.n) * (0.5 * im1 - im2);
}

// From S = E eta' (weight column 0 of wcols = 1):
//   e = 1 - c - (2/n) Im(S) + (2/n) Im(eta''/eta' - A'/A)   (eq. (e:bve))
__global__ void k_evec(const DomDev* __restrict__ doms) {
  const DomDev& D = doms[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  const double2 s = reduce_parts(D, 1, 0, i);
  const double2 p = D.etap[i], pp = D.etapp[i], a = D.A[i], ap = D.Ap[i];
  const double dp = p.x * p.x + p.y * p.y, da = a.x * a.x + a.y * a.y;
  const double im1 = (pp.y * p.x - pp.x * p.y) / dp;   // Im(eta''/eta')
  const double im2 = (ap.y * a.x - ap.x * a.y) / da;   // Im(A'/A)
  const double two_n = 2.0 / (double)D.n;
  D.e[i] = 1.0 - (double)D.c - two_n * s.y + two_n * (im1 - im2);
}

// ----------------------------------------------- source records and means
// FP64 records rec_d[j*stride], stride = 3 + 2 wcols (wcols = lead + ncols):
//   [0] eta_j, [1] u_j = -2 eta'_j, [2] (|eta'_j|^2, 0), with eta'_j = eta_j - c
//   (c the centre of j's far-form tile of kFarTile nodes),
//   [3 + q] w_q, [3 + wcols + q] b_q = w_q conj(eta'_j),
// with weight column q = 0 the leading coefficient C_j when lead, and
// q = lead + r the value C_j * x_j of the domain's column r, and
//   mean[c*M + k] = (1/n) sum_p x_{k n + p}   (optional, component means)
// grid (max m1, ncol): block (k, c) covers component k of column c.
__global__ __launch_bounds__(kT) void k_weights(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                                                int csel, const double* __restrict__ x,
                                                const int* __restrict__ active, int lead, double* __restrict__ mean,
                                                int M) {
  __shared__ double sh[kT / 64];
  const int k = blockIdx.x, c = blockIdx.y;
  const ColDev C = cols[c];
  const DomDev& D = doms[C.d];
  if (k >= D.m1) return;
  if (active && !active[c]) return;
  const int wcols = lead + D.ncols;
  const int stride = rec_stride(wcols);
  const double* xr = x + C.off + (size_t)k * D.n;
  double acc = 0.0;
  for (int p = threadIdx.x; p < D.n; p += blockDim.x) {
    const int j = k * D.n + p;
    const double v = xr[p];
    const double2 cf = coef(D, csel, j);
    const double2 ep = eta_rel(D, j);
    double2* rj = D.rec + (size_t)j * stride;
    const double2 w = make_double2(cf.x * v, cf.y * v);
    rj[kRecHead + lead + C.r] = w;
    rj[kRecHead + wcols + lead + C.r] = cmul_conj(w, ep);
    if (C.r == 0) {
      record_head(rj, D.eta[j], ep);
      if (lead) {
        rj[kRecHead] = cf;
        rj[kRecHead + wcols] = cmul_conj(cf, ep);
      }
    }
    acc += v;
  }
  if (mean) {
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) mean[(size_t)c * M + k] = t / (double)D.n;
  }
}

// Weight fields of node j, column r, in records without a leading column
// (wcols = ncols): w = C_j q and w conj(eta'_j); with `head`, the node's head too.
__device__ __forceinline__ void stage_weight(const DomDev& D, int csel, int r, int j, double q, bool head) {
  const int wcols = D.ncols;
  const double2 ep = eta_rel(D, j);
  const double2 cf = coef(D, csel, j);
  double2* rj = D.rec + (size_t)j * rec_stride(wcols);
  const double2 w = make_double2(cf.x * q, cf.y * q);
  rj[kRecHead + r] = w;
  rj[kRecHead + wcols + r] = cmul_conj(w, ep);
  if (head) record_head(rj, D.eta[j], ep);
}

// Sums of a chunk's entries over each component of n entries that it meets:
// out[k - i0/n] for components k = i0/n .. (i1-1)/n, from the chunk held in
// LDS (sq[i - i0]); wavefront q takes components i0/n + q, + q + 4, ...
__device__ __forceinline__ void chunk_component_sums(const double* sq, int i0, int i1, int n,
                                                     double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int k0 = i0 / n, k1 = (i1 - 1) / n;
  for (int k = k0 + wv; k <= k1; k += nw) {
    const int lo = max(i0, k * n), hi = min(i1, (k + 1) * n);
    double acc = 0.0;
    for (int i = lo + lane; i < hi; i += 64) acc += sq[i - i0];
    acc = wave_sum(acc);
    if (lane == 0) out[k - k0] = acc;
  }
}

// records holding only the leading column (wcols = 1): head, C_j, C_j conj(eta')
__global__ void k_lead_records(const DomDev* __restrict__ doms, int csel) {
  const DomDev& D = doms[blockIdx.y];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.N) return;
  const double2 ep = eta_rel(D, j);
  const double2 cf = coef(D, csel, j);
  double2* rj = D.rec + (size_t)j * rec_stride(1);
  record_head(rj, D.eta[j], ep);
  rj[kRecHead] = cf;
  rj[kRecHead + 1] = cmul_conj(cf, ep);
}

// records of one domain from column-major complex weights w (N x ncols)
__global__ void k_pack_records(const DomDev* __restrict__ doms, const double2* __restrict__ w, int ncols) {
  const DomDev& D = doms[0];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.N) return;
  const double2 ep = eta_rel(D, j);
  double2* rj = D.rec + (size_t)j * rec_stride(ncols);
  record_head(rj, D.eta[j], ep);
  for (int r = 0; r < ncols; ++r) {
    const double2 v = w[(size_t)r * D.N + j];
    rj[kRecHead + r] = v;
    rj[kRecHead + ncols + r] = cmul_conj(v, ep);
  }
}

// ------------------------------- conformal maps onto the disc with slits
// One block per component k: d = eta - alpha, its argument continued along the
// component from the principal value at the first node (sums of the angles
// arg(d_p / d_{p-1}) between neighbours: one contiguous chunk per thread, then
// an exclusive scan of the chunk sums), and with rot_k = exp(i (pi/2 - theta_k))
//   A = rot_k d (bounded G) or rot_k (unbounded G)   (eq. (e:A))
//   gamma = -Re[rot_k log d]         (Re[rot log f] constant on each component).
// wind[k] = the argument's total change around the closed component: 2 pi for
// the outer boundary of a bounded G and 0 for a hole when alpha lies in G.
__global__ __launch_bounds__(kT) void k_slit_setup(const double2* __restrict__ eta, int n, int bounded, double ax,
                                                   double ay, const double2* __restrict__ rot,
                                                   double2* __restrict__ A, double* __restrict__ gam,
                                                   double* __restrict__ wind) {
  __shared__ double sc[kT];
  const int k = blockIdx.x, t = threadIdx.x;
  const int chunk = (n + kT - 1) / kT;
  const int p0 = min(n, t * chunk), p1 = min(n, p0 + chunk);
  const double2* e = eta + (size_t)k * n;
  auto dz = [&](int p) {
    const double2 v = e[p];
    return make_double2(v.x - ax, v.y - ay);
  };
  auto turn = [](double2 a, double2 b) { return atan2(a.x * b.y - a.y * b.x, a.x * b.x + a.y * b.y); };
  double s = 0.0;
  if (p0 < p1) {
    double2 prev = dz(p0 > 0 ? p0 - 1 : 0);
    for (int p = p0; p < p1; ++p) {
      const double2 cur = dz(p);
      if (p > 0) s += turn(prev, cur);
      prev = cur;
    }
  }
  sc[t] = s;
  __syncthreads();
  if (t == 0) {
    double run = 0.0;
    for (int q = 0; q < kT; ++q) {
      const double v = sc[q];
      sc[q] = run;
      run += v;
    }
    wind[k] = run + turn(dz(n - 1), dz(0));
  }
  __syncthreads();
  const double2 r = rot[k];
  const double2 d0 = dz(0);
  double arg = atan2(d0.y, d0.x) + sc[t];
  if (p0 < p1) {
    double2 prev = dz(p0 > 0 ? p0 - 1 : 0);
    for (int p = p0; p < p1; ++p) {
      const double2 d = dz(p);
      if (p > 0) arg += turn(prev, d);
      prev = d;
      const size_t i = (size_t)k * n + p;
      A[i] = bounded ? make_double2(r.x * d.x - r.y * d.y, r.x * d.y + r.y * d.x) : r;
      gam[i] = -r.x * (0.5 * log(d.x * d.x + d.y * d.y)) + r.y * arg;
    }
  }
}

// hbar[k] = (1/n) sum over component k of h (fixed-order block reduction)
__global__ __launch_bounds__(kT) void k_comp_means(const double* __restrict__ h, int n, double* __restrict__ hbar) {
  __shared__ double sh[kT / 64];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int p = threadIdx.x; p < n; p += blockDim.x) acc += h[(size_t)k * n + p];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) hbar[k] = t / (double)n;
}

// f(eta_i) = exp(-shift) d_i exp((gamma_i + hbar_k + i mu_i) / rot_k), d = eta - alpha,
// shift = hbar_0 for a bounded G (|f| = 1 on the outer boundary), 0 for an unbounded
// one (f(z) = z + O(1)); |rot_k| = 1, so the division is a product with its conjugate
__global__ void k_slit_map(const double2* __restrict__ eta, int bounded, double ax, double ay,
                           const double2* __restrict__ rot, const double* __restrict__ gam,
                           const double* __restrict__ mu, const double* __restrict__ hbar, int64_t N, int n,
                           double2* __restrict__ f) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t k = i / n;
  const double2 r = rot[k];
  const double a = gam[i] + hbar[k], b = mu[i];
  const double mag = exp((a * r.x + b * r.y) - (bounded ? hbar[0] : 0.0));
  double s, c;
  sincos(b * r.x - a * r.y, &s, &c);
  const double2 e = eta[i];
  const double dx = e.x - ax, dy = e.y - ay;
  f[i] = make_double2(mag * (dx * c - dy * s), mag * (dx * s + dy * c));
}

// ------------------------------------------ Cauchy integral at interior points
// Records of the nodes for F[eta'] and F[f_q eta'] (Sec. 7, eqs. (e:cauchy5),
// (e:cauchy6)): weight column 0 is eta'_j, column 1 + q is f_{j,q} eta'_j
// (f: N x nrhs complex, column-major).
__global__ void k_fcau_records(const DomDev* __restrict__ doms, const double2* __restrict__ f, int nrhs) {
  const DomDev& D = doms[0];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D.N) return;
  const int wcols = 1 + nrhs;
  const double2 ep = eta_rel(D, j);
  const double2 p = D.etap[j];
  double2* rj = D.rec + (size_t)j * rec_stride(wcols);
  record_head(rj, D.eta[j], ep);
  rj[kRecHead] = p;
  rj[kRecHead + wcols] = cmul_conj(p, ep);
  for (int q = 0; q < nrhs; ++q) {
    const double2 w = cmul(f[(size_t)q * D.N + j], p);
    rj[kRecHead + 1 + q] = w;
    rj[kRecHead + wcols + 1 + q] = cmul_conj(w, ep);
  }
}

// a / b without overflow of |b|^2 (scaled division)
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.y + b.x * r;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// f(z_i) for column q (grid (blocks over Nt, nrhs)) from the split partial
// sums of P_1 = F[eta'] (weight column 0) and P_f = F[f_q eta'] (column 1 + q):
//   bounded:   P_f / P_1                                   (e:cauchy6-b)
//   unbounded: (f(inf) - P_f/(n i)) / (1 - P_1/(n i))      (e:cauchy6-u)
// finf: nrhs values, or null for bounded G. A target on a node makes both
// sums infinite; it takes that node's value (the limit of the ratio).
// tperm (or null): target i is the caller's point tperm[i], where it is written.
__global__ void k_fcau_epilogue(const DomDev* __restrict__ doms, const double2* __restrict__ f, int nrhs,
                                const double2* __restrict__ finf, double n, const int* __restrict__ tperm,
                                double2* __restrict__ fz) {
  const DomDev& D = doms[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x, q = blockIdx.y;
  const int Nt = D.Nt;
  if (i >= Nt) return;
  const int wcols = 1 + nrhs;
  double2 p1 = make_double2(0.0, 0.0), pf = make_double2(0.0, 0.0);
  for (int g = 0; g < D.splits; ++g) {
    const double2 a = D.parts[((size_t)g * wcols) * Nt + i];
    const double2 b = D.parts[((size_t)g * wcols + 1 + q) * Nt + i];
    p1.x += a.x;
    p1.y += a.y;
    pf.x += b.x;
    pf.y += b.y;
  }
  double2 r;
  if (finf == nullptr) {
    r = cdiv(pf, p1);
  } else {
    // P/(n i) = (Im P, -Re P)/n
    const double2 fi = finf[q];
    r = cdiv(make_double2(fi.x - pf.y / n, fi.y + pf.x / n), make_double2(1.0 - p1.y / n, p1.x / n));
  }
  if (!isfinite(r.x) || !isfinite(r.y)) {
    const double2 zi = D.tz[i];
    for (int j = 0; j < D.N; ++j) {
      const double2 e = D.eta[j];
      if (e.x == zi.x && e.y == zi.y) {
        r = f[(size_t)q * D.N + j];
        break;
      }
    }
  }
  fz[(size_t)q * Nt + (tperm ? tperm[i] : i)] = r;
}

// zp[i] = z[perm[i]]
__global__ void k_gather_points(const double2* __restrict__ z, const int* __restrict__ perm, int64_t nz,
                                double2* __restrict__ zp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < nz) zp[i] = z[perm[i]];
}

// S[r*N + i] = sum over the splits of column r (one domain, no lead column)
__global__ void k_reduce_parts(const DomDev* __restrict__ doms, double2* __restrict__ S) {
  const DomDev& D = doms[0];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= D.N) return;
  S[(size_t)r * D.N + i] = reduce_parts(D, D.ncols, r, i);
}

// Operator epilogue for column c (grid (blocks over max N, ncol)), S from
// weight column lead + r of the domain's last Cauchy launch:
//   y = a0 x + dsign dg x + cI Im(Cout S) + cR Re(Cout S) + mean[c][k(i)]
__global__ void k_epilogue(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                           const double* __restrict__ x, int csel_out, int dsel, double a0, double dsign, double cI,
                           double cR, const double* __restrict__ mean, int M, const int* __restrict__ active,
                           int lead, double* __restrict__ y) {
  const int c = blockIdx.y;
  const ColDev C = cols[c];
  const DomDev& D = doms[C.d];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.N) return;
  if (active && !active[c]) return;
  const double2 s = reduce_parts(D, lead + D.ncols, lead + C.r, i);
  const double2 cs = cmul(coef(D, csel_out, i), s);
  const double two_n = 2.0 / (double)D.n;
  const double xv = x[C.off + i];
  double v = a0 * xv + two_n * (cI * cs.y + cR * cs.x);
  if (dsel != D_NONE) v += dsign * diagv(D, dsel, i) * xv;
  if (mean) v += mean[(size_t)c * M + i / D.n];
  y[C.off + i] = v;
}

// y = a x + b y  (elementwise over len)
__global__ void k_axpby(double a, const double* x, double b, double* y, int64_t len) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < len) y[i] = a * x[i] + b * y[i];
}

// out[c] = ||x_c||_2, one block per column, fixed-order reduction
__global__ __launch_bounds__(kT) void k_col_norms(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                                                  const double* __restrict__ x, double* __restrict__ out) {
  __shared__ double sh[kT / 64];
  const ColDev C = cols[blockIdx.x];
  const int N = doms[C.d].N;
  double acc = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) acc = __builtin_fma(x[C.off + i], x[C.off + i], acc);
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(t);
}

// ------------------------------------------------------------------ GMRES
// Krylov vector l of column c: V + l*T + off_c (T = flat length of a vector set).
// Partial sums: P[(c*nblk + blk)*ldp + l]; blocks past the column's end write 0.

// Dots of the block's chunk of w with V_0..V_{nvec-1}: wavefront q takes
// vectors l = q, q+4, ...; each lane sums its strided elements and the wave
// reduces by shuffles.
__device__ __forceinline__ void chunk_dots(const double* __restrict__ V, int64_t T, int64_t off, int nvec,
                                           const double* __restrict__ w, int i0, int i1,
                                           double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int l = wv; l < nvec; l += nw) {
    const double* vl = V + (size_t)l * T + off;
    double acc = 0.0;
    for (int i = i0 + lane; i < i1; i += 64) acc = __builtin_fma(vl[i], w[i - i0], acc);
    acc = wave_sum(acc);
    if (lane == 0) out[l] = acc;
  }
}

// One Arnoldi step l = *st.step of every iterating column takes four launches:
// the Cauchy sums of V_l (whose pair records the step before wrote), then
//   k_epilogue_dots  w = op(V_l) into V_{l+1}; dots of w with V_0..V_l
//   k_gs_update      w -= V h1; dots of w with V_0..V_l and |w|^2
//   k_gs_finish      w -= V h2, |w| = beta, V_{l+1} = w / beta and its pair
//                    records; block 0 closes Hessenberg column l.
// (classical Gram-Schmidt with one re-orthogonalisation). Every kernel works
// on chunks of per_blk elements of a column (grid (nblk, ncol)) and writes its
// partial sums to (c*nblk + blk)*ldp. V is the basis (vector q at V + q*T).
// For operators with the component means (P-hat x), the kernel that writes a
// vector also writes its chunk's sums over each component it meets to mpart
// ((c*nblk + blk)*S + slot), which the next epilogue adds up.

// Component means of V_l on the block's chunk [i0, i1), from the partial sums
// of the blocks whose chunks meet each component (fixed order): sm[k - i0/n].
__device__ __forceinline__ void chunk_means(const double* __restrict__ mpart, int S, int c, int nblk, int per_blk,
                                            int i0, int i1, int n, double* sm) {
  const int k0 = i0 / n, k1 = (i1 - 1) / n;
  for (int k = k0 + (int)threadIdx.x; k <= k1; k += blockDim.x) {
    const int b0 = (int)(((int64_t)k * n) / per_blk);
    const int b1 = (int)(((int64_t)(k + 1) * n - 1) / per_blk);
    double s = 0.0;
    for (int b = b0; b <= b1; ++b)
      s += mpart[((size_t)c * nblk + b) * S + (k - (int)(((int64_t)b * per_blk) / n))];
    sm[k - k0] = s / (double)n;
  }
  __syncthreads();
}

// Start of a cycle: V_0 = r / beta in place (beta from k_cycle_start), the
// pair records of V_0 (with the node heads) and, when mpart is given, the
// chunk's component sums.
__global__ __launch_bounds__(kT) void k_stage(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                                              double* __restrict__ V, int per_blk, int csel, GmresState st,
                                              double* __restrict__ mpart, int S) {
  __shared__ double sq[kMaxChunk];
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (!st.active[c]) return;
  const ColDev C = cols[c];
  const DomDev& D = doms[C.d];
  const int i0 = blk * per_blk, i1 = min(D.N, i0 + per_blk);
  if (i0 >= D.N) return;
  const double s = st.invbeta[c];
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double q = V[C.off + i] * s;
    V[C.off + i] = q;
    sq[i - i0] = q;
    // every iterating column writes the heads (the same values), so they are
    // there whichever columns of the domain iterate
    stage_weight(D, csel, C.r, i, q, true);
  }
  if (mpart) {
    __syncthreads();
    chunk_component_sums(sq, i0, i1, D.n, mpart + ((size_t)c * nblk + blk) * S);
  }
}

// w = V_{l+1} = op(V_l) on the block's chunk from the Cauchy sums of the last
// pair launch, then the chunk's dots of w with V_0..V_l.
__global__ __launch_bounds__(kT) void k_epilogue_dots(const DomDev* __restrict__ doms,
                                                      const ColDev* __restrict__ cols, double* __restrict__ V,
                                                      int64_t T, int csel_out, int dsel, double a0, double dsign,
                                                      double cI, double cR, const double* __restrict__ mpart, int S,
                                                      const int* __restrict__ active, const int* __restrict__ step,
                                                      int per_blk, double* __restrict__ partial, int ldp) {
  __shared__ double sw[kMaxChunk];
  __shared__ double sm[kMaxMeanSlots];
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (!active[c]) return;
  const int l = *step;
  const int nvec = l + 1;
  const double* __restrict__ xl = V + (size_t)l * T;
  double* __restrict__ w = V + (size_t)nvec * T;
  const ColDev C = cols[c];
  const DomDev& D = doms[C.d];
  const int N = D.N;
  double* out = partial + ((size_t)c * nblk + blk) * ldp;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  if (i0 >= N) {
    for (int q = threadIdx.x; q < nvec; q += blockDim.x) out[q] = 0.0;
    return;
  }
  if (mpart) chunk_means(mpart, S, c, nblk, per_blk, i0, i1, D.n, sm);
  const int k0 = i0 / D.n;
  const double two_n = 2.0 / (double)D.n;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double2 s = reduce_parts(D, D.ncols, C.r, i);
    const double2 cs = cmul(coef(D, csel_out, i), s);
    const double xv = xl[C.off + i];
    double v = a0 * xv + two_n * (cI * cs.y + cR * cs.x);
    if (dsel != D_NONE) v += dsign * diagv(D, dsel, i) * xv;
    if (mpart) v += sm[i / D.n - k0];
    w[C.off + i] = v;
    sw[i - i0] = v;
  }
  __syncthreads();
  chunk_dots(V, T, C.off, nvec, sw, i0, i1, out);
}

// h_q = sum over blocks of the partials in[.. + q] for q = 0..nq-1 (fixed
// order), into LDS; wavefront v takes q = v, v + 4, ...
__device__ __forceinline__ void sum_partials(const double* __restrict__ in, int c, int nblk, int ldp, int nq,
                                             double* h) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int q = wv; q < nq; q += nw) {
    double acc = 0.0;
    for (int b = lane; b < nblk; b += 64) acc += in[((size_t)c * nblk + b) * ldp + q];
    acc = wave_sum(acc);
    if (lane == 0) h[q] = acc;
  }
  __syncthreads();
}

// First pass: h1 = V^T w from the epilogue's partials, H(:, l) = h1 (block 0),
// w -= V h1 on the chunk, then the chunk's dots of the updated w with
// V_0..V_l (entries 0..l) and its squared norm (entry l + 1).
__global__ __launch_bounds__(kT) void k_gs_update(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                                                  double* __restrict__ V, int64_t T, int per_blk,
                                                  const double* __restrict__ pin, double* __restrict__ pout,
                                                  int ldp, GmresState st) {
  __shared__ double h[kMaxRestart + 1];
  __shared__ double sw[kMaxChunk];
  __shared__ double sh[kT / 64];
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  if (!st.active[c]) return;
  const int col = *st.step;
  const int nvec = col + 1;
  double* __restrict__ w = V + (size_t)nvec * T;
  const ColDev C = cols[c];
  const int N = doms[C.d].N;
  sum_partials(pin, c, nblk, ldp, nvec, h);
  if (blk == 0) {
    double* Hr = st.H + (size_t)c * st.hstride + (size_t)col * st.ldh;
    for (int l = threadIdx.x; l < nvec; l += blockDim.x) Hr[l] = h[l];
  }
  double* out = pout + ((size_t)c * nblk + blk) * ldp;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  if (i0 >= N) {
    for (int l = threadIdx.x; l <= nvec; l += blockDim.x) out[l] = 0.0;
    return;
  }
  double* wr = w + C.off;
  double nrm = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    double v = wr[i];
    for (int l = 0; l < nvec; ++l) v = __builtin_fma(-h[l], V[(size_t)l * T + C.off + i], v);
    wr[i] = v;
    sw[i - i0] = v;
    nrm = __builtin_fma(v, v, nrm);
  }
  __syncthreads();
  chunk_dots(V, T, C.off, nvec, sw, i0, i1, out);
  const double t = block_sum(nrm, sh);
  if (threadIdx.x == 0) out[nvec] = t;
}

// partial norms^2 of the columns of x (grid (nblk, ncol)); entry (c*nblk + blk)*ldp
__global__ __launch_bounds__(kT) void k_norm_partial(const DomDev* __restrict__ doms,
                                                     const ColDev* __restrict__ cols, const double* __restrict__ x,
                                                     int per_blk, double* __restrict__ partial, int ldp) {
  __shared__ double sh[kT / 64];
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const ColDev C = cols[c];
  const int N = doms[C.d].N;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) acc = __builtin_fma(x[C.off + i], x[C.off + i], acc);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((size_t)c * nblk + blk) * ldp] = s;
}

// r = b - Ax (in place into ax) and partial ||r||^2
__global__ __launch_bounds__(kT) void k_residual(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                                                 const double* __restrict__ b, double* __restrict__ ax, int per_blk,
                                                 double* __restrict__ partial, int ldp) {
  __shared__ double sh[kT / 64];
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x;
  const ColDev C = cols[c];
  const int N = doms[C.d].N;
  const int i0 = blk * per_blk, i1 = min(N, i0 + per_blk);
  double acc = 0.0;
  for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const size_t idx = (size_t)C.off + i;
    const double v = b[idx] - ax[idx];
    ax[idx] = v;
    acc = __builtin_fma(v, v, acc);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[((size_t)c * nblk + blk) * ldp] = s;
}

// Sum of column c's nblk block partials, one 64-lane block per column (the
// lanes' loads are in flight together; the order is fixed).
__device__ __forceinline__ double column_partials(const double* partial, int nblk, int ldp, int c) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += partial[((size_t)c * nblk + b) * ldp];
  return wave_sum(s);
}

// ||b|| of column c = blockIdx.x from the partials (64 threads per block)
__global__ __launch_bounds__(64) void k_bnorm(const double* partial, int nblk, int ldp, GmresState st) {
  const int c = blockIdx.x;
  const double s = column_partials(partial, nblk, ldp, c);
  if (threadIdx.x == 0) st.bnorm[c] = sqrt(s);
}

// Start of a restart cycle, one 64-lane block per column: beta0 = ||r|| from
// the partials, true relative residual, convergence test, g = beta0 e_1. The
// number of iterating columns is accumulated in *st.live (zeroed before).
__global__ __launch_bounds__(64) void k_cycle_start(const double* partial, int nblk, int ldp, double tol,
                                                    GmresState st) {
  const int c = blockIdx.x;
  const double s = column_partials(partial, nblk, ldp, c);
  if (threadIdx.x != 0) return;
  const double beta = sqrt(s);
  const double bn = st.bnorm[c];
  const double rel = bn > 0.0 ? beta / bn : 0.0;
  st.true_relres[c] = rel;
  st.relres[c] = rel;
  st.kdim[c] = 0;
  double* g = st.g + (size_t)c * (kMaxRestart + 1);
  if (bn == 0.0 || rel <= tol || beta == 0.0) {
    st.converged[c] = 1;
    st.active[c] = 0;
    st.invbeta[c] = 0.0;
    g[0] = 0.0;
  } else {
    st.converged[c] = 0;
    st.active[c] = 1;
    st.invbeta[c] = 1.0 / beta;
    g[0] = beta;
    atomicAdd(st.live, 1);
  }
}

// start of a cycle: no iterating column counted yet, Arnoldi step 0
__global__ void k_cycle_reset(GmresState st) {
  *st.live = 0;
  *st.step = 0;
  *st.done = 0;
}

// Close Hessenberg column `col` of GMRES column c (all threads of one block):
// H(0..col, col) += h2 (the first pass stored h1), H(col+1, col) = beta, the
// column's earlier Givens rotations and a new one applied, the residual
// estimate |g_{col+1}| / ||b||, and the cycle's stop test.
__device__ void arnoldi_close(GmresState st, int c, int col, const double* h2, double beta, int restart,
                              double tol, double* hc, double* cs_, double* sn_) {
  double* Hc = st.H + (size_t)c * st.hstride + (size_t)col * st.ldh;
  double* cs = st.cs + (size_t)c * kMaxRestart;
  double* sn = st.sn + (size_t)c * kMaxRestart;
  for (int k = threadIdx.x; k <= col; k += blockDim.x) {
    hc[k] = Hc[k] + h2[k];
    if (k < col) {
      cs_[k] = cs[k];
      sn_[k] = sn[k];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    hc[col + 1] = beta;
    for (int k = 0; k < col; ++k) {
      const double t = cs_[k] * hc[k] + sn_[k] * hc[k + 1];
      hc[k + 1] = -sn_[k] * hc[k] + cs_[k] * hc[k + 1];
      hc[k] = t;
    }
    const double a = hc[col];
    const double den = hypot(a, beta);
    double cv = 1.0, sv = 0.0;
    if (den > 0.0) { cv = a / den; sv = beta / den; }
    cs[col] = cv;
    sn[col] = sv;
    hc[col] = den;
    hc[col + 1] = 0.0;
    double* g = st.g + (size_t)c * (kMaxRestart + 1);
    const double gc = g[col];
    g[col + 1] = -sv * gc;
    g[col] = cv * gc;
    const double est = fabs(sv * gc) / st.bnorm[c];
    st.relres[c] = est;
    st.kdim[c] = col + 1;
    st.inner_it[c] += 1;
    const bool stop = (est <= tol) || (beta == 0.0) || (col + 1 >= restart) || (den == 0.0);
    if (stop) {
      st.active[c] = 0;
      atomicSub(st.live, 1);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= col + 1; k += blockDim.x) Hc[k] = hc[k];
}

// Second pass and end of the step. Every block: h2 = V^T w and |w|^2 from
// the first pass's partials, w -= V h2 on its chunk; as h2 is orthogonal to
// the updated w, |w|^2 - |h2|^2 is its squared norm beta^2 (the first pass has
// already removed all but rounding-size components along V, so no
// cancellation occurs short of a breakdown); V_{l+1} = w / beta, its pair
// records and component sums. Block 0 of each column then closes Hessenberg
// column l. Those blocks count themselves in *st.done (after a device-scope
// fence); the last publishes the number of iterating columns to host_live[l]
// and, when given, the residual estimates to host_rel[l*ncol ..] (host-mapped
// memory the host reads after an event) and sets *step_next = l + 1. The
// step index is double-buffered (st.step is read by all of this step's
// launches, step_next by the next step's), so no block can read an index
// that another has already advanced. A block of a column that block 0 has
// just stopped may still write V_{l+1} and its records: no later step or the
// solution update reads them.
__global__ __launch_bounds__(kT) void k_gs_finish(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                                                  double* __restrict__ V, int64_t T, int per_blk,
                                                  const double* __restrict__ pin, int ldp, GmresState st,
                                                  int* __restrict__ step_next, int restart, double tol,
                                                  int* host_live, double* host_rel, int csel,
                                                  double* __restrict__ mpart, int S) {
  __shared__ double h[kMaxRestart + 2];
  __shared__ double sq[kMaxChunk];
  __shared__ double hc[kMaxRestart + 2];
  __shared__ double cs_[kMaxRestart], sn_[kMaxRestart];
  __shared__ int last;
  const int c = blockIdx.y, blk = blockIdx.x, nblk = gridDim.x, ncol = gridDim.y;
  const bool act = st.active[c] != 0;
  if (!act && blk != 0) return;
  const int col = *st.step;
  const int nvec = col + 1;
  double beta = 0.0;
  if (act) {
    sum_partials(pin, c, nblk, ldp, nvec + 1, h);
    double hh = 0.0;
    for (int l = 0; l < nvec; ++l) hh = __builtin_fma(h[l], h[l], hh);
    const double b2 = h[nvec] - hh;
    beta = b2 > 0.0 ? sqrt(b2) : 0.0;
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    const ColDev C = cols[c];
    const DomDev& D = doms[C.d];
    const int i0 = blk * per_blk, i1 = min(D.N, i0 + per_blk);
    if (i0 < D.N) {
      double* wr = V + (size_t)nvec * T + C.off;
      for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
        double v = wr[i];
        for (int l = 0; l < nvec; ++l) v = __builtin_fma(-h[l], V[(size_t)l * T + C.off + i], v);
        const double q = v * inv;
        wr[i] = q;
        sq[i - i0] = q;
        stage_weight(D, csel, C.r, i, q, false);
      }
      if (mpart) {
        __syncthreads();
        chunk_component_sums(sq, i0, i1, D.n, mpart + ((size_t)c * nblk + blk) * S);
      }
    }
  }
  if (blk != 0) return;
  if (act) arnoldi_close(st, c, col, h, beta, restart, tol, hc, cs_, sn_);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(st.done, 1) == ncol - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (host_rel)
    for (int q = threadIdx.x; q < ncol; q += blockDim.x) host_rel[(size_t)col * ncol + q] = st.relres[q];
  if (threadIdx.x == 0) {
    host_live[col] = atomicAdd(st.live, 0);
    *st.done = 0;
    *step_next = col + 1;
  }
}

// Back substitution H y = g (upper triangular kdim x kdim after the Givens
// rotations); one 64-lane block per column, each row sum split over lanes.
__global__ __launch_bounds__(64) void k_backsolve(GmresState st) {
  __shared__ double ys[kMaxRestart];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int k = st.converged[c] ? 0 : st.kdim[c];
  const double* Hr = st.H + (size_t)c * st.hstride;
  const double* g = st.g + (size_t)c * (kMaxRestart + 1);
  for (int l = k - 1; l >= 0; --l) {
    double s = 0.0;
    for (int q = l + 1 + lane; q < k; q += 64) s = __builtin_fma(Hr[(size_t)q * st.ldh + l], ys[q], s);
    s = wave_sum(s);
    if (lane == 0) {
      const double d = Hr[(size_t)l * st.ldh + l];
      ys[l] = d != 0.0 ? (g[l] - s) / d : 0.0;
    }
    __syncthreads();
  }
  double* y = st.y + (size_t)c * kMaxRestart;
  for (int l = lane; l < kMaxRestart; l += 64) y[l] = l < k ? ys[l] : 0.0;
}

// x_c += sum_{l < kdim_c} y_l V_l,c   (grid (blocks over max N, ncol))
__global__ void k_xupdate(const DomDev* __restrict__ doms, const ColDev* __restrict__ cols,
                          const double* __restrict__ V, int64_t T, double* __restrict__ x, GmresState st) {
  const int c = blockIdx.y;
  const ColDev C = cols[c];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= doms[C.d].N) return;
  const int k = st.converged[c] ? 0 : st.kdim[c];
  if (k == 0) return;
  const double* y = st.y + (size_t)c * kMaxRestart;
  double v = x[C.off + i];
  for (int l = 0; l < k; ++l) v = __builtin_fma(y[l], V[(size_t)l * T + C.off + i], v);
  x[C.off + i] = v;
}

// copy of the GMRES state into host-mapped memory (read by the host after a
// stream synchronisation) at a cycle start (and the end of a solve):
// dst[0] = iterating columns, dst[1 + c] =
// converged flags, dst[1 + ncol + c] = inner iterations, rel[c] = true
// relative residual, rel[ncol + c] = residual estimate
__global__ void k_publish_cycle(GmresState st, int ncol, int* __restrict__ dst, double* __restrict__ rel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) dst[0] = *st.live;
  if (i < ncol) {
    dst[1 + i] = st.converged[i];
    dst[1 + ncol + i] = st.inner_it[i];
    rel[i] = st.true_relres[i];
    rel[ncol + i] = st.relres[i];
  }
}

// inner_it counters etc. to zero
__global__ void k_gmres_init(int ncol, GmresState st) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  st.inner_it[c] = 0;
  st.relres[c] = 1.0;
  st.true_relres[c] = 1.0;
  st.converged[c] = 0;
  st.active[c] = 0;
  st.kdim[c] = 0;
}

}  // namespace gnk
